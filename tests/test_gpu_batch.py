"""Batched and served simulations give the same results as the same simulations run alone, and
the FP32 batched and served forms match the FP64 oracle.

FP64 batch: element by element within 1e-12 of the same simulations stepped alone (and of the
oracle).  FP32 batch and serving mix: end-of-run field energy, kinetic energies and the spectrum
of the total-current series within 1e-3 relative of the run alone and of the FP64 oracle's run of
the same request (its own loader; the FP32 form starts from the same draws rounded to FP32),
including one served request of the stream at its full grid scale and full step count (against
the FP64 form, itself checked against the oracle on that request).  Joining
and leaving a batch rewrite table entries only: the step graph is captured once.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if np.size(a) else 0.0


def _uneven(n_req=3, steps=40):
    """Small uneven 2D requests: different grids, geometries, ppc."""
    from paper_2501_07465_amd import workloads as W
    out = []
    for j in range(n_req):
        w = W.stream_request(j, scale=0.1)
        w["steps"] = steps
        w["tile"] = [16, 8, 1]
        out.append(w)
    return out


def _spectrum(series):
    s = np.asarray(series)
    win = np.hanning(s.shape[0])[:, None]
    return np.abs(np.fft.rfft(s * win, axis=0))


def _compare_results(a, b, tol, label):
    ef = abs(a["field_energy"] - b["field_energy"]) / max(abs(b["field_energy"]), 1e-300)
    ek = max(abs(x - y) / max(abs(y), 1e-300) for x, y in zip(a["kinetic_energy"], b["kinetic_energy"]))
    sa, sb = _spectrum(a["current_series"]), _spectrum(b["current_series"])
    es = _rel(sa, sb)
    print(f"{label}: field energy {ef:.2e}, kinetic {ek:.2e}, current spectrum {es:.2e}", flush=True)
    assert a["steps"] == b["steps"]
    assert ef <= tol and ek <= tol and es <= tol, (label, ef, ek, es)


def _oracle_result(oracle, w):
    ref = oracle.build_workload(w)
    ref.step(int(w["steps"]))
    return {"field_energy": ref.field_energy(),
            "kinetic_energy": [ref.kinetic_energy(s) for s in range(len(w["species"]))],
            "current_series": ref.current_series(), "steps": int(w["steps"])}


def test_batch_fp64_matches_alone_and_oracle(oracle):
    from paper_2501_07465_amd import pic
    ws = _uneven(3, 40)
    print("case batch fp64: " + ", ".join(f"{w['n'][0]}^2 {w['geometry']}" for w in ws), flush=True)
    alone = []
    for w in ws:
        s = pic.Simulation(w, precision="fp64", graphs=False)
        s.step(40)
        alone.append(s)
    batch = pic.Batch(4, 2, "fp64")
    mixed = [pic.Simulation(w, precision="fp64", graphs=False, stream=batch.stream) for w in ws]
    for s in mixed:
        batch.add(s)
    batch.step(20)
    batch.step(20)
    for s in list(mixed):
        batch.remove(s)
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m.steps_done == 40
        for sid in range(len(ws[i]["species"])):
            xa, va, _ = a.particles(sid)
            xm, vm, _ = m.particles(sid)
            assert _rel(xm, xa) < 1e-12 and _rel(vm, va) < 1e-12, (i, sid)
        ea, ba = a.fields()
        em, bm = m.fields()
        assert _rel(em, ea) < 1e-12 and _rel(bm, ba, np.max(np.abs(ea)) / 3e8 + np.max(np.abs(ba))) < 1e-12, i
    # one member against the oracle from the same initial state
    ref = oracle.build_workload(ws[0])
    s = pic.Simulation(ws[0], precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False,
                       stream=batch.stream)
    batch.add(s)
    batch.step(40)
    batch.remove(s)
    ref.step(40)
    eg, _ = s.fields()
    er, _ = ref.fields()
    print(f"batch fp64 vs oracle: E rel {_rel(eg, er):.2e}", flush=True)
    assert _rel(eg, er) < 1e-12


def test_batch_fp32_member_joining_mid_run(oracle):
    from paper_2501_07465_amd import pic, serve
    ws = _uneven(3, 80)
    print("case batch fp32 join", flush=True)
    ref = [serve.run_alone(w, "fp32") for w in ws]
    orc = [_oracle_result(oracle, w) for w in ws]
    batch = pic.Batch(4, 2, "fp32")
    sims = [pic.Simulation(w, precision="fp32", graphs=False, stream=batch.stream, block=512,
                           series_cap=w["steps"] + 64) for w in ws]
    batch.add(sims[0])
    batch.add(sims[1])
    batch.step(40)
    batch.add(sims[2])  # joins while the others are mid-run
    batch.step(40)
    batch.remove(sims[0])
    batch.remove(sims[1])
    batch.step(40)
    batch.remove(sims[2])
    for i, s in enumerate(sims):
        res = {"field_energy": s.field_energy(), "kinetic_energy": [s.kinetic_energy(k) for k in s.species],
               "current_series": s.current_series(), "steps": s.steps_done}
        _compare_results(res, ref[i], 1e-3, f"batch fp32 member {i}")
        _compare_results(res, orc[i], 1e-3, f"batch fp32 member {i} vs fp64 oracle")
    # membership changes the captured step graph covers (same tile and block) never capture it again
    assert batch.captures == 1


def test_batch_slots_reused_without_recapture():
    """Members leave and others take their slots between periods: one capture, and every member's
    result is bit-identical to its run alone (the current is accumulated exactly)."""
    from paper_2501_07465_amd import pic
    ws = _uneven(4, 60)
    print("case batch slot reuse", flush=True)
    alone = []
    for w in ws:
        a = pic.Simulation(w, precision="fp32", graphs=False, block=512)
        a.step(60)
        alone.append(a)
    batch = pic.Batch(2, 2, "fp32")
    sims = [pic.Simulation(w, precision="fp32", graphs=False, stream=batch.stream, block=512) for w in ws]
    batch.add(sims[0])
    batch.add(sims[1])
    batch.step(20)
    batch.remove(sims[0])
    batch.add(sims[2])        # takes slot 0 while sims[1] is mid-run
    batch.step(40)
    batch.remove(sims[1])     # sims[1] is done
    batch.add(sims[3])
    batch.step(20)
    batch.remove(sims[2])     # sims[2] is done
    batch.step(40)
    batch.remove(sims[3])
    batch.add(sims[0])        # back in, 40 steps to go
    batch.step(40)
    batch.remove(sims[0])
    assert batch.captures == 1 and len(batch) == 0
    for i, (a, s) in enumerate(zip(alone, sims)):
        assert s.steps_done == 60, (i, s.steps_done)
        ea, ba = a.fields()
        es, bs = s.fields()
        assert np.array_equal(ea, es) and np.array_equal(ba, bs), i
        assert np.array_equal(a.current_series(), s.current_series()), i


def test_serving_results_same_alone_and_in_mix(oracle):
    from paper_2501_07465_amd import serve, workloads as W
    reqs = []
    for j in range(5):
        w = W.stream_request(j, scale=0.1)
        w["steps"] = 40 * (1 + j % 3)
        w["tile"] = [16, 8, 1]
        reqs.append(serve.Request(j, w, arrival=0.02 * j))
    print("case serving mix", flush=True)
    ref = [serve.run_alone(r.w, "fp32") for r in reqs]
    orc = [_oracle_result(oracle, r.w) for r in reqs]
    # a budget that holds about three of them at once: later arrivals wait for memory
    fps = []
    for r in reqs:
        from paper_2501_07465_amd import pic
        fps.append(pic.footprint_of(r.w, "fp32", 512, series_cap=r.steps + 64))
    srv = serve.Server(dims=2, precision="fp32", hbm_budget=int(sum(sorted(fps)[-3:])), max_slots=4)
    stats = srv.run(reqs)
    print(f"serving: {stats}", flush=True)
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    assert stats["p99_s"] >= stats["p50_s"] > 0
    assert stats["graph_captures"] <= 1
    for r, a, o in zip(reqs, ref, orc):
        _compare_results(r.result, a, 1e-3, f"request {r.rid}")
        _compare_results(r.result, o, 1e-3, f"request {r.rid} vs fp64 oracle")


def test_fullscale_stream_request_served_fp32_matches_fp64(oracle):
    """Request 51 of the stream at its full grid scale (208^2 cells, a slab, 1420 steps) served
    beside two small requests.  Its whole FP32 run against the whole FP64 run of the same request
    (end-of-run metrics within 1e-3), and that FP64 form against the oracle over the first 100 steps
    of the same request at full scale (element by element within 1e-12; the oracle's whole run
    takes minutes on one core)."""
    from paper_2501_07465_amd import pic, serve, workloads as W
    big = W.stream_request(51, scale=1.0)
    assert big["n"][0] == 208 and big["steps"] == 1420
    big["tile"] = [16, 8, 1]
    reqs = [serve.Request(0, big, arrival=0.0)]
    for j in range(2):
        w = W.stream_request(j, scale=0.1)
        w["steps"] = 200
        w["tile"] = [16, 8, 1]
        reqs.append(serve.Request(1 + j, w, arrival=0.01 * (j + 1)))
    print("case full-scale stream request 51", flush=True)
    srv = serve.Server(dims=2, precision="fp32", hbm_budget=8 << 30, max_slots=4)
    stats = srv.run(reqs)
    assert stats["requests"] == 3
    r64 = serve.run_alone(big, "fp64")
    _compare_results(reqs[0].result, r64, 1e-3, "request 51 (full scale) fp32 served vs fp64")
    ref = oracle.build_workload(big)
    sim = pic.Simulation(big, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False)
    sim.step(100)
    ref.step(100)
    eg, bg = sim.fields()
    er, br = ref.fields()
    print(f"request 51 fp64 vs oracle, 100 steps: E {_rel(eg, er):.2e}, B {_rel(bg, br):.2e}", flush=True)
    assert _rel(eg, er) < 1e-12 and _rel(bg, br) < 1e-12
    assert _rel(sim.current_series(), ref.current_series()) < 1e-12


def test_batch_members_of_one_shape_with_different_periodic_axes():
    """Two members with the 32 x 32 tile, one periodic along y (the shape's kernel is compiled for
    that axis) and one open on both axes: the step graph is captured again when the second joins,
    with the kernel that reads the periodicity from the table.  The open member runs that kernel
    alone too and equals its run alone bit for bit; the periodic one is held to 1e-5 of its fields'
    scale (FP32 contractions of the two kernels may round differently)."""
    from paper_2501_07465_amd import pic
    ws = _uneven(2, 40)
    for w in ws:
        w["tile"] = [32, 32, 1]
    ws[1]["periodic"] = [0, 0, 1]
    print("case batch periodic masks", flush=True)
    alone = []
    for w in ws:
        a = pic.Simulation(w, precision="fp32", graphs=False, block=512)
        a.step(40)
        alone.append(a)
    batch = pic.Batch(2, 2, "fp32")
    sims = [pic.Simulation(w, precision="fp32", graphs=False, stream=batch.stream, block=512) for w in ws]
    batch.add(sims[0])
    batch.step(20)
    batch.add(sims[1])
    batch.step(20)
    batch.remove(sims[0])
    batch.step(20)
    batch.remove(sims[1])
    assert batch.captures == 2
    for i, (a, s) in enumerate(zip(alone, sims)):
        assert s.steps_done == 40
        ea, ba = a.fields()
        es, bs = s.fields()
        if i == 1:
            assert np.array_equal(ea, es) and np.array_equal(ba, bs), i
        else:
            print(f"periodic-y member: E rel {_rel(es, ea):.2e}", flush=True)
            assert _rel(es, ea) < 1e-5 and _rel(bs, ba) < 1e-5, i


def test_batch_mixed_tile_shapes():
    """A member whose tile has constant window geometry (32 x 32) beside one with a 16 x 8 tile: the
    step graph takes the kernel that reads each member's geometry, and is captured again when the
    second shape joins.  The 16 x 8 member equals its run alone bit for bit; the 32 x 32 member ran
    alone on the fixed-geometry kernel and here partly on the general one, whose FP32 contractions
    may round differently, so it is held to 1e-5 of its fields' scale."""
    from paper_2501_07465_amd import pic
    ws = _uneven(2, 40)
    ws[0]["tile"] = [32, 32, 1]
    ws[1]["tile"] = [16, 8, 1]
    print("case batch mixed tiles", flush=True)
    alone = []
    for w in ws:
        a = pic.Simulation(w, precision="fp32", graphs=False, block=512)
        a.step(40)
        alone.append(a)
    batch = pic.Batch(2, 2, "fp32")
    sims = [pic.Simulation(w, precision="fp32", graphs=False, stream=batch.stream, block=512) for w in ws]
    batch.add(sims[0])
    batch.step(20)              # the fixed-geometry kernel
    batch.add(sims[1])          # another tile shape: captured again with the general kernel
    batch.step(20)
    batch.remove(sims[0])
    batch.step(20)
    batch.remove(sims[1])
    assert batch.captures == 2
    for i, (a, s) in enumerate(zip(alone, sims)):
        assert s.steps_done == 40
        ea, ba = a.fields()
        es, bs = s.fields()
        if i == 1:
            assert np.array_equal(ea, es) and np.array_equal(ba, bs), i
            for sid in range(len(ws[i]["species"])):
                xa, va, _ = a.particles(sid)
                xs, vs, _ = s.particles(sid)
                assert np.array_equal(xa, xs) and np.array_equal(va, vs), (i, sid)
        else:
            print(f"fixed-geometry member: E rel {_rel(es, ea):.2e}", flush=True)
            assert _rel(es, ea) < 1e-5 and _rel(bs, ba) < 1e-5, i
