"""Diffusive (cosine-law) walls on the device, through the C ABI, against the oracle.

The draw of a reflected particle comes from Philox4x32-10 with counter (particle index, step,
species id, 2^31) under the species seed on both sides, so the runs are comparable element by
element: FP64 within 1e-12 of the oracle's scale (ball in 2D and 3D, box in 2D, the box and ball
with both in-plane axes open), FP32 one step from identical inputs within 1e-6.  A long FP32 run
keeps every free electron inside its region.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if a.size else 0.0


def _walls(name, fp64=True, box=False):
    from paper_2501_07465_amd import workloads as W
    w = W.small(name)
    if name == "sphere3d" and fp64:
        w["tile"] = [4, 4, 4]
    if box:
        rod = {"kind": "box", "lo": [20.5, 27.25, 0.0], "hi": [52.75, 40.5, 1.0]}
        for sp in w["species"]:
            sp["region"] = dict(rod)
    return W.with_diffuse_walls(w)


def _compare(sim, ref, w, tol, label):
    for sid in range(len(w["species"])):
        xg, vg, _ = sim.particles(sid)
        xr, vr, _ = ref.particles(sid)
        ex = float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) if len(xg) else 0.0
        ev = _rel(vg, vr)
        print(f"{label} species {sid}: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
        assert ex < tol and ev < tol, (label, sid, ex, ev)
    eg, bg = sim.fields()
    er, br = ref.fields()
    ee = _rel(eg, er)
    print(f"{label} fields: E rel {ee:.2e}", flush=True)
    assert ee < tol, (label, ee)


def _toward_walls(w, state, frac=0.012, seed=5):
    """The oracle state with every free electron within a cell of its wall sent outward at frac
    cells per step (plus a random tangential part), so that many reach the wall during the run."""
    rng = np.random.default_rng(seed)
    dims = w["dims"]
    dx = np.array(w["dx"])
    out = []
    for sid, (x, v, xi, wt) in enumerate(state):
        sp = w["species"][sid]
        v = v.copy()
        if sp["kind"] == "free" and sp.get("reflect"):
            reg = sp["region"]
            X = x / dx
            nrm = np.zeros_like(v)
            if reg["kind"] == "ball":
                d = X[:, :dims] - np.array(reg["center"][:dims])
                r = np.linalg.norm(d, axis=1)
                near = r > reg["radius"] - 1.0
                nrm[:, :dims] = d / r[:, None]
            else:
                lo, hi = np.array(reg["lo"][:dims]), np.array(reg["hi"][:dims])
                gap = np.concatenate([X[:, :dims] - lo, hi - X[:, :dims]], axis=1)
                k = np.argmin(gap, axis=1)
                near = gap[np.arange(len(k)), k] < 1.0
                ax = k % dims
                nrm[np.arange(len(k)), ax] = np.where(k < dims, -1.0, 1.0)
            t = rng.normal(size=v.shape)
            t -= np.sum(t * nrm, axis=1, keepdims=True) * nrm
            d = nrm + 0.5 * t / np.maximum(np.linalg.norm(t, axis=1, keepdims=True), 1e-30)
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            v[near] = d[near] * (frac * dx[0] / w["dt"])
        out.append((x, v, xi, wt))
    return out


def _oracle_from(oracle, w, state, fields):
    ref = oracle.Sim(w)
    for sid, (x, v, xi, wt) in enumerate(state):
        ref.add_species(w["species"][sid], wt, x, v, xi)
    ref.set_fields(*fields)
    return ref


@pytest.mark.parametrize("name,box,steps,periodic", [("disk2d", False, 120, None), ("disk2d", True, 120, None),
                                                     ("disk2d", True, 80, [0, 0, 1]), ("sphere3d", False, 40, None)])
def test_fp64_diffuse_walls_match_oracle(oracle, name, box, steps, periodic):
    from paper_2501_07465_amd import pic
    w = _walls(name, box=box)
    if periodic is not None:
        w["periodic"] = list(periodic)
        w["source"]["index"] = [6, 0, 0]
    print(f"case fp64 diffuse walls {name} box={box} periodic={periodic} {steps} steps", flush=True)
    base = oracle.build_workload(w)
    st, fl = _toward_walls(w, base.state()), base.fields()
    ref = _oracle_from(oracle, w, st, fl)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=fl, graphs=False)
    sim.step(steps)
    ref.step(steps)
    _compare(sim, ref, w, 1e-12, f"fp64 diffuse {name}")
    # the walls were hit: the same run with specular walls ends elsewhere
    ws = {**w, "species": [dict(sp, scatter="specular") for sp in w["species"]]}
    spec = _oracle_from(oracle, ws, st, fl)
    spec.step(steps)
    dv = _rel(ref.particles(0)[1], spec.particles(0)[1])
    print(f"diffuse vs specular oracle runs: v rel {dv:.2e}", flush=True)
    assert dv > 1e-3


def test_fp32_diffuse_walls_one_step(oracle):
    """FP32 form, one step from identical inputs with free electrons placed to cross the wall."""
    from paper_2501_07465_amd import pic
    w = _walls("disk2d", fp64=False)
    print("case fp32 diffuse walls one step", flush=True)
    base = oracle.build_workload(w)
    base.step(3)
    st = base.state()
    dx = np.array(w["dx"])
    x, v, xi, wt = st[0]
    # push every free electron at the wall outward with a speed that crosses it within the step
    c = np.array(w["species"][0]["region"]["center"])
    r = np.hypot(x[:, 0] / dx[0] - c[0], x[:, 1] / dx[1] - c[1])
    near = r > w["species"][0]["region"]["radius"] - 0.45
    out = np.zeros_like(v)
    out[:, 0] = (x[:, 0] / dx[0] - c[0]) / r
    out[:, 1] = (x[:, 1] / dx[1] - c[1]) / r
    v = v.copy()
    v[near] = out[near] * (0.5 * dx[0] / w["dt"])
    st32 = []
    for sid, (xs, vs, xis, ws) in enumerate([(x, v, xi, wt)] + list(st[1:])):
        X = xs / dx
        cc = np.floor(X)
        x32 = (cc + (X - cc).astype(np.float32).astype(np.float64)) * dx
        st32.append((x32, vs.astype(np.float32).astype(np.float64),
                     None if xis is None else xis.astype(np.float32).astype(np.float64), ws))
    e, b = base.fields()
    e32, b32 = e.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    ref = oracle.Sim(w)
    for sid, (xs, vs, xis, ws) in enumerate(st32):
        ref.add_species(w["species"][sid], ws, xs, vs, xis)
    ref.set_fields(e32, b32)
    sim = pic.Simulation(w, precision="fp32", states=st32, fields=(e32, b32), graphs=False)
    sim.step(1)
    ref.step(1)
    xg, vg, _ = sim.particles(0)
    xr, vr, _ = ref.particles(0)
    vscale = np.max(np.linalg.norm(vr, axis=1))
    ev = float(np.max(np.abs(vg - vr)) / vscale)
    ex = float(np.max(np.abs(xg - xr) / dx))
    print(f"fp32 diffuse: {int(near.sum())} crossing, v err {ev:.2e}, x err {ex:.2e} cells", flush=True)
    assert near.sum() > 10
    assert ev <= 1e-6 and ex <= 1e-6, (ev, ex)


def test_fp32_diffuse_walls_confine_over_a_long_run():
    from paper_2501_07465_amd import pic
    w = _walls("disk2d", fp64=False)
    print("case fp32 diffuse walls 600 steps", flush=True)
    sim = pic.Simulation(w, precision="fp32", graphs=True)
    sim.step(600)
    x, v, _ = sim.particles(0)
    reg = w["species"][0]["region"]
    r = np.hypot(x[:, 0] / w["dx"][0] - reg["center"][0], x[:, 1] / w["dx"][1] - reg["center"][1])
    assert np.all(r <= reg["radius"] + 1e-4)
    assert np.all(np.isfinite(v))


def test_diffuse_walls_refused_for_bound_species():
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    h = pic.pic_create(pic.grid_desc(w))
    sp = dict(w["species"][1], reflect=True, scatter="diffuse")
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_species(h, pic.species_desc(sp), 1)
    assert e.value.code == pic.PIC_EINVAL
    pic.pic_destroy(h)


def test_batch_mixes_diffuse_and_specular_members(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    wa = _walls("disk2d")
    wb = W.small("disk2d")
    print("case batch diffuse + specular", flush=True)
    base = oracle.build_workload(wa)
    sta, fla = _toward_walls(wa, base.state()), base.fields()
    refa = _oracle_from(oracle, wa, sta, fla)
    refb = oracle.build_workload(wb)
    batch = pic.Batch(2, 2, "fp64")
    sa = pic.Simulation(wa, precision="fp64", states=sta, fields=fla, graphs=False, stream=batch.stream)
    sb = pic.Simulation(wb, precision="fp64", states=refb.state(), fields=refb.fields(), graphs=False,
                        stream=batch.stream)
    batch.add(sa)
    batch.add(sb)
    batch.step(60)
    refa.step(60)
    refb.step(60)
    batch.remove(sa)
    batch.remove(sb)
    _compare(sa, refa, wa, 1e-12, "batch diffuse")
    _compare(sb, refb, wb, 1e-12, "batch specular")
