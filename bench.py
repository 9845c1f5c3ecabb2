"""Benchmark of the PIC step on one MI355X: particle-steps/s (sort + gather + push + deposit + fields).

Default workload (the headline): the 3D3V nanosphere, 256^3 cells of 1 nm with a metal sphere of
radius 100 cells holding 8 ppc Fermi-Dirac free electrons + 8 ppc bound Lorentz electrons
(65.5M particles), dipole pulse, cell sort every 20 steps, FP32 form (int32 cell + FP32 offset),
synthetic seeded inputs.  The warm-up is rounded up to a whole number of 20-step sort periods, so
the K timed steps start on a period boundary and replay captured graphs (one per period; a
remainder of K runs as plain launches, reported in ``config``), bracketed by device
synchronisation.

Beside it: the FP64 GPU rate of the same workload and the FP32/FP64 speedup; a roofline for the
dominant kernel (the particle kernel) and for the whole step; a secondary leg on the 2D3V disk
(1024^2 cells, 16 + 16 ppc) with its own roofline; a serving run (continuous batching of seeded
uneven requests with Poisson arrivals, p50/p99 latency); the plain-C FP64 oracle timed on the
host's cores (cpu_baseline: concurrent single-threaded copies, each on a 64^3 twin of the sphere
with the same ppc and physics).

A dielectric leg runs the disk with the metal's background permittivity (eps = 3.7 by
default) inside the disk, as a per-cell inverse permittivity (eq:consteps), and reports its rate
and its field kernel against the kernel without one.  A tensor leg does the same with a full
(anisotropic, off-diagonal) permittivity tensor in the disk, whose field step adds two
node-parallel passes (update terms, off-diagonal fold) before the field kernel.  Variant legs time
the other optional physics at full size against the plain workload: diffusive walls and the
work-function barrier on the disk, the per-carrier Dirac mass and diffusive ribbon ends on the sheet.

Algorithmic bytes (the minimum the method moves; no halos or re-reads):
  particle kernel, per launch: per particle its state read and written (FP32: 1D/2D/3D free
  40/48/56 B, 2D/3D bound 60/64 B, Dirac 48 B) + per occupied cell 24 B of E, B gathered and
  12 B of J written;
  whole step: particle kernel bytes + per cell 48 B (E, B read and written by the Yee update) +
  per occupied cell 12 B (J read by the Yee update);
  dielectric field kernel, per launch: per cell 48 B of E, B + 12 B of inverse permittivity, per
  occupied cell 12 B of J;
  full-tensor field step (three kernels): the dielectric kernel reading J at every cell (72 B per
  cell); the update-term pass over its node list (E, B gathered, J read, U written: 48 B per listed
  node); the fold over the nodes with an off-diagonal row (entries, inverse permittivity and the
  averaged U read, J read and written: 72 B per folded node).
achieved = bytes / average duration measured here with HIP events on the simulation's stream;
peak = 8 TB/s HBM3E.  ``traffic`` is the kernel's measured HBM bytes per launch from committed
rocprofv3 FETCH_SIZE/WRITE_SIZE runs (calibrated against a copy of known size) when those runs
were taken on the current kernel sources with the same tile and block, else null.

One GPU only: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit) FP32 vs FP64 GPU; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0


def particle_bytes_per_step(w, counts, es=4):
    """Particle state read and written per step, summed over species."""
    d = w["dims"]
    total = 0
    for sp, n in zip(w["species"], counts):
        if sp["kind"] == "bound":
            per = (4 + d * es + 6 * es) + 6 * es  # anchor cell/offset, xi, v read; xi, v written
        else:
            per = 2 * (4 + d * es + 3 * es)       # cell, offset, v read and written
        total += n * per
    return total


def occupied_cells(w):
    """Cells holding particles at load time (the species' region cells)."""
    import numpy as np
    n = w["n"]
    cells = np.zeros((n[2], n[1], n[0]), dtype=bool)
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for sp in w["species"]:
        reg = sp.get("region", {"kind": "all"})
        if reg["kind"] == "all":
            cells[:] = True
        elif reg["kind"] == "box":
            m = np.ones_like(cells)
            for a, g in enumerate((ii, jj, kk)[:w["dims"]]):
                m &= (g >= reg["lo"][a]) & (g + 1 <= reg["hi"][a])
            cells |= m
        else:
            m = np.ones_like(cells)
            for corner in range(1 << w["dims"]):
                r2 = np.zeros(cells.shape)
                for a, g in enumerate((ii, jj, kk)[:w["dims"]]):
                    r2 = r2 + (g + ((corner >> a) & 1) - reg["center"][a]) ** 2
                m &= r2 <= reg["radius"] ** 2
            cells |= m
    return int(cells.sum())


def describe(w, npart, precision="FP32"):
    n = "x".join(str(v) for v in w["n"][:w["dims"]])
    sp = " + ".join(f"{s.get('ppc', 0)} ppc {s['kind']}" for s in w["species"])
    dx = w["dx"][0] * 1e9
    return f"{w['name']}: {w['dims']}D3V {n} cells of {dx:g} nm, {sp} ({npart} particles), {precision}"


def run_gpu(w, precision, steps, warmup, graphs=True, time_kernels=0, block=256):
    import torch
    from paper_2501_07465_amd import pic
    sim = pic.Simulation(w, precision=precision, graphs=graphs, series_cap=steps + warmup + time_kernels + 64,
                         block=block, unit=w.get("unit", 0))
    counts = [sim.count(s) for s in sim.species]
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = pic.pic_time_kernels(sim.h, time_kernels) if time_kernels else None
    fe = sim.field_energy()
    del sim
    return counts, dt, kt, fe


def run_variants(w, block, kt, npart, value, args, graphs, log):
    """The optional physics at full size, FP32, each against its plain workload: particle-steps/s,
    ms per step and the particle kernel's event time."""
    from paper_2501_07465_amd import autotune, workloads as W
    steps, tk = args.variant_steps, 100

    def leg(wv, label, blk):
        log(f"bench: variant {label}")
        counts, dtv, ktv, _ = run_gpu(wv, "fp32", steps, 20, graphs, tk, blk)
        n = sum(counts)
        return {"value": n * steps / dtv, "unit": "particle-steps/s", "ms_per_step": dtv / steps * 1e3,
                "particle_kernel_ms": float(ktv[0]), "particles": n}

    out = {"steps": steps,
           "disk_plain": {"value": value, "particle_kernel_ms": float(kt[0]), "particles": npart},
           "f3a_diffuse_walls": leg(W.with_diffuse_walls(w), "diffuse walls (disk)", block),
           "f3b_work_function": leg(W.with_potential_wall(w, 9.8, 2.0), "work-function barrier (disk)", block)}
    ws = W.WORKLOADS["sheet2d"]()
    res = autotune.shipped(ws, "fp32")
    bs = 256
    if res is not None:
        ws = autotune.apply(ws, res)
        bs = int(res["block"])
    out["sheet_plain"] = leg(ws, "plain (sheet)", bs)
    wm = copy.deepcopy(ws)
    wm["species"][0]["mass_per_particle"] = True
    out["g11_dirac_mass"] = leg(wm, "per-carrier Dirac mass (sheet)", bs)
    wr = copy.deepcopy(ws)
    reg = wr["species"][0]["region"]
    reg["lo"][0], reg["hi"][0] = 64.0, float(wr["n"][0] - 64)
    wr["species"][0].update(reflect=True, scatter="diffuse")
    out["f3c_ribbon_edges"] = leg(wr, "diffusive ribbon ends (sheet)", bs)
    return out


def committed_traffic(workload, tile, block, unit, kernel="k_particles"):
    """Traffic per launch from the committed counter summary, if it matches the current kernels."""
    from paper_2501_07465_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    t = profiling.read_traffic_file(path)
    if (t.get("source_digest") != profiling.source_digest() or t.get("tile") != "x".join(str(v) for v in tile)
            or t.get("block") != str(block) or t.get("unit") != str(unit)):
        return None
    return float(t["traffic_bytes"])


def copy_ceiling(log):
    """HBM bandwidth a plain streaming copy reaches on this GPU: the library's structure-of-arrays copy
    (8 float arrays of 128 MiB each, read and written: 2 GiB moved per launch, far beyond the caches),
    timed with HIP events over 10 launches."""
    import torch
    from paper_2501_07465_amd import pic
    n = 32 << 20  # floats per array
    src = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(8)]
    dst = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(8)]
    st = torch.cuda.current_stream()
    sp, dp = [x.data_ptr() for x in src], [x.data_ptr() for x in dst]
    pic.pic_measure_soa_copy(sp, dp, n, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(10):
        pic.pic_measure_soa_copy(sp, dp, n, st.cuda_stream)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 10
    assert all(torch.equal(a, b) for a, b in zip(src, dst))
    gbs = 2 * 8 * n * 4 / (ms * 1e-3) / 1e9
    log(f"bench: copy ceiling {gbs:.0f} GB/s")
    del src, dst
    return {"achieved": gbs, "unit": "GB/s", "ms_per_launch": ms,
            "kernel": "pic_measure_soa_copy: 8 float arrays x 128 MiB, read and written"}


def sphere_twin(seed):
    """The 64^3 twin of the nanosphere: radius 25 cells, the same 8 + 8 ppc, species and cell size."""
    from paper_2501_07465_amd import workloads as W
    w = W.sphere3d(n=64, radius=25.0, src_gap=3)
    w["name"] = "sphere3d_twin64"
    w["seed"] = seed
    return w


def _oracle_worker(args):
    """One single-threaded oracle process: load the twin, then step it for budget_s seconds."""
    seed, budget_s = args
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    w = sphere_twin(seed)
    ref = O.build_workload(w)
    n = sum(ref.count(s) for s in range(len(w["species"])))
    t0 = time.perf_counter()
    steps = 0
    while True:
        ref.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return n, steps, el


def cpu_baseline(budget_s, log):
    """The FP64 oracle on the host's cores: one single-threaded copy per core, each on its own seeded
    64^3 twin of the sphere, all stepping concurrently for budget_s seconds (the oracle itself is
    single-threaded, as written); aggregate particle-steps/s over the copies."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    cores = max(1, min(16, ncpu))
    from oracle import oracle as O
    O.build()
    log(f"bench: cpu baseline, {cores} oracle processes on the 64^3 sphere twin")
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(3 + 1000 * k, budget_s) for k in range(cores)])
    wall = time.perf_counter() - t0
    total = sum(n * st for n, st, _ in res)
    rates = [n * st / el for n, st, el in res]
    n0 = res[0][0]
    return {"value": float(sum(rates)), "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "per_core": float(sum(rates) / cores),
            "sample": f"{cores} concurrent single-threaded plain C FP64 oracle processes, each on a seeded "
                      f"64^3 twin of the 256^3 sphere (radius 25 cells, 8 + 8 ppc, {n0} particles), "
                      f"{budget_s:.0f} s of steps each after loading; {total} particle-steps in total, "
                      f"{wall:.0f} s wall with loading"}


def run_serve(n_req, scale, load, block, tile, budget_gib, slots, log, unit=None):
    """Seeded uneven requests, Poisson arrivals at ``load`` x the measured batched capacity."""
    import numpy as np
    from paper_2501_07465_amd import serve, workloads as W
    base = [W.stream_request(j, scale=scale) for j in range(n_req)]
    # capacity: the first requests all at once
    nprobe = min(8, n_req)
    probe = serve.Server(dims=2, precision="fp32", hbm_budget=int(budget_gib * 2**30), max_slots=slots,
                         block=block, tile=tile, unit=unit)
    ps = probe.run([serve.Request(j, copy.deepcopy(base[j]), 0.0) for j in range(nprobe)])
    del probe
    cap = ps["particle_steps_per_s"]
    per_req = ps["particle_steps"] / max(ps["requests"], 1)
    lam = load * cap / per_req
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_req))
    arrivals -= arrivals[0]
    srv = serve.Server(dims=2, precision="fp32", hbm_budget=int(budget_gib * 2**30), max_slots=slots,
                       block=block, tile=tile, unit=unit)
    reqs = [serve.Request(j, copy.deepcopy(base[j]), float(arrivals[j])) for j in range(n_req)]
    log(f"bench: serving {n_req} requests at {lam:.1f}/s (capacity probe {cap:.3e} particle-steps/s)")
    st = srv.run(reqs)
    # the stream's aggregate HBM roofline: every finished request's algorithmic bytes (its particles,
    # E and B at every node, staging and current at its occupied cells) over the serving span
    es = 4
    total_bytes = 0.0
    for r in reqs:
        if r.result is None:
            continue
        ncells = r.w["n"][0] * r.w["n"][1]
        occ = occupied_cells(r.w)
        per_step = particle_bytes_per_step(r.w, r.counts, es) + occ * (6 * es + 3 * 8) + ncells * 12 * es + occ * 3 * 8 * 2
        total_bytes += per_step * r.steps
    agg = total_bytes / st["span_s"] / 1e9
    return {"requests": st["requests"], "rejected": st["rejected"], "p50_s": st["p50_s"], "p99_s": st["p99_s"],
            "mean_s": st["mean_s"], "span_s": st["span_s"], "particle_steps": st["particle_steps"],
            "particle_steps_per_s": st["particle_steps_per_s"], "arrival_rate_hz": lam, "load": load,
            "capacity_probe": cap, "grid_scale": scale, "hbm_budget_gib": budget_gib, "slots": slots,
            "step_graph_captures": st["graph_captures"],
            "roofline": {"bound": "hbm", "achieved": agg, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": agg / HBM_PEAK_GBS,
                         "bytes": total_bytes, "what": "algorithmic bytes of all finished requests over the serving span"},
            "requests_desc": f"{n_req} seeded 2D3V disk/rod/slab requests with Poisson arrivals, grid side "
                             f"U[128,1024] x {scale:g}, 8-32 ppc free + 8-32 ppc bound, 500-4000 steps, FP32; "
                             "latency is arrival to result read back"}


def tuned(name, log, autotune_now=False):
    """Workload dict with its shipped (or freshly measured) tile, block and unit."""
    from paper_2501_07465_amd import autotune, workloads as W
    w = W.WORKLOADS[name]()
    res = None if autotune_now else autotune.shipped(w, "fp32")
    how = "shipped"
    if res is None:
        log(f"bench: autotuning tile and block for {name}")
        res = autotune.tune(w, "fp32", periods=2, use_cache=False, log=log)
        how = "measured"
    return autotune.apply(w, res), int(res["block"]), how


def fp32_leg(w, block, steps, warmup, graphs, time_kernels, label, log):
    """FP32 rate of workload w, its particle-kernel roofline and its whole-step byte rate."""
    log(f"bench: {label} fp32 tile {w['tile'][:w['dims']]} block {block} warmup {warmup} steps {steps}")
    counts, dt, kt, fe = run_gpu(w, "fp32", steps, warmup, graphs, time_kernels, block)
    npart = sum(counts)
    occ = occupied_cells(w)
    ncells = 1
    for a in range(w["dims"]):
        ncells *= w["n"][a]
    es = 4
    # particle kernel: the particle state, the staged E and B of the occupied cells, and the current
    # window added into J (one FP64 word of quanta per component in the FP32 form)
    bytes_particle = particle_bytes_per_step(w, counts, es) + occ * (6 * es + 3 * 8)
    # field kernel: E and B read and written at every node; J read and cleared where deposits are
    bytes_field = ncells * 12 * es + occ * 3 * 8 * 2
    bytes_step = bytes_particle + bytes_field
    t_particle_ms = float(kt[0])
    achieved = bytes_particle / (t_particle_ms * 1e-3) / 1e9
    ms_step = dt / steps * 1e3
    step_gbs = bytes_step / (ms_step * 1e-3) / 1e9
    return {
        "rate": npart * steps / dt, "dt": dt, "npart": npart, "counts": counts, "occ": occ, "ncells": ncells,
        "ms_step": ms_step, "kt": kt, "field_energy_end": fe,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(w["name"], w["tile"][:w["dims"]], block, w.get("unit", 0)),
                     "kernel": f"k_particles<{w['dims']},float,false,false>", "bytes_per_launch": bytes_particle},
        "field_roofline": {"bound": "hbm", "achieved": bytes_field / (float(kt[1]) * 1e-3) / 1e9,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": bytes_field / (float(kt[1]) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "traffic": committed_traffic(w["name"], w["tile"][:w["dims"]], block, w.get("unit", 0),
                                                        "k_fields"),
                           "kernel": f"k_fields<{w['dims']},float,false>", "bytes_per_launch": bytes_field},
        "step_roofline": {"bytes_per_step": bytes_step, "achieved": step_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS},
        "kernels_ms": {"particles": t_particle_ms, "fields": float(kt[1]), "sort_per_sort": float(kt[2]),
                       "particle_kernel_rate": npart / (t_particle_ms * 1e-3)},
    }


def tensor_list_sizes(wt):
    """Lengths of the two node lists of the full-tensor passes: nodes whose update terms are averaged
    (each folded node's neighbours +s e_a - t e_b over its nonzero entries) and folded nodes."""
    import numpy as np
    from paper_2501_07465_amd import workloads as W
    off = W.eps_offdiag_map(wt)  # [6][z][y][x]
    dims = wt["dims"]
    fold = np.any(off != 0, axis=0)
    need = np.zeros_like(fold)
    for m in range(6):
        a = m // 2
        b = (m % 2) if (m % 2) < a else (m % 2) + 1
        nz = off[m] != 0
        for sa in range(2 if a < dims else 1):
            for tb in range(2 if b < dims else 1):
                shift = [0, 0, 0]
                shift[a] += sa
                shift[b] -= tb
                # arrays are [z, y, x]; the entries lie away from open faces, so a roll is exact
                need |= np.roll(nz, (shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    return int(need.sum()), int(fold.sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="sphere3d")
    ap.add_argument("--secondary", default="disk2d", help="second FP32 leg with its own roofline ('' skips it)")
    ap.add_argument("--secondary-steps", type=int, default=4000)
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=200)
    ap.add_argument("--time-kernels", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=str, default=None, help="particle tile, e.g. 16x16 (default: tuned)")
    ap.add_argument("--block", type=int, default=None, help="particle-kernel block (default: tuned)")
    ap.add_argument("--unit", type=int, default=None, help="particles per work unit (default: tuned; 0 = tile)")
    ap.add_argument("--autotune", action="store_true", help="measure the tile/block/unit candidates now")
    ap.add_argument("--eps-inf", type=float, default=3.7,
                    help="background permittivity of the metal for the dielectric legs on the disk (0: skip)")
    ap.add_argument("--eps-steps", type=int, default=400)
    ap.add_argument("--no-tensor", action="store_true", help="skip the full-tensor dielectric leg")
    ap.add_argument("--no-diagonal", action="store_true", help="skip the diagonal dielectric leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the legs of the other optional physics (walls, barrier, Dirac mass, ribbon)")
    ap.add_argument("--variant-steps", type=int, default=400)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-scale", type=float, default=1.0)
    ap.add_argument("--serve-load", type=float, default=0.75)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="also run a float32 elementwise copy of this many MiB 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2501_07465_amd import autotune, pic, workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    def log(m):
        print(m, file=sys.stderr, flush=True)

    if args.tile or args.block or args.unit is not None:
        w = W.WORKLOADS[args.workload]()
        if args.tile:
            t = [int(v) for v in args.tile.split("x")]
            w["tile"] = t + [1] * (3 - len(t))
        block = args.block or 256
        w["unit"] = args.unit or 0
        tuning = "explicit"
    else:
        w, block, tuning = tuned(args.workload, log, args.autotune)
    tile = w["tile"][:w["dims"]]
    graphs = not args.no_graphs
    P = int(w.get("sort_every", 20))
    # the timed steps start on a sort-period boundary, so whole periods replay captured graphs
    warmup = max(P, -(-args.warmup // P) * P)
    if args.calib_mib:
        # counter calibration: torch's vectorized elementwise copy of calib_mib MiB, and the library's
        # structure-of-arrays copy (8 float arrays, 4-byte accesses per lane, calib_mib MiB in total)
        a = torch.ones(args.calib_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        n8 = (args.calib_mib << 18) // 8
        srcs = [a[k * n8:(k + 1) * n8] for k in range(8)]
        dsts = [b[k * n8:(k + 1) * n8] for k in range(8)]
        st = torch.cuda.current_stream().cuda_stream
        for _ in range(3):
            pic.pic_measure_soa_copy([x.data_ptr() for x in srcs], [x.data_ptr() for x in dsts], n8, st)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        del a, b, srcs, dsts
    head = fp32_leg(w, block, args.steps, warmup, graphs, args.time_kernels, args.workload, log)
    npart, rate32 = head["npart"], head["rate"]
    log(f"bench: fp32 {rate32:.3e} particle-steps/s; fp64 {args.fp64_steps} steps")
    fp64 = None
    if args.fp64_steps > 0:
        # the FP64 form needs twice the LDS per window: halve the tile's longest axis until it fits
        w64 = copy.deepcopy(w)
        t64 = w64["tile"]
        while autotune.lds_bytes(t64[:w["dims"]], w["dims"], "fp64", block) > autotune.LDS_BYTES:
            a = max(range(w["dims"]), key=lambda k: t64[k])
            t64[a] //= 2
        fp64_steps = max(P, args.fp64_steps // P * P)
        _, dt64, _, _ = run_gpu(w64, "fp64", fp64_steps, warmup, graphs, 0, block)
        rate64 = npart * fp64_steps / dt64
        fp64 = {"value": rate64, "unit": "particle-steps/s", "steps": fp64_steps, "warmup": warmup,
                "tile": t64[:w["dims"]], "ms_per_step": dt64 / fp64_steps * 1e3, "fp32_speedup": rate32 / rate64,
                "graph_replays": fp64_steps // P if graphs else 0}
    line = {
        "metric": METRIC,
        "value": rate32,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(w, npart), "particles": npart, "cells": head["ncells"],
                   "occupied_cells": head["occ"], "graphs": graphs, "tile": tile, "block": block,
                   "unit": w.get("unit", 0), "tuning": tuning, "sort_every": P, "warmup_run": warmup,
                   "graph_replays": args.steps // P if graphs else 0,
                   "plain_steps": args.steps % P if graphs else args.steps},
        "fp64": fp64,
        "kernels_ms": head["kernels_ms"],
        "roofline": head["roofline"],
        "field_roofline": head["field_roofline"],
        "step_roofline": head["step_roofline"],
        "field_energy_end": head["field_energy_end"],
    }
    # the same kernels against what a plain streaming copy reaches on this GPU (not in the counter
    # runs, whose calibration copies must be the only launches of that kernel)
    if not args.calib_mib:
        ceiling = copy_ceiling(log)
        line["copy_ceiling"] = ceiling
        for k in ("roofline", "field_roofline"):
            line[k]["copy_frac"] = line[k]["achieved"] / ceiling["achieved"]
    wd, bd = None, 256
    if args.secondary:
        wd, bd, _ = tuned(args.secondary, log)
        sec = fp32_leg(wd, bd, args.secondary_steps, 200, graphs, args.time_kernels, args.secondary, log)
        line["secondary"] = {"workload": describe(wd, sec["npart"]), "value": sec["rate"],
                             "unit": "particle-steps/s", "steps": args.secondary_steps, "ms_per_step": sec["ms_step"],
                             "tile": wd["tile"][:wd["dims"]], "block": bd, "unit_particles": wd.get("unit", 0),
                             "kernels_ms": sec["kernels_ms"], "roofline": sec["roofline"],
                             "field_roofline": sec["field_roofline"], "step_roofline": sec["step_roofline"]}
    if wd is not None and wd["name"] == "disk2d" and args.eps_inf > 0 and not args.no_diagonal:
        # the disk with a per-cell inverse permittivity (the metal's background eps inside the disk):
        # the dielectric variant of the field kernel reads 3 more values per node
        es = 4
        ncd, occd = sec["ncells"], sec["occ"]
        we = W.with_dielectric(wd, [args.eps_inf] * 3)
        log(f"bench: dielectric leg, eps {args.eps_inf} in {we['dielectric']['region']['kind']}")
        _, dte, kte, _ = run_gpu(we, "fp32", args.eps_steps, 20, graphs, args.time_kernels, bd)
        f_bytes = ncd * 12 * es + occd * 3 * 8 * 2 + ncd * 3 * es  # E, B; J read and cleared; eps^-1
        f_ms = float(kte[1])
        f_gbs = f_bytes / (f_ms * 1e-3) / 1e9
        line["dielectric"] = {
            "workload": "disk2d", "eps": [args.eps_inf] * 3, "region": we["dielectric"]["region"]["kind"],
            "steps": args.eps_steps, "value": sec["npart"] * args.eps_steps / dte, "unit": "particle-steps/s",
            "ms_per_step": dte / args.eps_steps * 1e3,
            "kernels_ms": {"particles": float(kte[0]), "fields": f_ms, "fields_without": float(sec["kt"][1])},
            "field_roofline": {"bound": "hbm", "achieved": f_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": f_gbs / HBM_PEAK_GBS, "bytes_per_launch": f_bytes,
                               "kernel": "k_fields<2,float,true>"}}
    if wd is not None and wd["name"] == "disk2d" and args.eps_inf > 0 and not args.no_tensor:
        # a full tensor: the background permittivity with in-plane and out-of-plane off-diagonal terms
        es = 4
        e = args.eps_inf
        eps_t = [[e, 0.1 * e, 0.05 * e], [0.1 * e, 0.9 * e, 0.05 * e], [0.05 * e, 0.05 * e, 1.1 * e]]
        wt = W.with_dielectric(wd, eps_t)
        nu, nfold = tensor_list_sizes(wt)
        log(f"bench: full-tensor leg, {nfold} folded nodes, {nu} update-term nodes")
        _, dtt, ktt, _ = run_gpu(wt, "fp32", args.eps_steps, 20, graphs, args.time_kernels, bd)
        t_bytes = sec["ncells"] * 18 * es + sec["occ"] * 3 * 8 * 2 + nu * 12 * es + nfold * 18 * es
        t_ms = float(ktt[1])
        t_gbs = t_bytes / (t_ms * 1e-3) / 1e9
        line["tensor"] = {
            "workload": "disk2d", "eps": eps_t, "region": wt["dielectric"]["region"]["kind"],
            "steps": args.eps_steps, "folded_nodes": nfold, "update_term_nodes": nu,
            "value": sec["npart"] * args.eps_steps / dtt, "unit": "particle-steps/s",
            "ms_per_step": dtt / args.eps_steps * 1e3,
            "kernels_ms": {"particles": float(ktt[0]), "field_step": t_ms, "fields_without": float(sec["kt"][1])},
            "field_roofline": {"bound": "hbm", "achieved": t_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": t_gbs / HBM_PEAK_GBS, "bytes_per_step": t_bytes,
                               "kernels": ["k_tensor_u<2,float>", "k_tensor_fold<2,float>",
                                           "k_fields<2,float,true>"]}}
    if wd is not None and wd["name"] == "disk2d" and not args.no_variants:
        line["variants"] = run_variants(wd, bd, sec["kt"], sec["npart"], sec["rate"], args, graphs, log)
    if args.serve_requests > 0:
        # the disk's tuned tile, block and unit for every request of the stream
        line["serve"] = run_serve(args.serve_requests, args.serve_scale, args.serve_load, bd,
                                  wd["tile"][:2] if wd is not None else None, args.serve_budget_gib,
                                  args.serve_slots, log, wd.get("unit", 0) if wd is not None else 0)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, log)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
