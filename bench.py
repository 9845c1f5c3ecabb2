"""Benchmark of the PIC step on one MI355X: particle-steps/s (sort + gather + push + deposit + fields).

Default workload: the 2D3V disk (1024 x 1024 cells of 1 nm, 200 nm metal disk, 16 ppc Fermi-Dirac
free electrons + 16 ppc bound Lorentz electrons, 800 nm pulse at 1e9 V/m), FP32 form (int32 cell +
FP32 offset), synthetic seeded inputs.  W warm-up steps, then exactly K timed steps (captured
graphs replay one 20-step sort period at a time), bracketed by device synchronisation.

Beside it: the FP64 GPU rate of the same workload and the FP32/FP64 speedup; a roofline for the
dominant kernel (the particle kernel) and for the whole step; a serving run (continuous batching
of seeded uneven requests with Poisson arrivals, p50/p99 latency); the plain-C FP64 oracle timed
on the host on a bounded sample (cpu_baseline).

A dielectric leg runs the same workload with the metal's background permittivity (eps = 3.7 by
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
  cell), the update-term pass (E, B, J read, U written: 48 B per cell) and the fold (off-diagonal
  entries read: 24 B per cell; per folded node U, inverse permittivity and J read, J written: 48 B).
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


def committed_traffic(workload, tile, block, unit):
    """Traffic per launch from the committed counter summary, if it matches the current kernels."""
    from paper_2501_07465_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_k_particles_{workload}.txt")
    if not os.path.exists(path):
        return None
    t = profiling.read_traffic_file(path)
    if (t.get("source_digest") != profiling.source_digest() or t.get("tile") != "x".join(str(v) for v in tile)
            or t.get("block") != str(block) or t.get("unit") != str(unit)):
        return None
    return float(t["traffic_bytes"])


def cpu_baseline(w, budget_s):
    """The FP64 oracle on the host, on the first steps of the same workload."""
    from oracle import oracle as O
    ref = O.build_workload(w)
    n = sum(ref.count(s) for s in range(len(w["species"])))
    t0 = time.perf_counter()
    steps = 0
    while True:
        ref.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 200:
            break
    return {"value": n * steps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{w['name']} full size ({n} particles), first {steps} steps after loading, "
                      f"{el:.1f} s single-threaded plain C FP64"}


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
    return {"requests": st["requests"], "p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_s": st["mean_s"],
            "particle_steps_per_s": st["particle_steps_per_s"], "arrival_rate_hz": lam, "load": load,
            "capacity_probe": cap, "grid_scale": scale, "hbm_budget_gib": budget_gib, "slots": slots,
            "requests_desc": "seeded 2D3V disk/rod/slab requests, grid side U[128,1024] x scale, 8-32 ppc "
                             "free + 8-32 ppc bound, 500-4000 steps, FP32"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="disk2d")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=1000)
    ap.add_argument("--time-kernels", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=str, default=None, help="particle tile, e.g. 16x16 (default: tuned)")
    ap.add_argument("--block", type=int, default=None, help="particle-kernel block (default: tuned)")
    ap.add_argument("--unit", type=int, default=None, help="particles per work unit (default: tuned; 0 = tile)")
    ap.add_argument("--autotune", action="store_true", help="measure the tile/block/unit candidates now")
    ap.add_argument("--eps-inf", type=float, default=3.7,
                    help="background permittivity of the metal for the dielectric leg (0: skip it)")
    ap.add_argument("--eps-steps", type=int, default=400)
    ap.add_argument("--no-tensor", action="store_true", help="skip the full-tensor dielectric leg")
    ap.add_argument("--no-diagonal", action="store_true", help="skip the diagonal dielectric leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the legs of the other optional physics (walls, barrier, Dirac mass, ribbon)")
    ap.add_argument("--variant-steps", type=int, default=400)
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-scale", type=float, default=0.25)
    ap.add_argument("--serve-load", type=float, default=0.75)
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--calib-mib", type=int, default=0,
                    help="also run a float32 elementwise copy of this many MiB 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2501_07465_amd import autotune, workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    def log(m):
        print(m, file=sys.stderr, flush=True)

    w = W.WORKLOADS[args.workload]()
    tuning = "default"
    block = 256
    if args.tile or args.block or args.unit is not None:
        if args.tile:
            t = [int(v) for v in args.tile.split("x")]
            w["tile"] = t + [1] * (3 - len(t))
        block = args.block or 256
        w["unit"] = args.unit or 0
        tuning = "explicit"
    else:
        res = None if args.autotune else autotune.shipped(w, "fp32")
        tuning = "shipped"
        if res is None:
            log("bench: autotuning tile and block")
            res = autotune.tune(w, "fp32", periods=2, use_cache=False, log=log)
            tuning = "measured"
        w = autotune.apply(w, res)
        block = int(res["block"])
    tile = w["tile"][:w["dims"]]
    graphs = not args.no_graphs
    if args.calib_mib:
        a = torch.ones(args.calib_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    log(f"bench: {args.workload} fp32 tile {tile} block {block} warmup {args.warmup} steps {args.steps}")
    counts, dt32, kt, fe = run_gpu(w, "fp32", args.steps, args.warmup, graphs, args.time_kernels, block)
    npart = sum(counts)
    rate32 = npart * args.steps / dt32
    log(f"bench: fp32 {rate32:.3e} particle-steps/s; fp64 {args.fp64_steps} steps")
    fp64 = None
    if args.fp64_steps > 0:
        # the FP64 form needs twice the LDS per window: halve the tile's longest axis until it fits
        w64 = copy.deepcopy(w)
        t64 = w64["tile"]
        while autotune.lds_bytes(t64[:w["dims"]], w["dims"], "fp64", block) > autotune.LDS_BYTES:
            a = max(range(w["dims"]), key=lambda k: t64[k])
            t64[a] //= 2
        _, dt64, _, _ = run_gpu(w64, "fp64", args.fp64_steps, 20, graphs, 0, block)
        rate64 = npart * args.fp64_steps / dt64
        fp64 = {"value": rate64, "unit": "particle-steps/s", "steps": args.fp64_steps, "tile": t64[:w["dims"]],
                "ms_per_step": dt64 / args.fp64_steps * 1e3, "fp32_speedup": rate32 / rate64}
    occ = occupied_cells(w)
    ncells = 1
    for a in range(w["dims"]):
        ncells *= w["n"][a]
    es = 4
    bytes_particle = particle_bytes_per_step(w, counts, es) + occ * (6 * es + 3 * es)
    bytes_step = bytes_particle + ncells * 12 * es + occ * 3 * es
    t_particle_ms = float(kt[0])
    achieved = bytes_particle / (t_particle_ms * 1e-3) / 1e9
    ms_step = dt32 / args.steps * 1e3
    step_gbs = bytes_step / (ms_step * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": rate32,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(w, npart), "particles": npart, "cells": ncells, "occupied_cells": occ,
                   "graphs": graphs, "tile": tile, "block": block, "unit": w.get("unit", 0), "tuning": tuning,
                   "sort_every": 20},
        "fp64": fp64,
        "kernels_ms": {"particles": t_particle_ms, "fields": float(kt[1]), "sort_per_sort": float(kt[2]),
                       "particle_kernel_rate": npart / (t_particle_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(args.workload, tile, block, w.get("unit", 0)),
                     "kernel": f"k_particles<{w['dims']},float,false,false>", "bytes_per_launch": bytes_particle},
        "step_roofline": {"bytes_per_step": bytes_step, "achieved": step_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS},
        "field_energy_end": fe,
    }
    if args.eps_inf > 0 and not args.no_diagonal:
        # the same workload with a per-cell inverse permittivity (the metal's background eps inside the
        # first species' region): the dielectric variant of the field kernel reads 3 more values per node
        we = W.with_dielectric(w, [args.eps_inf] * 3)
        log(f"bench: dielectric leg, eps {args.eps_inf} in {we['dielectric']['region']['kind']}")
        _, dte, kte, _ = run_gpu(we, "fp32", args.eps_steps, 20, graphs, args.time_kernels, block)
        f_bytes = ncells * 12 * es + occ * 3 * es + ncells * 3 * es
        f_ms = float(kte[1])
        f_gbs = f_bytes / (f_ms * 1e-3) / 1e9
        line["dielectric"] = {
            "eps": [args.eps_inf] * 3, "region": we["dielectric"]["region"]["kind"], "steps": args.eps_steps,
            "value": npart * args.eps_steps / dte, "unit": "particle-steps/s",
            "ms_per_step": dte / args.eps_steps * 1e3,
            "kernels_ms": {"particles": float(kte[0]), "fields": f_ms, "fields_without": float(kt[1])},
            "field_roofline": {"bound": "hbm", "achieved": f_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": f_gbs / HBM_PEAK_GBS, "bytes_per_launch": f_bytes,
                               "kernel": f"k_fields<{w['dims']},float,true>"}}
    if args.eps_inf > 0 and not args.no_tensor:
        # a full tensor: the background permittivity with in-plane and out-of-plane off-diagonal terms
        e = args.eps_inf
        eps_t = [[e, 0.1 * e, 0.05 * e], [0.1 * e, 0.9 * e, 0.05 * e], [0.05 * e, 0.05 * e, 1.1 * e]]
        wt = W.with_dielectric(w, eps_t)
        nfold = int(np.count_nonzero(np.any(W.eps_offdiag_map(wt) != 0, axis=0)))
        log(f"bench: full-tensor leg, {nfold} folded nodes")
        _, dtt, ktt, _ = run_gpu(wt, "fp32", args.eps_steps, 20, graphs, args.time_kernels, block)
        t_bytes = ncells * 18 * es + ncells * 12 * es + ncells * 6 * es + nfold * 12 * es
        t_ms = float(ktt[1])
        t_gbs = t_bytes / (t_ms * 1e-3) / 1e9
        line["tensor"] = {
            "eps": eps_t, "region": wt["dielectric"]["region"]["kind"], "steps": args.eps_steps,
            "folded_nodes": nfold, "value": npart * args.eps_steps / dtt, "unit": "particle-steps/s",
            "ms_per_step": dtt / args.eps_steps * 1e3,
            "kernels_ms": {"particles": float(ktt[0]), "field_step": t_ms, "fields_without": float(kt[1])},
            "field_roofline": {"bound": "hbm", "achieved": t_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": t_gbs / HBM_PEAK_GBS, "bytes_per_step": t_bytes,
                               "kernels": [f"k_tensor_u<{w['dims']},float>", f"k_tensor_fold<{w['dims']},float>",
                                           f"k_fields<{w['dims']},float,true>"]}}
    if not args.no_variants and args.workload == "disk2d":
        line["variants"] = run_variants(w, block, kt, npart, line["value"], args, graphs, log)
    if args.serve_requests > 0:
        line["serve"] = run_serve(args.serve_requests, args.serve_scale, args.serve_load, block,
                                  None, args.serve_budget_gib, args.serve_slots, log, w.get("unit", 0))
    if not args.no_cpu:
        log("bench: cpu baseline")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
