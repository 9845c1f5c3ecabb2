"""Benchmark of the PIC step on one MI355X: particle-steps/s (gather + push + deposit + fields).

Workload: the 2D3V disk (1024 x 1024 cells of 1 nm, 200 nm metal disk, 16 ppc Fermi-Dirac
free electrons + 16 ppc bound Lorentz electrons, 800 nm plane-wave pulse), FP32 form, with
synthetic seeded inputs.  W warm-up steps, then exactly K timed steps (HIP graphs replay one
sort period of steps at a time), bracketed by device synchronisation.  The FP64 GPU rate of the
same workload is reported beside it, as is the plain-C FP64 oracle timed on the host on a
bounded sample (cpu_baseline).

roofline: the dominant kernel is the particle-tile kernel.  Its algorithmic bytes per launch are
the particle state read and written (per particle: 2D free 48 B, 2D bound 60 B, Dirac 48 B in
FP32) plus, per occupied cell, the six field components gathered (24 B) and the three current
components written (12 B).  achieved = bytes / average launch time (HIP events on the
simulation's stream, measured here), peak = 8 TB/s HBM3E.

One GPU only: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (gather+push+deposit) FP32 vs FP64 GPU; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0


def particle_bytes(w, counts, es):
    """Algorithmic bytes of one particle-kernel launch (see module docstring)."""
    d = w["dims"]
    total = 0
    occupied = set()
    for sp, n in zip(w["species"], counts):
        if sp["kind"] == "bound":
            per = (4 + d * es + 6 * es) + 6 * es  # anchor cell/offset, xi, v read; xi, v written
        else:
            per = 2 * (4 + d * es + 3 * es)       # cell, offset, v read and written
        total += n * per
    return total


def occupied_cells(sim_counts, w):
    """Cells holding particles at load time (region cells), from the workload geometry."""
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


def run_gpu(w, precision, steps, warmup, graphs=True, time_kernels=0, block=256):
    import torch
    from paper_2501_07465_amd import pic
    sim = pic.Simulation(w, precision=precision, graphs=graphs, series_cap=steps + warmup + time_kernels + 64,
                         block=block)
    counts = [sim.count(s) for s in sim.species]
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = None
    if time_kernels:
        kt = pic.pic_time_kernels(sim.h, time_kernels)
    fe = sim.field_energy()
    return sim, counts, dt, kt, fe


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
    ap.add_argument("--tile", type=str, default=None, help="particle tile, e.g. 8x8")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_07465_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = W.WORKLOADS[args.workload]()
    if args.tile:
        t = [int(v) for v in args.tile.split("x")]
        w["tile"] = t + [1] * (3 - len(t))
    graphs = not args.no_graphs
    if args.copy_mib:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"bench: {args.workload} fp32 warmup {args.warmup} steps {args.steps}", file=sys.stderr, flush=True)
    sim, counts, dt32, kt, fe = run_gpu(w, "fp32", args.steps, args.warmup, graphs, args.time_kernels, args.block)
    npart = sum(counts)
    rate32 = npart * args.steps / dt32
    del sim
    print(f"bench: fp32 {rate32:.3e} particle-steps/s; fp64 {args.fp64_steps} steps", file=sys.stderr, flush=True)
    sim64, _, dt64, _, _ = run_gpu(w, "fp64", args.fp64_steps, 20, graphs, 0)
    rate64 = npart * args.fp64_steps / dt64
    del sim64
    occ = occupied_cells(counts, w)
    es = 4
    bytes_launch = particle_bytes(w, counts, es) + occ * (6 * es + 3 * es)
    t_particle_ms = float(kt[0])
    achieved = bytes_launch / (t_particle_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": rate32,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: 2D3V {w['n'][0]}x{w['n'][1]} cells of 1 nm, disk radius 100 cells, "
                               f"16 ppc FD free + 16 ppc bound ({npart} particles), 800 nm pulse, FP32",
                   "particles": npart, "graphs": graphs, "tile": w["tile"], "block": args.block},
        "fp64": {"value": rate64, "unit": "particle-steps/s", "steps": args.fp64_steps,
                 "ms_per_step": dt64 / args.fp64_steps * 1e3, "fp32_speedup": rate32 / rate64},
        "kernels_ms": {"particles": t_particle_ms, "fields": float(kt[1]), "sort": float(kt[2])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_particles<2,float>", "bytes_per_launch": bytes_launch},
        "field_energy_end": fe,
    }
    if not args.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
