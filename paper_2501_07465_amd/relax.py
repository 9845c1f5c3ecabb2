"""The FD relaxation study of Sec. 2 on the device: the high-energy tail of the macroparticle
kinetic-energy histogram is fitted to exp(-E / beta) along the run, and the growth of the apparent
temperature beta(t) to beta = A sqrt(t).

The histogram is taken on the device (``pic_energy_histogram``); the fits are host arithmetic on
its counts:

* ``tail_beta``: weighted least squares of ln N over the tail bins (E at or above ``e_lo``, at
  least ``min_count`` macroparticles a bin, Poisson weights N), beta = -1 / slope.  Reading: the
  paper names the form exp(-E / beta) and not the window; the study's window starts two initial
  kT above mu, where the Fermi-Dirac occupation is within 12% of exponential (the fitted beta of
  the loaded state is then about 1.05 kT), with bins of about one initial kT.
* ``sqrt_law``: A of beta = A sqrt(t) by least squares through the origin over the samples t > 0.

``python -m paper_2501_07465_amd.relax --density 6e28 --ppc 16 32 64 128 --fs 20`` runs the study
and prints one JSON line per case.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

QE = 1.602176634e-19


def bin_centres(e_max: float, nbins: int) -> np.ndarray:
    return (np.arange(nbins) + 0.5) * (e_max / nbins)


def tail_beta(counts, e_max: float, e_lo: float, min_count: int = 10) -> float:
    """beta (J) of exp(-E / beta) fitted to the histogram bins at or above e_lo (the overflow entry
    counts[nbins] is ignored).  NaN if fewer than three bins qualify."""
    counts = np.asarray(counts, dtype=np.float64)
    nb = counts.size - 1
    e = bin_centres(e_max, nb)
    n = counts[:nb]
    m = (e >= e_lo) & (n >= min_count)
    if m.sum() < 3:
        return float("nan")
    x, y, wts = e[m], np.log(n[m]), n[m]
    xm = np.sum(wts * x) / np.sum(wts)
    ym = np.sum(wts * y) / np.sum(wts)
    slope = np.sum(wts * (x - xm) * (y - ym)) / np.sum(wts * (x - xm) ** 2)
    return float(-1.0 / slope) if slope < 0 else float("nan")


def sqrt_law(t, beta) -> float:
    """A of beta = A sqrt(t), least squares through the origin over the samples with t > 0."""
    t = np.asarray(t, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    m = (t > 0) & np.isfinite(beta)
    s = np.sqrt(t[m])
    return float(np.sum(s * beta[m]) / np.sum(s * s))


def run_case(density: float, ppc: int, t_end_fs: float, samples: int = 20, nbins: int = 200, n: int = 16,
             log=None):
    """One study case on the device: beta(t) at `samples` times over t_end_fs, and A."""
    from . import autotune, pic, workloads as W
    w = W.relax3d(density=density, ppc=ppc, n=n, t_end_fs=t_end_fs)
    # the tile, block and unit tuned for the 16^3, 128 ppc cube (small tiles split into units: the
    # cube has few cells for many particles)
    tuned = autotune.shipped(W.relax3d(n=16, ppc=128), "fp32")
    block = 256
    if tuned is not None:
        w = autotune.apply(w, tuned)
        block = int(tuned["block"])
    sp = w["species"][0]
    ef = sp["e_fermi"]
    kt0 = w["relax"]["temperature_ev"] * QE
    e_max = ef + 40.0 * kt0
    e_lo = ef + 2.0 * kt0
    sim = pic.Simulation(w, precision="fp32", graphs=True, block=block, unit=w.get("unit", 0))
    per = max(20, (w["steps"] // samples) // 20 * 20)
    t, beta = [], []
    steps = 0
    t0 = time.perf_counter()
    while True:
        h = pic.pic_energy_histogram(sim.h, 0, e_max, nbins)
        t.append(steps * w["dt"])
        beta.append(tail_beta(h, e_max, e_lo, min_count=5))
        if steps >= w["steps"]:
            break
        sim.step(per)
        steps += per
    sim.sync()
    wall = time.perf_counter() - t0
    A = sqrt_law(t, beta)
    out = {"density": density, "ppc": ppc, "particles": sim.count(0), "steps": steps, "dt": w["dt"],
           "t_fs": [x * 1e15 for x in t], "beta_ev": [b / QE for b in beta],
           "A_ev_per_sqrt_fs": A / QE * np.sqrt(1e-15), "wall_s": wall}
    if log:
        log(f"relax: n={density:.0e} ppc={ppc}: A = {out['A_ev_per_sqrt_fs']:.4g} eV/fs^0.5, "
            f"beta {out['beta_ev'][0]:.4f} -> {out['beta_ev'][-1]:.4f} eV in {wall:.1f} s")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--density", type=float, nargs="+", default=[6e28])
    ap.add_argument("--ppc", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--fs", type=float, default=20.0)
    ap.add_argument("--samples", type=int, default=20)
    args = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    for d in args.density:
        for p in args.ppc:
            print(json.dumps(run_case(d, p, args.fs, args.samples, log=log)), flush=True)


if __name__ == "__main__":
    main()
