"""Autotuner for the particle tile and the particle-kernel block size.

The tile sets the LDS window of a particle block (E, B on T + 4 nodes per axis, J on T + 3) and
the halo overhead; the unit (particles per block) splits a tile's particles over several blocks,
each with its own current slot, so that a few dense tiles still spread over every compute unit;
the block size sets how many wavefronts share one unit.  The best choice depends on the particle
density and on how much of the grid the material fills, so it is measured: every candidate that
fits 64 KiB of LDS is run for a few sort periods through the captured-graph path and scored by
wall time per step (sort, particle and field kernels together).  The search takes tile x block
with whole-tile units and with 2048-particle units, then more unit sizes for the best tile and
block.  Results are cached per workload shape in a JSON file under the user's cache directory.
"""
from __future__ import annotations

import copy
import json
import os
import time

from . import pic

TILES = {
    1: [(32,), (64,), (128,), (256,)],
    2: [(8, 8), (16, 8), (16, 16), (32, 8), (32, 16), (64, 8), (32, 32), (64, 16)],
    3: [(4, 4, 4), (8, 4, 4), (8, 8, 4), (16, 4, 4), (8, 8, 8)],
}
BLOCKS = (256, 512)
UNITS_FIRST = (0, 2048)
UNITS_SECOND = (1024, 4096, 8192)
LDS_BYTES = 65536


STRAY_SCRATCH = 48  # values of LDS scratch per wavefront in the particle kernel


def lds_bytes(tile, dims: int, precision: str, block: int = 512) -> int:
    """LDS of a particle workgroup: E, B window (T + 4 per axis) and the stray scratch as reals,
    then the current window (T + 3 per axis) as FP64 words (one per component; two in FP64)."""
    es = 8 if precision == "fp64" else 4
    vf = vj = 1
    for a in range(dims):
        vf *= tile[a] + 4
        vj *= tile[a] + 3
    f = es * (6 * vf + STRAY_SCRATCH * (block // 64))
    f = (f + 7) // 8 * 8
    return f + 8 * (2 if precision == "fp64" else 1) * 3 * vj


def candidates(w: dict, precision: str):
    dims = w["dims"]
    out = []
    for t in TILES[dims]:
        if any(t[a] > w["n"][a] for a in range(dims)):
            continue
        for b in BLOCKS:
            if lds_bytes(t, dims, precision, b) > LDS_BYTES:
                continue
            for u in UNITS_FIRST:
                out.append((tuple(t), b, u))
    return out


def shape_key(w: dict, precision: str) -> str:
    ppc = "+".join(str(sp.get("ppc", 0)) for sp in w["species"])
    return f"{w.get('name', 'w')}|{precision}|{'x'.join(str(v) for v in w['n'][:w['dims']])}|{ppc}"


def _cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_2501_07465_amd", "autotune.json")


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(w: dict, precision: str = "fp32", periods: int = 2, cands=None, use_cache: bool = True,
         log=None) -> dict:
    """Measure the candidates on workload ``w``; returns {"tile", "block", "ms_per_step", "trials"}."""
    key = shape_key(w, precision)
    path = _cache_path()
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            hit = dict(hit)
            hit["cached"] = True
            return hit
    P = int(w.get("sort_every", 20))
    trials = []

    def trial(tile, block, unit):
        wt = copy.deepcopy(w)
        wt["tile"] = list(tile) + [1] * (3 - len(tile))
        try:
            sim = pic.Simulation(wt, precision=precision, graphs=True, block=block, unit=unit,
                                 series_cap=P * (periods + 2) + 64)
        except pic.PicError as e:
            if log:
                log(f"autotune: tile {tile} block {block} unit {unit} rejected: {e}")
            return
        sim.step(2 * P)  # first replays load the code and warm the caches
        sim.sync()
        t0 = time.perf_counter()
        sim.step(P * periods)
        sim.sync()
        ms = (time.perf_counter() - t0) * 1e3 / (P * periods)
        trials.append({"tile": list(tile), "block": block, "unit": unit, "ms_per_step": ms})
        if log:
            log(f"autotune: tile {tile} block {block} unit {unit}: {ms:.4f} ms/step")
        del sim

    for tile, block, unit in (cands or candidates(w, precision)):
        trial(tile, block, unit)
    if not trials:
        raise RuntimeError("autotune: no candidate fits")
    if cands is None:
        first = min(trials, key=lambda t: t["ms_per_step"])
        for unit in UNITS_SECOND:
            trial(tuple(first["tile"]), first["block"], unit)
    best = min(trials, key=lambda t: t["ms_per_step"])
    res = {"tile": best["tile"], "block": best["block"], "unit": best["unit"], "ms_per_step": best["ms_per_step"],
           "trials": trials}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache = _load_cache(path)
            cache[key] = {k: v for k, v in res.items()}
            with open(path + ".tmp", "w") as f:
                json.dump(cache, f)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    res["cached"] = False
    return res


def apply(w: dict, res: dict) -> dict:
    """A copy of ``w`` with the tuned tile and unit (the block size is a launch argument)."""
    wt = copy.deepcopy(w)
    t = list(res["tile"])
    wt["tile"] = t + [1] * (3 - len(t))
    wt["unit"] = int(res.get("unit", 0))
    return wt


# ---- shipped tuning table --------------------------------------------------------------------------
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def shipped(w: dict, precision: str = "fp32"):
    """The tuned (tile, block) recorded for this workload shape on an MI355X, or None."""
    try:
        with open(SHIPPED) as f:
            hit = json.load(f).get(shape_key(w, precision))
    except (OSError, ValueError):
        return None
    return dict(hit) if hit else None


def main():
    import argparse
    from . import workloads as W
    ap = argparse.ArgumentParser(description="measure tile/block candidates for a workload on this GPU")
    ap.add_argument("--workload", default="disk2d")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--periods", type=int, default=3)
    ap.add_argument("--write", action="store_true", help="record the result in the shipped table")
    ap.add_argument("--out", default=SHIPPED, help="table to update with --write")
    a = ap.parse_args()
    w = W.WORKLOADS[a.workload]()
    res = tune(w, a.precision, periods=a.periods, use_cache=False, log=lambda m: print(m, flush=True))
    print(json.dumps({k: v for k, v in res.items() if k != "trials"}))
    if a.write:
        try:
            with open(a.out) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
        table[shape_key(w, a.precision)] = {"tile": res["tile"], "block": res["block"], "unit": res["unit"],
                                            "ms_per_step": res["ms_per_step"], "trials": res["trials"]}
        with open(a.out, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
