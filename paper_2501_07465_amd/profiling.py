"""Summaries of rocprofv3 output: per-kernel durations, per-dispatch HBM counters, and the HBM
traffic of one kernel calibrated against an elementwise copy of known size.

Inputs are the CSV files rocprofv3 writes with ``--output-format csv``:
``*_kernel_stats.csv`` (from ``--kernel-trace --stats``) and ``*_counter_collection.csv`` (from
``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, one counter per run; values in KiB per dispatch).

Two calibration kernels run in the same process (``bench.py --calib-mib M``, three times each),
each reading and writing exactly M MiB: torch's float32 elementwise multiply (wide vector
accesses) and the library's structure-of-arrays copy ``k_measure_soa_copy`` (8 float arrays, one
4-byte element of each per lane: the access pattern of the particle kernel).  The factor
M * 1024 / (KiB counted) of a calibration kernel turns the counted KiB of a kernel into bytes; the
summaries report the raw counted bytes, the bytes under each factor, and take the
structure-of-arrays factor as the traffic.  ``requests`` checks the factor: it counts the L2's read
requests by size (32, 64 and 128 bytes) and its write requests (32 and 64 bytes), whose byte sums
need no factor for a copy of known size.

    python -m paper_2501_07465_amd.profiling traffic --fetch DIR --write DIR --kernel NAME \
        --calib-mib M --out FILE --command "..."
    python -m paper_2501_07465_amd.profiling stats --trace DIR --out FILE --command "..."
    python -m paper_2501_07465_amd.profiling counters --run DIR --kernel NAME --out FILE --command "..."
    python -m paper_2501_07465_amd.profiling requests --rd DIR --wr DIR --kernel NAME --calib-mib M \
        --workload W --out FILE --command "..."
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_KERNEL = "MulFunctor"  # torch's vectorized elementwise kernel of the calibration multiply
SOA_KERNEL = "k_measure_soa_copy"  # the library's structure-of-arrays calibration copy
# the kernels, and the host code and sort that decide their launches and the order of their work
KERNEL_SOURCES = ("csrc/pic_kernels.inc", "csrc/pic_internal.h", "csrc/pic_k32.hip", "csrc/pic_k64.hip",
                  "csrc/pic_dpp.h", "csrc/pic_sort.hip", "csrc/pic_sort.h", "csrc/pic_host.hip")


def source_digest() -> str:
    """SHA-256 over the sources that decide what the profiled kernels do (counters go stale when it changes)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(pattern_dir: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(pattern_dir, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {pattern_dir}")
    return hits[0]


def kernel_stats(trace_dir: str) -> list[dict]:
    rows = []
    with open(_one(trace_dir, "_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]), "total_ns": float(r["TotalDurationNs"]),
                         "avg_ns": float(r["AverageNs"]), "pct": float(r["Percentage"]),
                         "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])})
    rows.sort(key=lambda r: -r["total_ns"])
    return rows


def counter_per_dispatch(run_dir: str, counter: str) -> dict:
    """kernel name -> list of counter values, one per dispatch."""
    out = collections.defaultdict(list)
    with open(_one(run_dir, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def _match(d: dict, sub: str) -> list:
    vals = []
    for k, v in d.items():
        if sub in k:
            vals.extend(v)
    if not vals:
        raise KeyError(f"no dispatch of a kernel matching {sub!r}")
    return vals


def traffic(fetch_dir: str, write_dir: str, kernel: str, calib_mib: float) -> dict:
    fetch = counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = counter_per_dispatch(write_dir, "WRITE_SIZE")
    kf, kw = _match(fetch, kernel), _match(write, kernel)
    cf, cw = _match(fetch, CALIB_KERNEL), _match(write, CALIB_KERNEL)
    sf, sw = _match(fetch, SOA_KERNEL), _match(write, SOA_KERNEL)
    for name, v in (("elementwise fetch", cf), ("elementwise write", cw), ("soa fetch", sf), ("soa write", sw)):
        if max(v) > 1.1 * min(v):
            raise ValueError(f"calibration dispatches of {name} disagree ({min(v)} .. {max(v)} KiB): "
                             "another launch of the kernel ran in the counter run")
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    ref_kib = calib_mib * 1024.0
    f_factor, w_factor = ref_kib / mean(cf), ref_kib / mean(cw)
    sf_factor, sw_factor = ref_kib / mean(sf), ref_kib / mean(sw)
    fetch_kib, write_kib = mean(kf), mean(kw)
    fetch_b = fetch_kib * 1024.0 * sf_factor
    write_b = write_kib * 1024.0 * sw_factor
    return {"kernel": kernel, "dispatches": len(kf), "fetch_kib": fetch_kib, "write_kib": write_kib,
            "raw_fetch_bytes": fetch_kib * 1024.0, "raw_write_bytes": write_kib * 1024.0,
            "calib_mib": calib_mib,
            "calib_fetch_kib": mean(cf), "calib_write_kib": mean(cw),
            "fetch_factor": f_factor, "write_factor": w_factor,
            "soa_calib_fetch_kib": mean(sf), "soa_calib_write_kib": mean(sw),
            "soa_fetch_factor": sf_factor, "soa_write_factor": sw_factor,
            "fetch_bytes_elementwise_factor": fetch_kib * 1024.0 * f_factor,
            "write_bytes_elementwise_factor": write_kib * 1024.0 * w_factor,
            "fetch_bytes": fetch_b, "write_bytes": write_b, "traffic_bytes": fetch_b + write_b}


def counter_summary(run_dir: str, kernels: list[str]) -> dict:
    """Per-dispatch averages of every counter in a counter-collection run, for matching kernels."""
    out = {}
    with open(_one(run_dir, "_counter_collection.csv")) as f:
        rows = list(csv.DictReader(f))
    for sub in kernels:
        acc = collections.defaultdict(list)
        meta = None
        for r in rows:
            if sub in r["Kernel_Name"]:
                acc[r["Counter_Name"]].append(float(r["Counter_Value"]))
                meta = {"grid": r["Grid_Size"], "workgroup": r["Workgroup_Size"], "vgpr": r["VGPR_Count"],
                        "lds": r["LDS_Block_Size"]}
        if acc:
            out[sub] = {"meta": meta, "counters": {c: sum(v) / len(v) for c, v in acc.items()},
                        "dispatches": max(len(v) for v in acc.values())}
    return out


RD_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
WR_COUNTERS = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum")


def request_bytes(rd_dir: str, wr_dir: str, kernels: list[str]) -> dict:
    """Bytes the L2 requested from memory per dispatch, from the request counts by size: reads as
    32 n_32 + 64 n_64 + 128 n_128 (and the share of each size), writes as 32 (n - n_64) + 64 n_64.
    Counted this way a copy of known size needs no factor, so the result checks the calibrated
    FETCH_SIZE and WRITE_SIZE figures."""
    rd = {c: counter_per_dispatch(rd_dir, c) for c in RD_COUNTERS}
    wr = {c: counter_per_dispatch(wr_dir, c) for c in WR_COUNTERS}
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    out = {}
    for k in kernels:
        m = {c: mean(_match(rd[c], k)) for c in RD_COUNTERS}
        w = {c: mean(_match(wr[c], k)) for c in WR_COUNTERS}
        n = m["TCC_EA0_RDREQ_sum"]
        sized = m["TCC_EA0_RDREQ_32B_sum"] + m["TCC_EA0_RDREQ_64B_sum"] + m["TCC_EA0_RDREQ_128B_sum"]
        out[k] = {"dispatches": len(_match(rd["TCC_EA0_RDREQ_sum"], k)),
                  "read_requests": n, "sized_fraction": sized / n if n else 0.0,
                  "share_32B": m["TCC_EA0_RDREQ_32B_sum"] / n if n else 0.0,
                  "share_64B": m["TCC_EA0_RDREQ_64B_sum"] / n if n else 0.0,
                  "share_128B": m["TCC_EA0_RDREQ_128B_sum"] / n if n else 0.0,
                  "read_bytes": 32 * m["TCC_EA0_RDREQ_32B_sum"] + 64 * m["TCC_EA0_RDREQ_64B_sum"]
                  + 128 * m["TCC_EA0_RDREQ_128B_sum"],
                  "write_bytes": 32 * (w["TCC_EA0_WRREQ_sum"] - w["TCC_EA0_WRREQ_64B_sum"])
                  + 64 * w["TCC_EA0_WRREQ_64B_sum"]}
    return out


def read_traffic_file(path: str) -> dict:
    """key = value lines of a traffic summary (values as text)."""
    out = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                out[k.strip()] = v.strip()
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib-mib", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--tile", required=True)
    t.add_argument("--block", required=True)
    t.add_argument("--unit", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--run", required=True)
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", action="append", default=[])
    q = sub.add_parser("requests")
    q.add_argument("--rd", required=True)
    q.add_argument("--wr", required=True)
    q.add_argument("--kernel", action="append", required=True)
    q.add_argument("--calib-mib", type=float, required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--command", action="append", default=[])
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--top", type=int, default=16)
    a = ap.parse_args()
    if a.cmd == "traffic":
        r = traffic(a.fetch, a.write, a.kernel, a.calib_mib)
        with open(a.out, "w") as f:
            f.write(f"# HBM traffic per dispatch of {a.kernel} on {a.workload} (rocprofv3 FETCH_SIZE, WRITE_SIZE)\n")
            for c in a.command:
                f.write(f"# command: {c}\n")
            f.write("# calibration: torch float32 elementwise multiply and the library's structure-of-arrays copy, "
                    "each reading and writing calib_mib MiB; factor = calib bytes / counted bytes; "
                    "fetch_bytes and write_bytes use the structure-of-arrays factors\n")
            f.write(f"workload = {a.workload}\ntile = {a.tile}\nblock = {a.block}\nunit = {a.unit}\n"
                    f"source_digest = {source_digest()}\n")
            for k, v in r.items():
                f.write(f"{k} = {v}\n")
        print(open(a.out).read())
    elif a.cmd == "requests":
        ks = [CALIB_KERNEL, SOA_KERNEL] + a.kernel
        r = request_bytes(a.rd, a.wr, ks)
        ref = a.calib_mib * 1024.0 * 1024.0
        with open(a.out, "w") as f:
            f.write(f"# memory requests of the L2 by size on {a.workload}, average per dispatch "
                    f"(rocprofv3 --pmc {' '.join(RD_COUNTERS)}, then {' '.join(WR_COUNTERS)})\n")
            for c in a.command:
                f.write(f"# command: {c}\n")
            f.write(f"# read_bytes = 32 n_32B + 64 n_64B + 128 n_128B; write_bytes = 32 (n - n_64B) + 64 n_64B; "
                    f"the calibration copies each read and write calib_mib = {a.calib_mib:g} MiB\n")
            f.write(f"# source_digest = {source_digest()}\n")
            for k, v in r.items():
                f.write(f"\n[{k}] dispatches {v['dispatches']}\n")
                for cn, cv in v.items():
                    if cn != "dispatches":
                        f.write(f"{cn} = {cv:.6g}\n")
                if k in (CALIB_KERNEL, SOA_KERNEL):
                    f.write(f"read_over_copy_size = {v['read_bytes'] / ref:.4f}\n"
                            f"write_over_copy_size = {v['write_bytes'] / ref:.4f}\n")
        print(open(a.out).read())
    elif a.cmd == "counters":
        r = counter_summary(a.run, a.kernel)
        with open(a.out, "w") as f:
            f.write("# rocprofv3 --pmc counters, average per dispatch\n")
            for cmd in a.command:
                f.write(f"# command: {cmd}\n")
            f.write(f"# source_digest = {source_digest()}\n")
            for k, v in r.items():
                f.write(f"\n[{k}] dispatches {v['dispatches']} {v['meta']}\n")
                for cn, cv in sorted(v["counters"].items()):
                    f.write(f"{cn} = {cv:.1f}\n")
        print(open(a.out).read())
    else:
        rows = kernel_stats(a.trace)
        with open(a.out, "w") as f:
            f.write("# rocprofv3 --kernel-trace --stats summary\n")
            for c in a.command:
                f.write(f"# command: {c}\n")
            f.write(f"# source_digest = {source_digest()}\n")
            f.write(f"{'kernel':80s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}\n")
            for r in rows[:a.top]:
                f.write(f"{r['name'][:80]:80s} {r['calls']:7d} {r['avg_ns'] / 1e3:10.2f} {r['min_ns'] / 1e3:10.2f} "
                        f"{r['max_ns'] / 1e3:10.2f} {r['pct']:6.2f}\n")
        print(open(a.out).read())


if __name__ == "__main__":
    main()
