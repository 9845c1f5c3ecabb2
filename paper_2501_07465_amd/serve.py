"""Serving: continuous batching of independent simulations on one GPU.

Requests (workload dicts with an ``arrival`` time in seconds and a step count) are admitted in
arrival order while a slot is free and the sum of the admitted simulations' device footprints
stays within the HBM budget.  Admitted simulations keep their particle and field state resident
in their own arenas and advance together: every sort period is one captured graph holding the
members' sorts and, per step, one particle launch and one field launch over the whole batch.
A request that has run its steps is retired (its diagnostics are read back) and its slot and
memory go to the next arrivals, while the others keep running.

Latency is arrival -> result read back; throughput is the particle-steps of all finished requests
over the span from the first arrival to the last result.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import pic


class Request:
    def __init__(self, rid: int, w: dict, arrival: float | None = None):
        self.rid = rid
        self.w = w
        self.arrival = float(w.get("arrival", 0.0) if arrival is None else arrival)
        self.steps = int(w["steps"])
        self.left = self.steps
        self.footprint = 0
        self.sim = None
        self.t_admit = None
        self.t_done = None
        self.particles = 0
        self.result = None
        self.error = None


class Server:
    """Admission by HBM footprint and slot count, continuous batching, per-request results."""

    def __init__(self, dims: int = 2, precision: str = "fp32", hbm_budget: int = 16 << 30, max_slots: int = 64,
                 block: int = 512, sort_every: int = 20, tile=None, max_ahead: int = 2, unit: int | None = None):
        self.dims = dims
        self.precision = precision
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.block = block
        self.period = sort_every
        self.tile = tile
        self.unit = unit
        self.max_ahead = max_ahead
        self.batch = self._make_batch(max_slots, dims, precision)
        self.used = 0
        self.active: list[Request] = []

    def _make_batch(self, max_slots, dims, precision):
        return pic.Batch(max_slots, dims, precision)

    def _prepare(self, r: Request):
        w = r.w
        if self.tile is not None:
            w["tile"] = list(self.tile) + [1] * (3 - len(self.tile))
        if w["dims"] != self.dims:
            raise ValueError("request dimensionality differs from the server's")
        if w.get("sort_every", 20) != self.period or r.steps % self.period:
            raise ValueError("request steps must be whole sort periods of the server")
        r.footprint = pic.footprint_of(w, self.precision, self.block, series_cap=r.steps + 64, unit=self.unit)

    def _admit(self, r: Request, now: float):
        r.sim = pic.Simulation(r.w, precision=self.precision, graphs=False, stream=self.batch.stream,
                               block=self.block, series_cap=r.steps + 64, unit=self.unit)
        r.particles = sum(r.sim.count(s) for s in r.sim.species)
        self.batch.add(r.sim)
        self.used += r.footprint
        r.t_admit = now
        self.active.append(r)

    def _retire(self, r: Request, t0: float):
        sim = r.sim
        self.batch.remove(sim)  # synchronizes the batch stream
        r.result = {
            "field_energy": sim.field_energy(),
            "kinetic_energy": [sim.kinetic_energy(s) for s in sim.species],
            "current_series": sim.current_series(),
            "steps": sim.steps_done,
        }
        r.t_done = time.perf_counter() - t0
        self.active.remove(r)
        self.used -= r.footprint
        r.sim = None
        del sim

    def _record(self):
        """An event after the work enqueued so far (bounds how far the host runs ahead)."""
        import torch
        ev = torch.cuda.Event()
        ev.record(self.batch.stream)
        return ev

    def run(self, requests: list[Request], log=None) -> dict:
        """Serve ``requests`` (arrival times relative to the call); returns latency and throughput."""
        for r in requests:
            self._prepare(r)
            if r.footprint > self.budget:
                r.error = f"footprint {r.footprint} exceeds the HBM budget"
        pending = collections.deque(sorted((r for r in requests if r.error is None), key=lambda r: r.arrival))
        inflight = collections.deque()
        t0 = time.perf_counter()
        while pending or self.active:
            now = time.perf_counter() - t0
            while (pending and pending[0].arrival <= now and len(self.active) < self.max_slots
                   and self.used + pending[0].footprint <= self.budget):
                self._admit(pending.popleft(), now)
                if log:
                    log(f"admit: {len(self.active)} active, {self.used / 2**30:.2f} GiB")
            if not self.active:
                time.sleep(max(0.0, min(0.05, pending[0].arrival - now)))
                continue
            self.batch.step(self.period)
            inflight.append(self._record())
            for r in self.active:
                r.left -= self.period
            done = [r for r in self.active if r.left <= 0]
            for r in done:
                self._retire(r, t0)
            if done:
                inflight.clear()
            while len(inflight) > self.max_ahead:
                inflight.popleft().synchronize()
        served = [r for r in requests if r.result is not None]
        lat = np.array([r.t_done - r.arrival for r in served]) if served else np.zeros(0)
        first = min((r.arrival for r in served), default=0.0)
        last = max((r.t_done for r in served), default=0.0)
        psteps = float(sum(r.particles * r.steps for r in served))
        span = max(last - first, 1e-9)
        return {
            "requests": len(served),
            "rejected": sum(1 for r in requests if r.error is not None),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "span_s": span,
            "particle_steps": psteps,
            "particle_steps_per_s": psteps / span,
        }


def run_alone(w: dict, precision: str = "fp32", block: int = 512) -> dict:
    """One request on its own (its own stream and graphs): the reference for the in-mix result."""
    sim = pic.Simulation(w, precision=precision, graphs=True, block=block, series_cap=int(w["steps"]) + 64)
    sim.step(int(w["steps"]))
    sim.sync()
    return {
        "field_energy": sim.field_energy(),
        "kinetic_energy": [sim.kinetic_energy(s) for s in sim.species],
        "current_series": sim.current_series(),
        "steps": sim.steps_done,
    }
