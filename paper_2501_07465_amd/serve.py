"""Serving: continuous batching of independent simulations on one GPU.

Requests (workload dicts with an ``arrival`` time in seconds and a step count) are admitted in
arrival order while a slot is free and the sum of the admitted simulations' device footprints
stays within the HBM budget.  Admitted simulations keep their particle and field state resident
in their own arenas and advance together in one batch of fixed slots: every sort period is the
members' sort graphs and one captured step graph (per step, one particle launch and one field
launch over all slots).  A request is built on a loading stream of its own (so building it never
waits for the batch), joins the batch between two periods, and leaves it after its last period:
its slot is free for the next arrival at once, while its diagnostics are read on a read-back stream
that waits only for its own last period (an event), after which its memory is released.

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
        self.counts = []
        self.result = None
        self.error = None
        self.done_event = None


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
        self.load_stream = self._make_stream()
        self.read_stream = self._make_stream()
        self.used = 0
        self.active: list[Request] = []
        self.leaving: collections.deque = collections.deque()

    def _make_batch(self, max_slots, dims, precision):
        return pic.Batch(max_slots, dims, precision)

    def _make_stream(self):
        import torch
        return torch.cuda.Stream()

    def _event_on(self, stream):
        """An event after the work enqueued on ``stream`` so far."""
        import torch
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

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
        # built (loaded, first fields) on the loading stream, then moved behind the batch's work
        r.sim = pic.Simulation(r.w, precision=self.precision, graphs=False, stream=self.load_stream,
                               block=self.block, series_cap=r.steps + 64, unit=self.unit)
        r.counts = [r.sim.count(s) for s in r.sim.species]
        r.particles = sum(r.counts)
        r.sim.set_stream(self.batch.stream)
        self.batch.add(r.sim)
        self.used += r.footprint
        r.t_admit = now
        self.active.append(r)

    def _leave(self, r: Request):
        """After its last period is enqueued: free the slot, move the read-back behind that period."""
        self.batch.remove(r.sim)
        r.sim.set_stream(self.read_stream)
        r.done_event = self._event_on(self.read_stream)
        self.active.remove(r)
        self.leaving.append(r)

    def _collect(self, r: Request, t0: float):
        sim = r.sim
        r.result = {
            "field_energy": sim.field_energy(),
            "kinetic_energy": [sim.kinetic_energy(s) for s in sim.species],
            "current_series": sim.current_series(),
            "steps": sim.steps_done,
        }
        r.t_done = time.perf_counter() - t0
        self.used -= r.footprint
        r.sim = None
        del sim

    def _collect_ready(self, t0: float, wait: bool = False):
        while self.leaving and (wait or self.leaving[0].done_event.query()):
            self._collect(self.leaving.popleft(), t0)
            wait = False

    def _record(self):
        """An event after the batch work enqueued so far (bounds how far the host runs ahead)."""
        return self._event_on(self.batch.stream)

    def run(self, requests: list[Request], log=None) -> dict:
        """Serve ``requests`` (arrival times relative to the call); returns latency and throughput."""
        for r in requests:
            self._prepare(r)
            if r.footprint > self.budget:
                r.error = f"footprint {r.footprint} exceeds the HBM budget"
        pending = collections.deque(sorted((r for r in requests if r.error is None), key=lambda r: r.arrival))
        inflight = collections.deque()
        captures0 = self.batch.captures
        t0 = time.perf_counter()
        while pending or self.active or self.leaving:
            now = time.perf_counter() - t0
            self._collect_ready(t0)
            while (pending and pending[0].arrival <= now and len(self.active) < self.max_slots
                   and self.used + pending[0].footprint <= self.budget):
                self._admit(pending.popleft(), now)
                if log:
                    log(f"admit: {len(self.active)} active, {self.used / 2**30:.2f} GiB")
            if not self.active:
                if self.leaving:
                    self._collect_ready(t0, wait=True)
                elif pending:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - now)))
                continue
            self.batch.step(self.period)
            inflight.append(self._record())
            for r in self.active:
                r.left -= self.period
            for r in [r for r in self.active if r.left <= 0]:
                self._leave(r)
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
            "graph_captures": self.batch.captures - captures0,
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
