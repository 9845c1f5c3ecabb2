"""Host logic of the serving loop (admission by footprint and slots, retirement, latency
accounting) with stand-ins for the device simulations: no GPU needed."""
import time

import pytest


class _FakeSim:
    live = 0
    peak = 0

    def __init__(self, w, **kw):
        self.w = w
        self.species = [0]
        self.done = 0
        _FakeSim.live += 1
        _FakeSim.peak = max(_FakeSim.peak, _FakeSim.live)

    def count(self, sid):
        return self.w["particles"]

    def set_stream(self, stream):
        self.stream = stream

    def field_energy(self):
        return float(self.w["seed"])

    def kinetic_energy(self, sid):
        return 1.0

    def current_series(self):
        return [[0.0, 0.0, 0.0]] * self.done

    @property
    def steps_done(self):
        return self.done

    def __del__(self):
        _FakeSim.live -= 1


class _FakeBatch:
    def __init__(self):
        self.members = []
        self.stream = "batch"
        self.max_members = 0
        self.captures = 0

    def add(self, s):
        self.members.append(s)
        self.max_members = max(self.max_members, len(self.members))

    def remove(self, s):
        self.members.remove(s)

    def step(self, k):
        time.sleep(0.001)
        for s in self.members:
            s.done += k


class _Ev:
    """Done after ``polls`` queries (a read-back that is not finished at once)."""
    polls = 0

    def __init__(self):
        self.left = _Ev.polls

    def query(self):
        self.left -= 1
        return self.left < 0

    def synchronize(self):
        self.left = -1


@pytest.fixture
def server(monkeypatch):
    from paper_2501_07465_amd import serve
    monkeypatch.setattr(serve.pic, "Simulation", _FakeSim)
    monkeypatch.setattr(serve.pic, "footprint_of", lambda w, *a, **k: w["fp"])
    monkeypatch.setattr(serve.Server, "_make_batch", lambda self, *a: _FakeBatch())
    monkeypatch.setattr(serve.Server, "_make_stream", lambda self: "side")
    monkeypatch.setattr(serve.Server, "_event_on", lambda self, st: _Ev())
    _FakeSim.live = _FakeSim.peak = 0
    _Ev.polls = 0
    return serve


def _req(serve, rid, fp, steps, arrival):
    w = {"dims": 2, "steps": steps, "sort_every": 20, "fp": fp, "particles": 100, "seed": rid}
    return serve.Request(rid, w, arrival=arrival)


def test_admission_respects_budget_and_slots(server):
    serve = server
    reqs = [_req(serve, i, fp=30, steps=40 + 20 * (i % 3), arrival=0.0) for i in range(8)]
    srv = serve.Server(dims=2, hbm_budget=100, max_slots=5, tile=None)
    stats = srv.run(reqs)
    assert stats["requests"] == 8 and stats["rejected"] == 0
    # 100 / 30 -> at most three resident at once, below the slot cap of five
    assert srv.batch.max_members == 3
    for r in reqs:
        assert r.result["steps"] == r.steps
        assert r.result["field_energy"] == float(r.rid)
        assert r.t_done >= r.arrival and r.t_admit is not None
    assert srv.used == 0 and not srv.active
    assert stats["particle_steps"] == sum(100 * r.steps for r in reqs)


def test_slot_cap_and_arrival_order(server):
    serve = server
    reqs = [_req(serve, i, fp=1, steps=20, arrival=0.0) for i in range(6)]
    srv = serve.Server(dims=2, hbm_budget=10**9, max_slots=2)
    srv.run(reqs)
    assert srv.batch.max_members == 2
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)


def test_oversized_request_is_rejected_not_blocking(server):
    serve = server
    reqs = [_req(serve, 0, fp=500, steps=20, arrival=0.0), _req(serve, 1, fp=10, steps=20, arrival=0.0)]
    srv = serve.Server(dims=2, hbm_budget=100, max_slots=4)
    stats = srv.run(reqs)
    assert stats["rejected"] == 1 and stats["requests"] == 1
    assert reqs[0].error and reqs[1].result is not None


def test_later_arrivals_wait_for_their_time(server):
    serve = server
    reqs = [_req(serve, 0, fp=1, steps=20, arrival=0.0), _req(serve, 1, fp=1, steps=20, arrival=0.05)]
    srv = serve.Server(dims=2, hbm_budget=100, max_slots=4)
    srv.run(reqs)
    assert reqs[1].t_admit >= 0.05


def test_steps_must_be_whole_periods(server):
    serve = server
    srv = serve.Server(dims=2, hbm_budget=100, max_slots=4)
    with pytest.raises(ValueError):
        srv.run([_req(serve, 0, fp=1, steps=30, arrival=0.0)])


def test_slot_is_reused_before_the_read_back_finishes(server):
    """A request leaves the batch after its last period; the next one takes the slot at once, while
    the finished one is collected (and its memory released) only once its read-back event is done."""
    serve = server
    _Ev.polls = 3
    reqs = [_req(serve, i, fp=1, steps=20, arrival=0.0) for i in range(4)]
    srv = serve.Server(dims=2, hbm_budget=10**9, max_slots=1)
    stats = srv.run(reqs)
    assert stats["requests"] == 4 and srv.batch.max_members == 1
    # request k + 1 joined before request k was collected
    for a, b in zip(reqs, reqs[1:]):
        assert b.t_admit <= a.t_done
    assert all(r.sim is None for r in reqs) and srv.used == 0 and not srv.leaving
    assert stats["graph_captures"] == 0
