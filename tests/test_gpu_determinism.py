"""Bit-identical replays.

The current is accumulated as exact integer multiples of a quantum (FP64 words holding integers
below 2^53), so its sums do not depend on the order in which wavefronts, work units or batch
members add them.  Every other kernel is free of order-dependent arithmetic.  Hence:
* the same run twice gives bit-identical particles and fields;
* the captured-graph path equals plain launches bit for bit;
* a simulation run as a member of a batch equals the same simulation run alone, bit for bit.
In both forms (FP32 and FP64).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _small(name, precision):
    from paper_2501_07465_amd import workloads as W
    w = W.small(name)
    if name == "sphere3d" and precision == "fp64":
        w["tile"] = [4, 4, 4]
    return w


def _state(sim, w):
    out = []
    for sid in range(len(w["species"])):
        out.extend(sim.particles(sid))
    out.extend(sim.fields())
    out.append(sim.current_series())
    return out


def _same(a, b, label):
    for i, (x, y) in enumerate(zip(a, b)):
        assert x.shape == y.shape, (label, i)
        assert np.array_equal(x, y), (label, i, float(np.max(np.abs(x - y))))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["disk2d", "sheet2d", "sphere3d", "slab1d"])
def test_replay_and_graphs_bit_identical(name, precision):
    from paper_2501_07465_amd import pic
    w = _small(name, precision)
    print(f"case replay {name} {precision}", flush=True)
    runs = []
    for graphs in (True, True, False):
        sim = pic.Simulation(w, precision=precision, graphs=graphs)
        sim.step(60)
        runs.append(_state(sim, w))
        del sim
    _same(runs[0], runs[1], f"{name} {precision} replay")
    _same(runs[0], runs[2], f"{name} {precision} graphs vs plain")


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_member_equals_alone_bit_for_bit(precision):
    import torch
    from paper_2501_07465_amd import pic, workloads as W
    print(f"case batch bit-identical {precision}", flush=True)
    ws = [W.stream_request(j, scale=0.12) for j in (3, 8, 11)]
    for w in ws:
        w["steps"] = 60
    alone = []
    for w in ws:
        sim = pic.Simulation(w, precision=precision, graphs=True)
        sim.step(60)
        alone.append(_state(sim, w))
        del sim
    stream = torch.cuda.Stream()
    b = pic.Batch(4, 2, precision, stream=stream)
    sims = [pic.Simulation(w, precision=precision, graphs=True, stream=stream) for w in ws]
    b.add(sims[0])
    b.add(sims[1])
    b.step(20)
    b.add(sims[2])  # joins two periods behind the others
    b.step(40)
    b.remove(sims[0])
    b.remove(sims[1])
    b.step(20)
    for i, (w, sim) in enumerate(zip(ws, sims)):
        _same(_state(sim, w), alone[i], f"batch member {i} {precision}")
