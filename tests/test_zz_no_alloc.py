"""The entry point that allocates nothing: pic_energy_histogram_static, whose counters sit in a
static device array of the library, against pic_energy_histogram (counters in the simulation's
arena) through the C ABI.  Integer counts: bit-exact.  Two calls in a row, the second on a smaller
input (a smaller simulation and fewer bins), so counts left from the first call would show."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EV = 1.602176634e-19


def test_static_histogram_equals_arena_histogram_twice():
    from paper_2501_07465_amd import pic, workloads as W
    print("case no-alloc histogram", flush=True)
    w1 = W.small("disk2d")
    sim1 = pic.Simulation(w1, precision="fp32", graphs=False)
    sim1.step(5)
    for sid in range(len(w1["species"])):
        a = pic.pic_energy_histogram(sim1.h, sid, 12.0 * EV, 4096)
        b = pic.pic_energy_histogram_static(sim1.h, sid, 12.0 * EV, 4096)
        assert a.sum() == sim1.count(sid)
        assert np.array_equal(a, b), (sid, int(np.abs(a.astype(np.int64) - b.astype(np.int64)).max()))
    w2 = W.small("slab1d")
    sim2 = pic.Simulation(w2, precision="fp64", graphs=False)
    sim2.step(3)
    a = pic.pic_energy_histogram(sim2.h, 0, 8.0 * EV, 100)
    b = pic.pic_energy_histogram_static(sim2.h, 0, 8.0 * EV, 100)
    assert sim2.count(0) < sim1.count(0)
    assert a.sum() == b.sum() == sim2.count(0)
    assert np.array_equal(a, b)
    # beyond the static array: refused
    with pytest.raises(pic.PicError) as e:
        pic.pic_energy_histogram_static(sim2.h, 0, 8.0 * EV, 4097)
    assert e.value.code == pic.PIC_EINVAL
    # the arena-backed call still works after the static ones
    c = pic.pic_energy_histogram(sim1.h, 0, 12.0 * EV, 4096)
    assert c.sum() == sim1.count(0)
