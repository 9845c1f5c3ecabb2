"""Pins of the oracle's static external (work-function) field (Sec. 3: an electrostatic barrier
outside the Maxwell solve, gathered like E).

* A uniform external field accelerates a particle at rest by exactly (q/m) E dt per step (the
  Boris push with B = 0), and leaves the Maxwell fields alone.
* A barrier of height W turns back an electron with kinetic energy K < W at its own speed, and
  lets one with K > W through with K - W left (energy conservation across the ramp).
* The input field of the barrier is a discrete gradient: its discrete curl vanishes, it is zero
  inside the region, and summing it along a path out of the region gives the barrier height.
"""
import math

import numpy as np
import pytest

QE = 1.602176634e-19
ME = 9.1093837015e-31
C = 299792458.0


def _grid1d(n, dx, periodic=1):
    from paper_2501_07465_amd import workloads as W
    return {"name": "wall1d", "dims": 1, "n": [n, 1, 1], "dx": [dx] * 3, "dt": W.cfl_dt(dx, 1),
            "periodic": [periodic, 1, 1], "tile": [16, 1, 1], "sort_every": 20, "species": [], "seed": 3}


def test_uniform_external_field_accelerates_exactly(oracle):
    w = _grid1d(64, 1e-9)
    s = oracle.Sim(w)
    L = s.shape()
    e = np.zeros((3, L[2], L[1], L[0]))
    E0 = np.array([2.0e8, -1.0e8, 5.0e7])
    for c in range(3):
        e[c] = E0[c]
    s.set_ext_field(e)
    sp = {"kind": "free", "q": -QE, "m": ME, "reflect": False}
    # a macroparticle of negligible weight: its own field is ~1e-9 of a single electron's
    s.add_species(sp, 1e-9, np.array([[20.3e-9, 0, 0]]), np.zeros((1, 3)))
    n = 50
    s.step(n)
    _, v, _ = s.particles(0)
    want = n * (-QE / ME) * E0 * w["dt"]
    np.testing.assert_allclose(v[0], want, rtol=1e-9)
    eg, bg = s.fields()
    assert np.max(np.abs(eg)) < 1e-6 * np.max(np.abs(E0))


def test_external_field_stays_out_of_maxwell(oracle):
    w = _grid1d(64, 1e-9)
    s = oracle.Sim(w)
    L = s.shape()
    e = np.random.default_rng(1).normal(size=(3, L[2], L[1], L[0])) * 1e9
    s.set_ext_field(e)
    s.step(40)
    eg, bg = s.fields()
    assert not np.any(eg) and not np.any(bg)
    assert s.field_energy() == 0.0


def _wall_world(height_ev=2.0, width=4.0):
    from paper_2501_07465_amd import workloads as W
    w = _grid1d(240, 1e-9)
    slab = {"kind": "box", "lo": [60.0, 0.0, 0.0], "hi": [160.0, 1.0, 1.0]}
    w["species"] = [{"kind": "free", "q": -QE, "m": ME, "reflect": False, "region": slab}]
    return W.with_potential_wall(w, height_ev, width, slab)


@pytest.mark.parametrize("k_ev", [1.0, 3.0])
def test_barrier_turns_back_or_passes_with_energy_conserved(oracle, k_ev):
    from paper_2501_07465_amd import workloads as W
    height = 2.0
    w = _wall_world(height)
    s = oracle.Sim(w)
    s.set_ext_field(W.wall_field(w))
    speed = math.sqrt(2 * k_ev * QE / ME)
    s.add_species(w["species"][0], 1e-9, np.array([[150.0e-9, 0, 0]]), np.array([[speed, 0.0, 0.0]]))
    # enough steps to cross 10 + 4 cells of ramp and 8 more cells at the lowest speed involved
    steps = int(24e-9 / (math.sqrt(2 * abs(k_ev - height) * QE / ME) * w["dt"]))
    s.step(steps)
    x, v, _ = s.particles(0)
    X = x[0, 0] / 1e-9
    K = 0.5 * ME * np.sum(v[0] ** 2) / QE
    if k_ev < height:
        # turned back: moving left, inside the slab, with its initial energy
        assert v[0, 0] < 0 and 60.0 < X < 160.0
        assert abs(K / k_ev - 1) < 1e-3
    else:
        # over the barrier: beyond the ramp (x in (164, 240)), with K - W left
        assert v[0, 0] > 0 and 164.0 < X < 240.0
        assert abs(K / (k_ev - height) - 1) < 1e-3


def test_wall_field_is_a_discrete_gradient():
    from paper_2501_07465_amd import workloads as W
    w = W.with_potential_wall(W.small("disk2d"), 4.5, 3.0)
    e = W.wall_field(w)
    dx, dy = w["dx"][0], w["dx"][1]
    # discrete curl (z component) of (E_x, E_y) on the periodic grid vanishes
    ex, ey = e[0, 0], e[1, 0]
    curl = (np.roll(ey, -1, axis=1) - ey) / dx - (np.roll(ex, -1, axis=0) - ex) / dy
    assert np.max(np.abs(curl)) <= 1e-9 * np.max(np.abs(ex)) / dx
    # zero inside the disk, and the barrier height along a ray out of it
    reg = w["wall"]["region"]
    cx, cy = reg["center"][0], reg["center"][1]
    i0, j0 = int(math.ceil(cx)), int(round(cy))
    assert abs(ex[j0, i0]) == 0.0
    # -sum E_x dx along +x from the centre to past the ramp = phi(end) - phi(start) = -height
    i1 = int(cx + reg["radius"] + 3.0 + 2)
    drop = -np.sum(ex[j0, i0:i1]) * dx
    phi = lambda i: -4.5 * min(max((math.hypot(i - cx, j0 - cy) - reg["radius"]) / 3.0, 0.0), 1.0)
    assert abs(drop - (phi(i1) - phi(i0))) < 1e-12 and abs(phi(i1) + 4.5) < 1e-12
