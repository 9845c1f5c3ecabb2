"""Pins of the oracle's diffusive scattering at the material boundary (Sec. 3 names specular and
diffusive models; the reading taken: elastic, position mirrored as in the specular case, direction
from the cosine (Lambert) law about the inward normal at the escaped point).

* Philox4x32-10 reproduces the published known-answer vectors (tests/golden), and the scatter
  uniforms are Philox output turned into 53-bit uniforms in (0, 1).
* The cosine law, independent of the tangent basis: for any inward normal n the draws have unit
  length times |v|, d.n > 0, (d.n)^2 uniform on (0, 1), <d.n> = 2/3, and zero mean with variance
  1/4 along any tangent.
* In a run, every particle that crossed the wall keeps its speed and leaves with d.n > 0; the
  others are untouched; particles stay in the region; diffuse walls randomise the direction of a
  beam that specular walls keep ordered.
* Diffusive scattering is refused for bound species and for Dirac species without a sheet.
"""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
QE = 1.602176634e-19
ME = 9.1093837015e-31


def test_philox_known_answers(oracle):
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    assert len(rows) >= 3
    for r in rows:
        got = oracle.philox(r[0:4], r[4:6])
        assert list(got) == r[6:10]


def test_scatter_uniforms_are_philox_uniforms(oracle):
    seed = 0x1234_5678_9ABC_DEF0
    for p, step, sid in [(0, 0, 0), (17, 5, 1), (2**31 - 1, 123456, 3)]:
        u = oracle.scatter_uniforms(seed, p, step, sid)
        r = oracle.philox([p, step, sid, 0x80000000], [seed & 0xFFFFFFFF, seed >> 32])
        assert u[0] == oracle.u53(r[0], r[1]) and u[1] == oracle.u53(r[2], r[3])
        assert 0.0 < u[0] < 1.0 and 0.0 < u[1] < 1.0
    us = np.array([oracle.scatter_uniforms(7, p, 3, 0) for p in range(4000)])
    assert abs(us.mean() - 0.5) < 5 * math.sqrt(1 / 12 / us.size)


@pytest.mark.parametrize("n", [[1, 0, 0], [0, -1, 0], [0.6, -0.8, 0.0], [1 / 3, 2 / 3, -2 / 3]])
def test_cosine_law_moments(oracle, n):
    n = np.array(n, dtype=float)
    n /= np.linalg.norm(n)
    rng = np.random.default_rng(11)
    N = 20000
    speed = 1.3e6
    v0 = np.array([speed, 0.0, 0.0])
    D = np.empty((N, 3))
    for i in range(N):
        D[i] = oracle.lambert(n, rng.uniform(0, 1, 2), v0)
    assert np.max(np.abs(np.linalg.norm(D, axis=1) / speed - 1)) < 1e-14
    d = D / speed
    c = d @ n
    assert np.all(c > 0)
    # cos^2 theta is uniform on (0, 1): mean 1/2, variance 1/12, and a flat histogram
    c2 = c * c
    assert abs(c2.mean() - 0.5) < 5 * math.sqrt(1 / 12 / N)
    assert abs(c.mean() - 2 / 3) < 5 * math.sqrt(1 / 18 / N)
    h, _ = np.histogram(c2, bins=10, range=(0, 1))
    assert np.all(np.abs(h - N / 10) < 5 * math.sqrt(N / 10))
    # along any two orthogonal tangents: zero mean, variance (1 - 1/2) / 2
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    t1 = a - (a @ n) * n
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    for t in (t1, t2, (t1 + t2) / math.sqrt(2)):
        s = d @ t
        assert abs(s.mean()) < 5 * math.sqrt(0.25 / N)
        assert abs((s * s).mean() - 0.25) < 5 * math.sqrt(0.125 / N)


def _ring_state(n_part, radius, center, speed, seed):
    """Particles just inside a circle, moving outward (each crosses the wall within a step)."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0, 2 * math.pi, n_part)
    r = radius - rng.uniform(0.01, 0.2, n_part)
    X = np.zeros((n_part, 3))
    X[:, 0] = center[0] + r * np.cos(ang)
    X[:, 1] = center[1] + r * np.sin(ang)
    out = np.stack([np.cos(ang), np.sin(ang), np.zeros(n_part)], axis=1)
    tang = np.stack([-np.sin(ang), np.cos(ang), np.zeros(n_part)], axis=1)
    mix = rng.uniform(-0.5, 0.5, (n_part, 1))
    v = out + mix * tang + rng.uniform(-0.3, 0.3, (n_part, 1)) * np.array([0, 0, 1.0])
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * speed
    return X, v


def _disk_world(scatter):
    from paper_2501_07465_amd import workloads as W
    dx = 1e-9
    w = {"name": "walls", "dims": 2, "n": [32, 32, 1], "dx": [dx] * 3, "dt": W.cfl_dt(dx, 2),
         "periodic": [1, 1, 1], "tile": [8, 8, 1], "sort_every": 20, "species": [], "seed": 9}
    sp = {"kind": "free", "q": -QE * 1e-12, "m": ME, "reflect": True, "scatter": scatter,
          "region": {"kind": "ball", "center": [16.0, 16.0, 0.0], "radius": 10.0}}
    w["species"] = [sp]
    return w, sp


def test_diffuse_wall_one_step_properties(oracle):
    w, sp = _disk_world("diffuse")
    dx = w["dx"][0]
    # speed such that one step moves about 0.3 cell: every particle crosses the wall
    speed = 0.3 * dx / w["dt"]
    X, v = _ring_state(500, 10.0, [16.0, 16.0], speed, 3)
    s = oracle.Sim(w)
    s.add_species(sp, 1.0, X * dx, v)
    x0, v0, _ = s.particles(0)
    s.step(1)
    x1, v1, _ = s.particles(0)
    # particles are matched by position (the sort at step 0 may reorder them)
    order0 = np.lexsort((x0[:, 1], x0[:, 0]))
    Xs = x0[order0] / dx
    vs = v0[order0]
    # each particle's escaped point is start + dt v (tiny q: no field kick)
    esc = Xs + vs * w["dt"] / dx
    r_esc = np.hypot(esc[:, 0] - 16.0, esc[:, 1] - 16.0)
    crossed = r_esc > 10.0
    assert crossed.sum() > 400
    # locate each particle after the step by its mirrored end point
    nin = np.zeros((len(Xs), 3))
    nin[:, 0] = 16.0 - esc[:, 0]
    nin[:, 1] = 16.0 - esc[:, 1]
    nin /= np.linalg.norm(nin, axis=1, keepdims=True)
    mirrored = esc.copy()
    mirrored[:, :2] = 16.0 + ((2 * 10.0 - r_esc) / r_esc)[:, None] * (esc[:, :2] - 16.0)
    end = np.where(crossed[:, None], mirrored, esc)
    # match by end position (unique to round-off)
    x1c = x1 / dx
    idx = [int(np.argmin(np.sum((x1c[:, :2] - e[:2]) ** 2, axis=1))) for e in end]
    assert len(set(idx)) == len(idx)
    assert np.max(np.abs(x1c[idx, :2] - end[:, :2])) < 1e-9
    vn = v1[idx]
    assert np.max(np.abs(np.linalg.norm(vn, axis=1) / speed - 1)) < 1e-9
    assert np.all(np.sum(vn[crossed] * nin[crossed], axis=1) > 0)
    if (~crossed).any():
        assert np.max(np.abs(vn[~crossed] - vs[~crossed])) <= 1e-9 * speed
    # the outgoing directions are not the specular ones
    spec = vs - 2 * np.sum(vs * -nin, axis=1, keepdims=True) * -nin
    assert np.mean(np.abs(vn[crossed] - spec[crossed])) > 0.1 * speed


@pytest.mark.parametrize("scatter", ["specular", "diffuse"])
def test_walls_confine_and_diffuse_walls_randomise_a_beam(oracle, scatter):
    w, sp = _disk_world(scatter)
    dx = w["dx"][0]
    rng = np.random.default_rng(4)
    N = 400
    r = 8.0 * np.sqrt(rng.uniform(0, 1, N))
    a = rng.uniform(0, 2 * math.pi, N)
    X = np.stack([16 + r * np.cos(a), 16 + r * np.sin(a), np.zeros(N)], axis=1)
    speed = 0.4 * dx / w["dt"]
    v = np.tile([speed, 0.0, 0.0], (N, 1))  # a beam along x
    s = oracle.Sim(w)
    s.add_species(sp, 1.0, X * dx, v)
    s.step(300)
    x1, v1, _ = s.particles(0)
    rr = np.hypot(x1[:, 0] / dx - 16, x1[:, 1] / dx - 16)
    assert np.all(rr <= 10.0 + 1e-9)
    assert np.max(np.abs(np.linalg.norm(v1, axis=1) / speed - 1)) < 1e-9
    if scatter == "specular":
        # a specular circle keeps every velocity in the plane (v_z = 0)
        assert np.max(np.abs(v1[:, 2])) < 1e-9 * speed
    else:
        # diffuse walls give out-of-plane velocities and spread the directions
        assert np.mean(np.abs(v1[:, 2])) > 0.2 * speed
        assert abs(np.mean(v1[:, 0])) < 0.2 * speed


def test_diffuse_refused_for_bound_and_sheetless_dirac(oracle):
    w, sp = _disk_world("diffuse")
    s = oracle.Sim(w)
    for kind, extra in (("bound", {"omega0": [1e15] * 3, "gamma": [1e13] * 3}),
                        ("dirac", {"v_f": 1e6, "sheet_normal": -1, "m": 1e-32})):
        bad = dict(sp, kind=kind, **extra)
        with pytest.raises(RuntimeError):
            s.add_species(bad, 1.0, np.array([[16e-9, 16e-9, 0.0]]), np.array([[1e5, 0.0, 0.0]]),
                          xi=np.zeros((1, 3)) if kind == "bound" else None)
