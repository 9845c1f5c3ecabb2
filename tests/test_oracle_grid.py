"""Pins of the oracle's grid arithmetic: deposit, gather and the Yee update.

* Continuity (rho^{n+1} - rho^n)/dt + div J = 0 to round-off, with rho built
  here by an independent numpy cloud-in-cell deposit, over enumerated moves
  that cross faces and corners (1D, 2D, 3D, unequal cell sizes).
* The summed current of each component equals sum q w v (pins the
  prefactors of the components without a divergence, e.g. J_z in 2D).
* Gather of a linear field is exact.
* The Yee update reproduces the vacuum lattice dispersion relation of
  Sec. 4.1 (the left bracket of eq:numdispersion set to zero).
* Open faces absorb an outgoing pulse; Gauss's law is kept to round-off.
"""
import itertools
import math

import numpy as np
import pytest

QE = 1.602176634e-19
ME = 9.1093837015e-31
C = 299792458.0
EPS0 = 8.8541878128e-12


def grid(dims, n, dx, dt, periodic=(1, 1, 1), tile=None):
    n = list(n) + [1] * (3 - len(n))
    dx = list(dx) + [dx[-1]] * (3 - len(dx))
    return {"dims": dims, "n": n, "dx": dx, "dt": dt, "periodic": list(periodic),
            "tile": tile or [max(1, v // 2) for v in n], "sort_every": 1, "species": []}


def cic_rho(X, qw, w, L):
    """Independent nodal CIC charge density (periodic), X in cell units [N,3]."""
    dims = w["dims"]
    dv = np.prod(w["dx"][:dims])
    rho = np.zeros((L[2], L[1], L[0]))
    for p in range(X.shape[0]):
        base = np.floor(X[p, :dims]).astype(int)
        frac = X[p, :dims] - base
        for corner in itertools.product((0, 1), repeat=dims):
            wgt = 1.0
            idx = [0, 0, 0]
            for a in range(dims):
                wgt *= frac[a] if corner[a] else 1.0 - frac[a]
                idx[a] = (base[a] + corner[a]) % w["n"][a]
            rho[idx[2], idx[1], idx[0]] += qw * wgt / dv
    return rho


def div_periodic(J, w):
    dims = w["dims"]
    out = np.zeros(J.shape[1:])
    for a in range(dims):
        ax = 2 - a  # arrays are [z, y, x]
        out += (J[a] - np.roll(J[a], 1, axis=ax)) / w["dx"][a]
    return out


def enumerated_moves(dims):
    starts = [0.03, 0.5, 0.97]
    moves = [-0.9, -0.06, 0.0, 0.06, 0.9]
    X0, D = [], []
    for s in itertools.product(starts, repeat=dims):
        for m in itertools.product(moves, repeat=dims):
            X0.append(list(s) + [0.0] * (3 - dims))
            D.append(list(m) + [0.0] * (3 - dims))
    return np.array(X0), np.array(D)


@pytest.mark.parametrize("dims,n,dx", [(1, [7], [0.5e-9]),
                                       (2, [6, 5], [1e-9, 0.7e-9]),
                                       (3, [4, 5, 3], [1e-9, 0.8e-9, 1.3e-9])])
def test_esirkepov_continuity_and_total_current(oracle, dims, n, dx):
    dt = 1e-18
    w = grid(dims, n, dx, dt)
    X0, D = enumerated_moves(dims)
    rng = np.random.default_rng(dims)
    cells = np.zeros_like(X0)
    for a in range(dims):
        cells[:, a] = rng.integers(0, n[a], size=X0.shape[0])
    X0 = X0 + cells
    dxv = np.array(w["dx"])
    x0 = X0 * dxv
    v = D * dxv / dt
    v[:, dims:] = rng.normal(size=(X0.shape[0], 3 - dims)) * 1e5  # invariant-axis velocity
    s = oracle.Sim(w)
    weight = 1.0e3
    s.add_species({"kind": "free", "q": -QE, "m": ME}, weight, x0, v)
    s.step(1)
    J = s.current()
    L = s.shape()
    x1, v1, _ = s.particles(0)
    X1 = x1 / dxv
    qw = -QE * weight
    rho0 = cic_rho(X0, qw, w, L)
    rho1 = cic_rho(X1, qw, w, L)
    res = (rho1 - rho0) / dt + div_periodic(J, w)
    scale = np.max(np.abs(rho0)) / dt
    assert np.max(np.abs(res)) <= 1e-13 * scale
    # total current per component: sum_cells J dV = sum_p q w dX dx / dt (moving axes), q w v (invariant)
    dv = np.prod(w["dx"][:dims])
    for a in range(3):
        total = J[a].sum() * dv
        if a < dims:
            expect = qw * np.sum(D[:, a]) * dxv[a] / dt
        else:
            expect = qw * np.sum(v[:, a])
        assert abs(total - expect) <= 1e-12 * (abs(qw) * np.sum(np.abs(v[:, a])) + 1e-300)
    # every single particle conserves charge on its own too (corner crossings)
    for p in rng.choice(X0.shape[0], size=min(12, X0.shape[0]), replace=False):
        s1 = oracle.Sim(w)
        s1.add_species({"kind": "free", "q": -QE, "m": ME}, weight, x0[p:p + 1], v[p:p + 1])
        s1.step(1)
        J1 = s1.current()
        xe, _, _ = s1.particles(0)
        r = (cic_rho(xe / dxv, qw, w, L) - cic_rho(X0[p:p + 1], qw, w, L)) / dt + div_periodic(J1, w)
        assert np.max(np.abs(r)) <= 1e-13 * np.max(np.abs(cic_rho(X0[p:p + 1], qw, w, L))) / dt


def test_continuity_tracker_agrees(oracle):
    # the oracle's own per-step continuity residual is at round-off on a thermal 2D plasma
    from paper_2501_07465_amd import workloads as W
    w = W.small("disk2d")
    s = oracle.build_workload(w)
    s.track_continuity(True)
    s.step(3)
    r, sc = s.continuity_residual()
    assert r <= 1e-12 * sc


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_gather_linear_field_exact(oracle, dims):
    n = [9, 8, 7][:dims]
    dx = [1e-9, 0.6e-9, 1.4e-9][:dims]
    w = grid(dims, n, dx, 1e-18, periodic=(0, 0, 0))
    s = oracle.Sim(w)
    L = s.shape()
    rng = np.random.default_rng(10 + dims)
    coef = rng.normal(size=(6, 4))
    e = np.zeros((3, L[2], L[1], L[0])); b = np.zeros_like(e)
    kk, jj, ii = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    pos = [ii.astype(float), jj.astype(float), kk.astype(float)]
    for c in range(3):
        hE = [1.0 if a == c else 0.0 for a in range(3)]
        hB = [0.0 if a == c else 1.0 for a in range(3)]
        e[c] = coef[c, 0] + sum(coef[c, 1 + a] * (pos[a] + 0.5 * hE[a]) for a in range(dims))
        b[c] = coef[3 + c, 0] + sum(coef[3 + c, 1 + a] * (pos[a] + 0.5 * hB[a]) for a in range(dims))
    s.set_fields(e, b)
    for _ in range(50):
        X = np.zeros(3)
        X[:dims] = rng.uniform(1.5, np.array(n) - 1.5)
        E, B = s.gather_at(X * np.array(w["dx"]))
        for c in range(3):
            ee = coef[c, 0] + sum(coef[c, 1 + a] * X[a] for a in range(dims))
            bb = coef[3 + c, 0] + sum(coef[3 + c, 1 + a] * X[a] for a in range(dims))
            assert abs(E[c] - ee) < 1e-13 * (1 + abs(ee))
            assert abs(B[c] - bb) < 1e-13 * (1 + abs(bb))


def _plane_wave(dims, n, dx, dt, m):
    """Discrete Yee eigenmode with E polarised along z (2D/3D) or y (1D), k in the x-y plane."""
    k = [2 * math.pi * m[a] / (n[a] * dx[a]) if a < dims else 0.0 for a in range(3)]
    s2 = sum((math.sin(k[a] * dx[a] / 2) / dx[a]) ** 2 for a in range(min(dims, 2)))
    om = 2.0 / dt * math.asin(C * dt * math.sqrt(s2))
    wdt = math.sin(om * dt / 2) / dt
    return k, om, wdt


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_yee_vacuum_dispersion(oracle, dims):
    n = {1: [64, 1, 1], 2: [32, 24, 1], 3: [16, 12, 6]}[dims]
    dx = {1: [1e-9] * 3, 2: [1e-9, 0.8e-9, 1e-9], 3: [1e-9, 0.8e-9, 1.1e-9]}[dims]
    dt = 0.9 / (C * math.sqrt(sum(1 / dx[a] ** 2 for a in range(dims))))
    m = [3, 2, 0]
    k, om, wdt = _plane_wave(dims, n, dx, dt, m)
    w = grid(dims, n[:dims], dx[:dims], dt)
    s = oracle.Sim(w)
    L = s.shape()
    kk, jj, ii = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    X = ii * dx[0]; Y = jj * dx[1]; Z = kk * dx[2]
    e = np.zeros((3, L[2], L[1], L[0])); b = np.zeros_like(e)
    cw = math.cos(om * dt / 2)
    if dims == 1:
        e[1] = np.cos(k[0] * X)
        b[2] = (math.sin(k[0] * dx[0] / 2) / dx[0]) / wdt * cw * np.cos(k[0] * (X + dx[0] / 2))
    else:
        e[2] = np.cos(k[0] * X + k[1] * Y)
        bx0 = (math.sin(k[1] * dx[1] / 2) / dx[1]) / wdt
        by0 = -(math.sin(k[0] * dx[0] / 2) / dx[0]) / wdt
        b[0] = bx0 * cw * np.cos(k[0] * X + k[1] * (Y + dx[1] / 2))
        b[1] = by0 * cw * np.cos(k[0] * (X + dx[0] / 2) + k[1] * Y)
    s.set_fields(e, b)
    nsteps = 400
    s.step(nsteps)
    e1, _ = s.fields()
    t = nsteps * dt
    comp = 1 if dims == 1 else 2
    expect = np.cos(k[0] * X + k[1] * Y - om * t)
    assert np.max(np.abs(e1[comp] - expect)) < 1e-10
    # discrete energy stays bounded (no growth)
    assert abs(s.field_energy()) > 0


def test_mur_absorbs_outgoing_pulse(oracle):
    n = 400
    dx = 1e-9
    dt = 0.95 * dx / C
    w = grid(1, [n], [dx], dt, periodic=(0, 1, 1))
    s = oracle.Sim(w)
    L = s.shape()
    x = np.arange(L[0]) * dx
    e = np.zeros((3, 1, 1, L[0])); b = np.zeros_like(e)
    e[1, 0, 0] = np.exp(-((x - 200 * dx) / (12 * dx)) ** 2)
    s.set_fields(e, b)
    u0 = s.field_energy()
    s.step(int(1.4 * n * dx / (C * dt)))
    assert s.field_energy() < 2e-3 * u0


def test_gauss_law_kept_1d(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("slab1d")
    s = oracle.build_workload(w)
    r0, sc = s.gauss_residual()
    assert r0 <= 1e-12 * sc
    s.step(60)
    r1, sc1 = s.gauss_residual()
    assert r1 <= 1e-12 * sc1


def test_gauss_law_kept_2d_with_reflection_and_source(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("disk2d")
    w["steps"] = 30
    s = oracle.build_workload(w)
    r0, sc = s.gauss_residual()
    assert r0 <= 1e-12 * sc
    s.step(30)
    r1, sc1 = s.gauss_residual()
    assert r1 <= 1e-11 * sc1


@pytest.mark.parametrize("dims", [1, 2])
def test_invariant_axis_current_is_time_averaged_shape(oracle, dims):
    # For a move inside one cell the first-order weights are linear in time along the path,
    # so the current along an invariant axis is q w v times the exact time average of the
    # shape product, which Simpson's rule integrates exactly (the product is quadratic in t).
    n = [6, 5][:dims]
    dx = [1e-9, 0.7e-9][:dims]
    dt = 1e-18
    w = grid(dims, n, dx, dt)
    rng = np.random.default_rng(20 + dims)
    dxv = np.array(w["dx"])
    for _ in range(20):
        X0 = np.zeros(3); X1 = np.zeros(3)
        X0[:dims] = rng.integers(0, n) + rng.uniform(0.05, 0.95, size=dims)
        X1[:dims] = np.floor(X0[:dims]) + rng.uniform(0.05, 0.95, size=dims)
        v = np.zeros(3)
        v[:dims] = (X1 - X0)[:dims] * dxv[:dims] / dt
        v[dims:] = rng.normal(size=3 - dims) * 1e5
        s = oracle.Sim(w)
        s.add_species({"kind": "free", "q": -QE, "m": ME}, 1.0, (X0 * dxv)[None, :], v[None, :])
        s.step(1)
        J = s.current()
        L = s.shape()
        qw = -QE
        dv = np.prod(dxv[:dims])
        mid = 0.5 * (X0 + X1)
        avg = (cic_rho(X0[None, :], 1.0, w, L) + 4 * cic_rho(mid[None, :], 1.0, w, L)
               + cic_rho(X1[None, :], 1.0, w, L)) / 6.0 * dv
        for a in range(dims, 3):
            expect = qw * v[a] * avg / dv
            assert np.max(np.abs(J[a] - expect)) <= 1e-13 * np.max(np.abs(expect))


def test_sheet_source_radiates_closed_form_amplitude(oracle):
    """A soft current sheet J(t) on one node radiates E = -J dx / (2 eps0 c) each way (the plane-wave
    solution of the curl equations with a surface current J dx); the 1D vacuum run reproduces it,
    retarded by the travel time, to the Yee dispersion error (about 1e-5 at 800 cells per
    wavelength)."""
    from paper_2501_07465_amd import workloads as W
    dx = 1e-9
    dt = W.cfl_dt(dx, 1)
    e0 = 1e9
    src = W._source("sheet", 1, 0, [150, 0, 0], e0, wavelength=800e-9, dx=dx)
    w = {"name": "sheet_source_1d", "dims": 1, "n": [400, 1, 1], "dx": [dx, dx, dx], "dt": dt,
         "periodic": [0, 1, 1], "tile": [64, 1, 1], "sort_every": 20, "species": [], "source": src,
         "ion": "uniform", "steps": 0}
    sim = oracle.Sim(w)
    probe = 150 + 100
    eps0, c = oracle.const(3), oracle.const(2)
    nsteps = int(src["tau"] / dt) + 200
    got, want = [], []
    for n in range(nsteps):
        sim.step(1)
        e, _ = sim.fields()
        got.append(e[1, 0, 0, probe])
        # E_y^{n+1} is the field at t_{n+1}: the sheet current retarded by the travel time
        t = (n + 1) * dt - 100 * dx / c
        env = np.sin(np.pi * t / src["tau"]) ** 2 if 0.0 <= t <= src["tau"] else 0.0
        want.append(-src["j0"] * env * np.sin(src["omega"] * t) * dx / (2.0 * eps0 * c))
    got, want = np.array(got), np.array(want)
    assert np.max(np.abs(want)) > 0.5 * e0
    assert abs(np.max(np.abs(got)) / np.max(np.abs(want)) - 1.0) < 1e-4
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-4
