"""Pins of the oracle's FP64 diagnostics against closed forms.

* Field energy: a discrete Yee travelling wave in a periodic box carries
  eps0 E0^2 V / 4 in E and eps0 E0^2 cos^2(omega dt / 2) V / 4 in B at integer
  steps (B at an integer step is the mean of its two half-step values, and the
  half-step amplitude is E0 / c by Faraday's law with the lattice dispersion
  relation of Sec. 4.1), at every step.  Uniform fields on a grid with an open
  axis: the components half-located along it have n valid entries (their
  index n is padding), the others n + 1.  A uniform dielectric weights the
  electric part by eps = 1 / einv.
* Kinetic energy: a Fermi-Dirac species loaded at T = 0 carries
  N w (3/5) E_F (eq:fddist at T = 0) within 5 sigma; cold and bound species
  loaded at rest carry exactly 0.
* Current series: the first step of a cold beam in zero fields records
  N q w v0; on a periodic grid without walls every step's entry equals the
  integral of the deposited current J^{n+1/2} over the grid (the deposit of
  each particle carries q w v_{n+1/2}; pinned separately against a
  brute-force charge density).

Each would fail on a dropped factor 1/2, a missing weight, a miscounted
padding entry or a wrong sign.
"""
import math

import numpy as np
import pytest

QE = 1.602176634e-19
ME = 9.1093837015e-31
C = 299792458.0
EPS0 = 8.8541878128e-12
MU0 = 1.0 / (EPS0 * C * C)


def _grid(dims, n, dx, dt, periodic=(1, 1, 1)):
    n = list(n) + [1] * (3 - len(n))
    dx = list(dx) + [dx[-1]] * (3 - len(dx))
    return {"dims": dims, "n": n, "dx": dx, "dt": dt, "periodic": list(periodic),
            "tile": [max(1, v // 2) for v in n], "sort_every": 1, "species": []}


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_field_energy_of_travelling_wave(oracle, dims):
    n = {1: [64, 1, 1], 2: [32, 24, 1], 3: [16, 12, 10]}[dims]
    dx = {1: [1e-9] * 3, 2: [1e-9, 0.8e-9, 1e-9], 3: [1e-9, 0.8e-9, 1.1e-9]}[dims]
    dt = 0.9 / (C * math.sqrt(sum(1 / dx[a] ** 2 for a in range(dims))))
    m = [3, 2, 0]
    k = [2 * math.pi * m[a] / (n[a] * dx[a]) if a < dims else 0.0 for a in range(3)]
    s2 = sum((math.sin(k[a] * dx[a] / 2) / dx[a]) ** 2 for a in range(min(dims, 2)))
    om = 2.0 / dt * math.asin(C * dt * math.sqrt(s2))
    wdt = math.sin(om * dt / 2) / dt
    cw = math.cos(om * dt / 2)
    e0 = 3.0e8
    w = _grid(dims, n[:dims], dx[:dims], dt)
    s = oracle.Sim(w)
    L = s.shape()
    kk, jj, ii = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    X = ii * dx[0]; Y = jj * dx[1]
    e = np.zeros((3, L[2], L[1], L[0])); b = np.zeros_like(e)
    if dims == 1:
        e[1] = e0 * np.cos(k[0] * X)
        b[2] = e0 * (math.sin(k[0] * dx[0] / 2) / dx[0]) / wdt * cw * np.cos(k[0] * (X + dx[0] / 2))
    else:
        e[2] = e0 * np.cos(k[0] * X + k[1] * Y)
        b[0] = e0 * (math.sin(k[1] * dx[1] / 2) / dx[1]) / wdt * cw * np.cos(k[0] * X + k[1] * (Y + dx[1] / 2))
        b[1] = -e0 * (math.sin(k[0] * dx[0] / 2) / dx[0]) / wdt * cw * np.cos(k[0] * (X + dx[0] / 2) + k[1] * Y)
    s.set_fields(e, b)
    vol = 1.0
    for a in range(dims):
        vol *= n[a] * dx[a]
    expect = EPS0 * e0 * e0 * vol / 4.0 * (1.0 + cw * cw)
    for nsteps in (0, 1, 37):
        if nsteps:
            s.step(nsteps)
        u = s.field_energy()
        assert abs(u / expect - 1.0) < 1e-12, (dims, nsteps, u, expect)
    # the electric part alone: remove B and compare with eps0 E0^2 V / 4
    e1, _ = s.fields()
    s.set_fields(e1, np.zeros_like(b))
    assert abs(s.field_energy() / (EPS0 * e0 * e0 * vol / 4.0) - 1.0) < 1e-12


def test_field_energy_counts_valid_entries_on_open_axes(oracle):
    """2D, x open (Mur), y periodic: uniform values in every array entry, padding included."""
    nx, ny = 10, 6
    dx, dy = 1e-9, 0.7e-9
    w = _grid(2, [nx, ny], [dx, dy], 1e-18, periodic=(0, 1, 1))
    s = oracle.Sim(w)
    L = s.shape()
    assert L[0] == nx + 1 and L[1] == ny
    ex, ey, ez, bx, by, bz = 2.0, 3.0, 5.0, 7e-9, 11e-9, 13e-9
    e = np.zeros((3, L[2], L[1], L[0])); b = np.zeros_like(e)
    e[0], e[1], e[2] = ex, ey, ez
    b[0], b[1], b[2] = bx, by, bz
    s.set_fields(e, b)
    dv = dx * dy
    # half-located along x: E_x, B_y, B_z have nx valid columns; E_y, E_z, B_x have nx + 1
    expect = (0.5 * EPS0 * (ex * ex * nx + (ey * ey + ez * ez) * (nx + 1)) * ny * dv
              + 0.5 / MU0 * (bx * bx * (nx + 1) + (by * by + bz * bz) * nx) * ny * dv)
    assert abs(s.field_energy() / expect - 1.0) < 1e-13
    # E_x alone is the physical energy of a uniform field in the box, (1/2) eps0 E^2 V
    e2 = np.zeros_like(e); e2[0] = ex
    s.set_fields(e2, np.zeros_like(b))
    assert abs(s.field_energy() / (0.5 * EPS0 * ex * ex * nx * dx * ny * dy) - 1.0) < 1e-13
    # a uniform dielectric eps = 4 weights the electric energy by eps
    s.set_eps_inv(np.full((3, L[2], L[1], L[0]), 0.25))
    assert abs(s.field_energy() / (0.5 * EPS0 * 4.0 * ex * ex * nx * dx * ny * dy) - 1.0) < 1e-13


def test_kinetic_energy_fermi_dirac_at_zero_temperature(oracle):
    """N w (3/5) E_F for a T = 0 Fermi-Dirac species (eq:fddist), within 5 sigma; sigma of one
    particle's energy is sqrt(3/7 - 9/25) E_F (energies E_F u^{2/3})."""
    ef = 5.5 * QE
    w = _grid(3, [12, 12, 12], [1e-9] * 3, 1.0e-18)
    w["species"] = [{"kind": "free", "q": -QE, "m": ME, "ppc": 40, "momentum": "fd", "e_fermi": ef,
                     "temperature": 0.0, "density": 5.9e28, "region": {"kind": "all"}, "reflect": False}]
    s = oracle.Sim(w)
    sid = s.init_species(w["species"][0], 7)
    nn = s.count(sid)
    wt = s.weight(sid)
    assert nn == 12 ** 3 * 40
    # the weight is n dV / ppc
    assert abs(wt / (5.9e28 * 1e-27 / 40) - 1.0) < 1e-14
    ke = s.kinetic_energy(sid)
    expect = nn * wt * 0.6 * ef
    sigma = math.sqrt(3.0 / 7.0 - 9.0 / 25.0) * ef * wt * math.sqrt(nn)
    assert abs(ke - expect) < 5.0 * sigma, (ke, expect, sigma)
    # a factor 2 (or a dropped weight) is far outside
    assert 5.0 * sigma < 0.01 * expect


def test_kinetic_energy_of_species_at_rest_is_zero(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("disk2d")
    s = oracle.build_workload(w)
    for sid, sp in enumerate(w["species"]):
        if sp["kind"] == "bound":
            assert s.kinetic_energy(sid) == 0.0
        else:
            assert s.kinetic_energy(sid) > 0.0
    w = _grid(2, [8, 8], [1e-9, 1e-9], 1e-18)
    w["species"] = [{"kind": "free", "q": -QE, "m": ME, "ppc": 4, "momentum": "cold", "density": 5.9e28,
                     "region": {"kind": "all"}, "reflect": False}]
    s = oracle.Sim(w)
    sid = s.init_species(w["species"][0], 3)
    assert s.count(sid) == 256
    assert s.kinetic_energy(sid) == 0.0


def test_current_series_first_step_of_cold_beam(oracle):
    """Zero fields, a cold beam drifting at v0: the first entry is N q w v0."""
    w = _grid(2, [8, 6], [1e-9, 1e-9], 1.5e-18)
    rng = np.random.default_rng(5)
    nn = 300
    x = np.zeros((nn, 3))
    x[:, 0] = rng.uniform(0, 8e-9, nn)
    x[:, 1] = rng.uniform(0, 6e-9, nn)
    v0 = np.array([3.0e5, -1.2e5, 7.0e4])
    v = np.tile(v0, (nn, 1))
    s = oracle.Sim(w)
    weight = 2.5e3
    s.add_species({"kind": "free", "q": -QE, "m": ME}, weight, x, v)
    s.step(1)
    ser = s.current_series()
    assert ser.shape == (1, 3)
    expect = nn * (-QE) * weight * v0
    assert np.max(np.abs(ser[0] - expect)) <= 1e-14 * np.max(np.abs(expect))


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_current_series_equals_integral_of_deposited_current(oracle, dims):
    """Periodic thermal plasma without walls, several steps with self-consistent fields: each step's
    entry sum q w v_{n+1/2} equals sum_nodes J^{n+1/2} dV of the same step."""
    n = {1: [32], 2: [10, 8], 3: [6, 5, 4]}[dims]
    dx = {1: [0.5e-9], 2: [1e-9, 0.8e-9], 3: [1e-9, 0.9e-9, 1.1e-9]}[dims]
    dt = 0.5 * min(dx) / (C * math.sqrt(dims))
    w = _grid(dims, n, dx, dt)
    w["sort_every"] = 20
    sp = {"kind": "free", "q": -QE, "m": ME, "ppc": 16, "momentum": "fd", "e_fermi": 5.5 * QE,
          "temperature": 300.0, "density": 0.0, "region": {"kind": "all"}, "reflect": False}
    w["species"] = [sp]
    s = oracle.Sim(w)
    sid = s.init_species(sp, 11)
    s.set_ion_background(True)
    dv = float(np.prod(w["dx"][:dims]))
    qw = -QE * s.weight(sid)
    for step in range(6):
        s.step(1)
        J = s.current()
        ser = s.current_series()
        assert ser.shape == (step + 1, 3)
        _, v, _ = s.particles(sid)
        scale = abs(qw) * np.sum(np.abs(v), axis=0)
        for a in range(3):
            total = J[a].sum() * dv
            assert abs(ser[step, a] - total) <= 1e-11 * scale[a], (dims, step, a, ser[step, a], total)
