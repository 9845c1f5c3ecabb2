"""Pins of the oracle's per-particle Dirac transverse mass (Sec. 5: the input mass is m_d = p / v_F;
with p = e / v_F of each carrier, m_d = e / v_F^2 per particle).

* Energies under the 2D density of states: at T = 0 they are E_F sqrt(u); at a tiny temperature the
  tabulated sampler approaches that closed form (with the 3D weighting it would approach
  E_F u^(2/3) instead); at 0.0375 eV they pass a Kolmogorov-Smirnov test against the CDF of
  e f(e) integrated independently.
* The loader gives every carrier |v| = v_F in the sheet, m_d = e / v_F^2 > 0 in xi[i][0], and the
  mean energy of the 2D Fermi-Dirac gas.
* In a uniform B normal to the sheet, two carriers of different m_d turn by their own Boris angle
  2 atan(q B dt / (2 m_d)) per step.
* The species-constant mass is unchanged, and the option is refused for other kinds.
"""
import math

import numpy as np
import pytest

QE = 1.602176634e-19
KB = 1.380649e-23


def test_zero_and_tiny_temperature_energies(oracle):
    ef = 0.2 * QE
    u = np.random.default_rng(1).uniform(size=2000)
    e0 = oracle.dirac_energies(ef, 0.0, u)
    np.testing.assert_allclose(e0, ef * np.sqrt(u), rtol=1e-15)
    e1 = oracle.dirac_energies(ef, 1e-5 * ef, u)
    assert np.max(np.abs(e1 - ef * np.sqrt(u))) < 2e-3 * ef
    assert np.max(np.abs(e1 - ef * u ** (2.0 / 3.0))) > 0.05 * ef


def test_room_temperature_energies_follow_2d_fermi_dirac(oracle):
    from scipy import integrate, stats
    ef, kt = 0.2 * QE, 0.0375 * QE
    u = np.random.default_rng(2).uniform(size=20000)
    e = oracle.dirac_energies(ef, kt, u)
    f = lambda x: x / (1.0 + math.exp((x - ef) / kt))
    top = ef + 40 * kt
    tot = integrate.quad(f, 0, top, limit=400, points=[ef])[0]
    cdf = lambda x: np.array([integrate.quad(f, 0, min(xx, top), limit=400)[0] / tot for xx in np.atleast_1d(x)])
    grid = np.linspace(0, top, 401)
    table = cdf(grid)
    D, p = stats.kstest(e, lambda x: np.interp(x, grid, table))
    assert p > 1e-3, (D, p)


def _sheet(mpp=True, temperature=435.17):
    from paper_2501_07465_amd import workloads as W
    w = W.small("sheet2d")
    w["species"] = [dict(w["species"][0], mass_per_particle=mpp, temperature=temperature)]
    return w


def test_loader_masses_and_speeds(oracle):
    from scipy import integrate
    w = _sheet()
    s = oracle.build_workload(w)
    sp = w["species"][0]
    x, v, xi = s.particles(0)
    vf, normal = sp["v_f"], sp["sheet_normal"]
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), vf, rtol=1e-14)
    assert np.all(v[:, normal] == 0.0)
    md = xi[:, 0]
    assert np.all(md > 0)
    e = md * vf * vf
    ef, kt = sp["e_fermi"], KB * sp["temperature"]
    f = lambda x: x / (1.0 + math.exp((x - ef) / kt))
    mean = integrate.quad(lambda x: x * f(x), 0, ef + 40 * kt, limit=400, points=[ef])[0] / \
        integrate.quad(f, 0, ef + 40 * kt, limit=400, points=[ef])[0]
    assert abs(e.mean() / mean - 1) < 5 * e.std() / math.sqrt(len(e)) / mean


def test_each_carrier_turns_at_its_own_cyclotron_angle(oracle):
    from paper_2501_07465_amd import workloads as W
    dx = 1e-9
    w = {"name": "cyc", "dims": 2, "n": [16, 16, 1], "dx": [dx] * 3, "dt": W.cfl_dt(dx, 2),
         "periodic": [1, 1, 1], "tile": [8, 8, 1], "sort_every": 20, "species": [], "seed": 4}
    vf = 1e6
    sp = {"kind": "dirac", "q": -QE, "m": 1e-32, "v_f": vf, "sheet_normal": 2, "reflect": False,
          "mass_per_particle": True}
    s = oracle.Sim(w)
    L = s.shape()
    Bz = 50.0
    e = np.zeros((3, L[2], L[1], L[0]))
    b = np.zeros_like(e)
    b[2] = Bz
    s.set_fields(e, b)
    masses = np.array([0.01, 0.03]) * 9.1093837015e-31
    x = np.array([[5.2e-9, 5.3e-9, 0], [9.7e-9, 9.1e-9, 0]])
    v = np.array([[vf, 0, 0], [0, vf, 0]])
    xi = np.zeros((2, 3))
    xi[:, 0] = masses
    s.add_species(sp, 1e-12, x, v, xi)   # negligible weight: no self-field
    n = 40
    s.step(n)
    _, v1, xi1 = s.particles(0)
    dt = w["dt"]
    for k in range(2):
        i = int(np.argmin(np.abs(xi1[:, 0] - masses[k])))
        th = 2 * math.atan(-QE * Bz * dt / (2 * masses[k]))  # Boris angle per step (sign of q B)
        v0 = v[k]
        # rotation of v0 in the sheet by -n th about z (v x B with B along +z)
        ang = -n * th
        want = np.array([v0[0] * math.cos(ang) - v0[1] * math.sin(ang),
                         v0[0] * math.sin(ang) + v0[1] * math.cos(ang), 0.0])
        np.testing.assert_allclose(v1[i], want, atol=1e-9 * vf)
    # the two carriers no longer share a direction
    assert np.abs(np.dot(v1[0], v1[1])) < 0.999 * vf * vf


def test_species_constant_mass_unchanged_and_option_refused_elsewhere(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("sheet2d")
    a = oracle.build_workload(w)
    wb = {**w, "species": [dict(w["species"][0], mass_per_particle=False), w["species"][1]]}
    b = oracle.build_workload(wb)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.particles(0)[1], b.particles(0)[1])
    s = oracle.Sim(w)
    with pytest.raises(RuntimeError):
        s.add_species(dict(w["species"][1], mass_per_particle=True), 1.0, np.array([[1e-9, 15e-9, 0]]),
                      np.zeros((1, 3)), xi=np.zeros((1, 3)))
