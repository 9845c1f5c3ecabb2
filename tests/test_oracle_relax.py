"""The FD relaxation study's pieces on the CPU (Sec. 2): the stated Fermi energies, the oracle's
energy histogram, and the host fits of relax.py.

* The relaxation workload's E_F values equal hbar^2 (3 pi^2 n)^(2/3) / (2 m) of its densities.
* or_energy_histogram puts hand-placed energies in the bins floor(E / e_max * nbins), the rest in
  the overflow entry, and counts every macroparticle once.
* The FD loader's energy histogram follows sqrt(E) f(E) (Poisson, 5 sigma per bin and chi^2).
* tail_beta recovers beta of an exact exponential tail to round-off and kT of a sampled
  Fermi-Dirac tail to a few per cent; sqrt_law recovers A of beta = A sqrt(t) exactly.
"""
import math

import numpy as np
import pytest

QE = 1.602176634e-19
ME = 9.1093837015e-31
KB = 1.380649e-23


def test_relax_fermi_energies_match_closed_form(oracle):
    from paper_2501_07465_amd import workloads as W
    for n, ef in W.RELAX_EF_EV.items():
        assert abs(oracle.fermi_energy(n, ME) / QE / ef - 1) < 1e-9


def test_energy_histogram_bins_hand_placed(oracle):
    w = {"name": "h", "dims": 1, "n": [16, 1, 1], "dx": [1e-9] * 3, "dt": 1e-18, "periodic": [1, 1, 1],
         "tile": [8, 1, 1], "species": [], "seed": 1}
    s = oracle.Sim(w)
    e_max, nb = 4.0 * QE, 8
    # bin k holds [0.5 k, 0.5 (k + 1)) eV; the energies sit away from the bin edges
    ev = np.array([0.1, 0.6, 0.6, 1.2, 3.9, 4.5, 7.0, 0.0])
    speeds = np.sqrt(2 * ev * QE / ME)
    v = np.zeros((len(ev), 3))
    v[:, 1] = speeds
    x = np.tile([3e-9, 0, 0], (len(ev), 1))
    s.add_species({"kind": "free", "q": -QE, "m": ME, "reflect": False}, 1.0, x, v)
    h = s.energy_histogram(0, e_max, nb)
    want = np.zeros(nb + 1, dtype=np.uint64)
    for e in ev:
        b = int(e / 4.0 * nb)
        want[min(b, nb)] += 1
    # 4.5 and 7 eV land in the overflow (at or above e_max); 0.0 in bin 0
    assert want[nb] == 2
    assert np.array_equal(h, want)
    assert int(h.sum()) == len(ev)


def test_loader_energy_histogram_follows_fd(oracle):
    from scipy import integrate
    from paper_2501_07465_amd import workloads as W
    w = W.relax3d(ppc=64, n=8, box_nm=1.0, t_end_fs=0.1, tile=(4, 4, 4))
    s = oracle.build_workload(w)
    N = s.count(0)
    sp = w["species"][0]
    ef, kt = sp["e_fermi"], KB * sp["temperature"]
    e_max, nb = ef + 10 * kt, 40
    h = s.energy_histogram(0, e_max, nb).astype(float)
    f = lambda e: math.sqrt(e) / (1.0 + math.exp((e - ef) / kt))
    tot = integrate.quad(f, 0, ef + 60 * kt, limit=400, points=[ef])[0]
    edges = np.linspace(0, e_max, nb + 1)
    p = np.array([integrate.quad(f, edges[i], edges[i + 1], limit=200)[0] for i in range(nb)]) / tot
    exp = N * p
    assert np.all(np.abs(h[:nb] - exp) < 5 * np.sqrt(exp) + 2)
    chi2 = np.sum((h[:nb] - exp) ** 2 / np.maximum(exp, 1))
    assert chi2 < nb + 5 * math.sqrt(2 * nb)


def test_tail_beta_exact_exponential():
    from paper_2501_07465_amd import relax
    e_max, nb = 10.0 * QE, 200
    beta = 0.17 * QE
    e = relax.bin_centres(e_max, nb)
    counts = np.append(1e9 * np.exp(-e / beta), 0.0)
    got = relax.tail_beta(counts, e_max, 1.0 * QE, min_count=1)
    assert abs(got / beta - 1) < 1e-9


def test_tail_beta_of_sampled_fermi_dirac_tail_is_kt(oracle):
    from paper_2501_07465_amd import relax
    ef, kt = 5.5886 * QE, 0.0375 * QE
    rng = np.random.default_rng(3)
    u = rng.uniform(size=2_000_000)
    speed = oracle.fd_speeds(ef, kt, ME, u)
    e = 0.5 * ME * speed ** 2
    e_max, nb = ef + 40 * kt, 400
    counts = np.bincount(np.minimum((e / e_max * nb).astype(int), nb), minlength=nb + 1)
    beta = relax.tail_beta(counts, e_max, ef + 3 * kt)
    assert abs(beta / kt - 1) < 0.05, beta / kt


def test_sqrt_law_exact():
    from paper_2501_07465_amd import relax
    t = np.linspace(0, 20e-15, 21)
    A = 3.0e-12
    beta = A * np.sqrt(t)
    beta[0] = 0.04 * QE  # the t = 0 sample is left out of the fit
    assert abs(relax.sqrt_law(t, beta) / A - 1) < 1e-12
