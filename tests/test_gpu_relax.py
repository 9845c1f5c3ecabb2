"""The FD relaxation workload and the device energy histogram, through the C ABI.

FP64 from the oracle's loaded state: the device histogram equals the oracle's bin for bin, before
and after 200 steps (the states agree to 1e-12, far from any bin edge in practice), and the
particles and fields agree within 1e-12.  The device loader's histogram of the full-size cube
follows the oracle loader's within Poisson noise.  The study driver runs a short case end to end.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

QE = 1.602176634e-19


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_fp64_relax_histogram_and_state_match_oracle(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("relax3d")
    print("case fp64 relax3d small 200 steps", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False)
    sp = w["species"][0]
    e_max = sp["e_fermi"] + 40 * 0.0375 * QE
    for nb in (400, 4096):
        assert np.array_equal(pic.pic_energy_histogram(sim.h, 0, e_max, nb), ref.energy_histogram(0, e_max, nb))
    sim.step(200)
    ref.step(200)
    x, v, _ = sim.particles(0)
    xr, vr, _ = ref.particles(0)
    ex, ev = float(np.max(np.abs(x - xr) / np.array(w["dx"]))), _rel(v, vr)
    print(f"relax fp64: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
    assert ex < 1e-12 and ev < 1e-12
    hg = pic.pic_energy_histogram(sim.h, 0, e_max, 400)
    hr = ref.energy_histogram(0, e_max, 400)
    assert int(np.abs(hg.astype(np.int64) - hr.astype(np.int64)).sum()) <= 2
    assert int(hg.sum()) == sim.count(0)
    assert _rel(sim.fields()[0], ref.fields()[0]) < 1e-12


def test_device_loader_histogram_matches_oracle_loader(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    w = W.relax3d(ppc=32, n=16)
    print("case relax3d loader histogram", flush=True)
    sim = pic.Simulation(w, precision="fp32", graphs=False)
    ref = oracle.build_workload(w)
    sp = w["species"][0]
    e_max = sp["e_fermi"] + 40 * 0.0375 * QE
    hg = pic.pic_energy_histogram(sim.h, 0, e_max, 200).astype(float)
    hr = ref.energy_histogram(0, e_max, 200).astype(float)
    assert hg.sum() == hr.sum() == sim.count(0)
    # same seed and generator: the two loaders agree to FP32 rounding of the velocities
    moved = np.abs(hg - hr).sum()
    print(f"loader histograms: {int(moved)} of {int(hg.sum())} counts differ", flush=True)
    assert moved <= 1e-3 * hg.sum()


def test_study_driver_short_case(oracle):
    from paper_2501_07465_amd import relax, workloads as W
    print("case relax study driver", flush=True)
    out = relax.run_case(6e28, 256, 2.0, samples=5, n=8)
    print({k: out[k] for k in ("particles", "steps", "A_ev_per_sqrt_fs", "beta_ev")}, flush=True)
    assert out["particles"] == 8 ** 3 * 256
    assert len(out["beta_ev"]) >= 5
    # beta of the loaded state equals the fit of the oracle loader's histogram of the same workload
    w = W.relax3d(density=6e28, ppc=256, n=8, t_end_fs=2.0)
    ef, kt = w["species"][0]["e_fermi"], 0.0375 * QE
    h = oracle.build_workload(w).energy_histogram(0, ef + 40 * kt, 200)
    b_ref = relax.tail_beta(h, ef + 40 * kt, ef + 2 * kt, min_count=5) / QE
    b0 = out["beta_ev"][0]
    assert abs(b0 / b_ref - 1) < 1e-2, (b0, b_ref)
    # and it is the loaded 0.0375 eV tail to within the noise of a few hundred tail particles
    assert abs(b0 / 0.0375 - 1) < 0.5, b0
    assert all(math.isfinite(b) for b in out["beta_ev"])
    assert math.isfinite(out["A_ev_per_sqrt_fs"]) and out["A_ev_per_sqrt_fs"] > 0


def test_energy_histogram_errors():
    from paper_2501_07465_amd import pic, workloads as W
    sim = pic.Simulation(W.small("relax3d"), precision="fp32", graphs=False)
    for nb, em in ((0, 1e-18), (4097, 1e-18), (10, 0.0), (10, float("nan"))):
        with pytest.raises(pic.PicError) as e:
            pic.pic_energy_histogram(sim.h, 0, em, nb)
        assert e.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError):
        pic.pic_energy_histogram(sim.h, 3, 1e-18, 10)
