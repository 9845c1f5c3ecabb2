"""FP32 form over a whole run against the FP64 oracle.

Both start from the same state (the oracle's FD-sampled particles and initial fields).  After the
run, the field energy and the spectrum of the total-current series (Hann window, magnitude of the
real FFT of each component) agree within 1e-3 relative; the spectrum error is taken against the
largest spectral magnitude.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _spectrum(series):
    s = np.asarray(series, dtype=np.float64)
    win = np.hanning(s.shape[0])[:, None]
    return np.abs(np.fft.rfft(s * win, axis=0))


@pytest.mark.parametrize("name,steps", [("slab1d", 1000), ("disk2d", 400), ("sheet2d", 400), ("sphere3d", 100)])
def test_fp32_run_field_energy_and_current_spectrum(oracle, name, steps):
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small(name)
    print(f"case fp32 run {name} {steps} steps", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp32", states=ref.state(), fields=ref.fields(), graphs=True,
                         series_cap=steps + 64)
    sim.step(steps)
    ref.step(steps)
    u32, u64 = sim.field_energy(), ref.field_energy()
    s32 = _spectrum(sim.current_series()[:steps])
    s64 = _spectrum(ref.current_series()[:steps])
    eu = abs(u32 - u64) / u64
    es = float(np.max(np.abs(s32 - s64)) / np.max(s64))
    print(f"fp32 {name}: field energy rel {eu:.2e}, current spectrum rel {es:.2e}", flush=True)
    assert eu <= 1e-3 and es <= 1e-3, (name, eu, es)


def test_fp32_dirac_speed_stays_at_fermi_speed():
    """FP32 Dirac carriers keep |v| = v_F at every step (renormalised push, Sec. 5) to within two FP32
    machine epsilons relative (2 * 2^-23 v_F; rounding of the squared speed, its reciprocal square root
    and the three products each contribute about one half to one), and never acquire a sheet-normal
    velocity."""
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("sheet2d")
    sp = w["species"][0]
    vf, normal = sp["v_f"], sp["sheet_normal"]
    eps = float(np.finfo(np.float32).eps)
    sim = pic.Simulation(w, precision="fp32", graphs=False)
    worst = 0.0
    for _ in range(8):
        sim.step(5)
        _, v, _ = sim.particles(0)
        speed = np.linalg.norm(v.astype(np.float64), axis=1)
        worst = max(worst, float(np.max(np.abs(speed - vf))) / (eps * vf))
        assert np.all(v[:, normal] == 0.0)
    print(f"FP32 Dirac |v| - v_F: {worst:.2f} machine epsilons of v_F", flush=True)
    assert worst <= 2.0


@pytest.mark.parametrize("variant,steps,tol", [("dielectric", 400, 1e-3), ("barrier", 400, 1e-3),
                                               ("diffuse", 400, 1e-3)])
def test_fp32_run_with_next_row_physics(oracle, variant, steps, tol):
    """The same whole-run check on the disk with a per-cell permittivity, a work-function barrier,
    or diffusive walls (measured 1e-6 .. 6e-6).  With diffusive walls a particle that reaches the
    wall a step apart in FP32 would draw another direction; in 400 steps of the small disk that
    does not move the collective quantities beyond the same bar."""
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    if variant == "dielectric":
        w = W.with_dielectric(w, [3.7, 3.7, 2.5])
    elif variant == "barrier":
        w = W.with_potential_wall(w, 9.8, 2.0)
    else:
        w = W.with_diffuse_walls(w)
    print(f"case fp32 run disk {variant} {steps} steps", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp32", states=ref.state(), fields=ref.fields(), graphs=True,
                         series_cap=steps + 64)
    sim.step(steps)
    ref.step(steps)
    u32, u64 = sim.field_energy(), ref.field_energy()
    s32 = _spectrum(sim.current_series()[:steps])
    s64 = _spectrum(ref.current_series()[:steps])
    eu = abs(u32 - u64) / u64
    es = float(np.max(np.abs(s32 - s64)) / np.max(s64))
    print(f"fp32 disk {variant}: field energy rel {eu:.2e}, current spectrum rel {es:.2e}", flush=True)
    assert eu <= tol and es <= tol, (variant, eu, es)
