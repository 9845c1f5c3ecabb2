"""Gyrotropic bound push on the GPU (Appendix A.2, eq:modborisBrot, with its numerator read as
R = L_-^{-1} L_+, L_- = I + G - eps(b), L_+ = I - G + eps(b), b = (dt/2)(q/m)B, G = (dt/2) gamma):
bound species with the magnetic force weighted in (b_weight = 1) in a static magnetic field.

The device solves the 3x3 system by Cramer's rule, the oracle by a pivoted elimination; the two
are compared element by element.  FP64 within 1e-12 of the oracle's scale over whole runs; FP32 one
step from identical inputs within 1e-6.  The same runs with b_weight = 0 end elsewhere, so the
rotation is exercised.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# static field per workload [T]: oblique in 3D so every off-diagonal entry of eps(b) is nonzero; in the
# sheet's plane (along x) for the graphene sheet, so the light Dirac carriers (m_d = 0.0176 m_e) are
# not spun into a strongly cancelling current, whose sum-order rounding would dominate E
B_STATIC = {"disk2d": (1.5e3, -2.0e3, 4.0e3), "sheet2d": (2.0e3, 0.0, 0.0), "sphere3d": (2.0e3, -3.0e3, 3.5e3)}


def _gyro_workload(name, fp64=True):
    from paper_2501_07465_amd import workloads as W
    w = W.small(name)
    if name == "sphere3d" and fp64:
        w["tile"] = [4, 4, 4]  # FP64 3D windows within 64 KiB of LDS
    n = 0
    for sp in w["species"]:
        if sp["kind"] == "bound":
            sp["b_weight"] = 1.0
            n += 1
    assert n == 1
    return w


def _with_static_b(ref, w, name):
    e, b = ref.fields()
    for c in range(3):
        b[c] += B_STATIC[name][c]
    ref.set_fields(e, b)
    return e, b


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if a.size else 0.0


@pytest.mark.parametrize("name,steps", [("disk2d", 40), ("sheet2d", 40), ("sphere3d", 20)])
def test_fp64_gyrotropic_bound_push_matches_oracle(oracle, name, steps):
    from paper_2501_07465_amd import pic
    w = _gyro_workload(name)
    print(f"case fp64 gyro {name} {steps} steps", flush=True)
    loaded = oracle.build_workload(w)
    st = loaded.state()
    e, b = _with_static_b(loaded, w, name)

    # both oracle runs start from the exported state (positions in metres, as the device gets them):
    # a bound particle moves ~1e-6 cell in its first steps, so a one-ulp difference in its start
    # offset would already be a 1e-10 part of its current
    def from_state(ww):
        r = oracle.Sim(ww)
        for sid, (x, v, xi, wt) in enumerate(st):
            r.add_species(ww["species"][sid], wt, x, v, xi)
        r.set_ion_background(False)
        r.set_fields(e, b)
        return r

    ref = from_state(w)
    # the same state without the magnetic force on the bound species
    w0 = _gyro_workload(name)
    for sp in w0["species"]:
        if sp["kind"] == "bound":
            sp["b_weight"] = 0.0
    ref0 = from_state(w0)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=(e, b), graphs=False)
    sim.step(steps)
    ref.step(steps)
    ref0.step(steps)
    for sid, sp in enumerate(w["species"]):
        xg, vg, xig = sim.particles(sid)
        xr, vr, xir = ref.particles(sid)
        ev = _rel(vg, vr)
        ex = float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) if len(xr) else 0.0
        print(f"fp64 gyro {name} species {sid} ({sp['kind']}): v rel {ev:.2e}, x err {ex:.2e}", flush=True)
        assert ev < 1e-12 and ex < 1e-12, (name, sid, ev, ex)
        if sp["kind"] == "bound":
            exi = _rel(xig, xir)
            assert exi < 1e-12, (name, sid, exi)
            _, v0, _ = ref0.particles(sid)
            d = _rel(v0, vr)
            print(f"  without the magnetic force the bound velocities differ by {d:.2e}", flush=True)
            assert d > 1e-6, d
    eg, bg = sim.fields()
    er, br = ref.fields()
    assert _rel(eg, er) < 1e-12
    assert _rel(bg, br) < 1e-12
    assert _rel(sim.current_series(), ref.current_series()) < 1e-12


@pytest.mark.parametrize("name", ["disk2d", "sheet2d", "sphere3d"])
def test_fp32_gyrotropic_bound_push_one_step(oracle, name):
    """FP32 form, one step from identical inputs (FP64 values rounded to FP32) within 1e-6."""
    from paper_2501_07465_amd import pic
    w = _gyro_workload(name, fp64=False)
    print(f"case fp32 gyro one step {name}", flush=True)
    base = oracle.build_workload(w)
    _with_static_b(base, w, name)
    base.step(3)
    dx = np.array(w["dx"])
    st32 = []
    for x, v, xi, wt in base.state():
        X = x / dx
        c = np.floor(X)
        off32 = (X - c).astype(np.float32).astype(np.float64)
        st32.append(((c + off32) * dx, v.astype(np.float32).astype(np.float64),
                     None if xi is None else xi.astype(np.float32).astype(np.float64), wt))
    e, b = base.fields()
    e32, b32 = e.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    ref = oracle.Sim(w)
    for sid, (x, v, xi, wt) in enumerate(st32):
        ref.add_species(w["species"][sid], wt, x, v, xi)
    ref.set_fields(e32, b32)
    sim = pic.Simulation(w, precision="fp32", states=st32, fields=(e32, b32), graphs=False)
    sim.step(1)
    ref.step(1)
    for sid, sp in enumerate(w["species"]):
        xg, vg, xig = sim.particles(sid)
        xr, vr, xir = ref.particles(sid)
        vscale = np.max(np.linalg.norm(vr, axis=1))
        ev = float(np.max(np.abs(vg - vr)) / vscale)
        ex = float(np.max(np.abs(xg - xr) / dx))
        print(f"fp32 gyro {name} species {sid} ({sp['kind']}): v err {ev:.2e}, x err {ex:.2e}", flush=True)
        assert ev <= 1e-6 and ex <= 1e-6, (name, sid, ev, ex)
        if sp["kind"] == "bound":
            exi = float(np.max(np.abs(xig - xir)) / np.max(np.abs(xir)))
            assert exi <= 1e-6, (name, sid, exi)
