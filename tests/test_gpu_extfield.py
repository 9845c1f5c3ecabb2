"""The static external (work-function) field on the device, through the C ABI, against the oracle.

The particles gather E + E_ext (Sec. 3 barrier outside the Maxwell solve).  FP64: element by
element within 1e-12 of the oracle's scale, with electrons sent toward the barrier so that it turns
many of them back; in a batch next to a member without one.  FP32: one step from identical inputs
within 1e-6.  The field diagnostics and the Maxwell fields leave E_ext out.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HEIGHT_EV = 9.8   # E_F + work function of a noble metal
WIDTH = 2.0       # cells


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if a.size else 0.0


def _walled(name, fp64=True):
    from paper_2501_07465_amd import workloads as W
    w = W.small(name)
    if name == "sphere3d" and fp64:
        w["tile"] = [4, 4, 4]
    return W.with_potential_wall(w, HEIGHT_EV, WIDTH)


def _outward(w, state, frac=0.01, seed=8):
    """Free electrons within 1.5 cells of the surface sent outward at frac cells per step."""
    rng = np.random.default_rng(seed)
    dims = w["dims"]
    dx = np.array(w["dx"])
    reg = w["wall"]["region"]
    out = []
    for sid, (x, v, xi, wt) in enumerate(state):
        v = v.copy()
        if w["species"][sid]["kind"] == "free":
            d = x[:, :dims] / dx[:dims] - np.array(reg["center"][:dims])
            r = np.linalg.norm(d, axis=1)
            near = r > reg["radius"] - 1.5
            nrm = np.zeros_like(v)
            nrm[:, :dims] = d / r[:, None]
            t = rng.normal(size=v.shape) * 0.3
            dirs = nrm + t
            dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
            v[near] = dirs[near] * (frac * dx[0] / w["dt"])
        out.append((x, v, xi, wt))
    return out


def _oracle_from(oracle, w, state, fields):
    from paper_2501_07465_amd import workloads as W
    ref = oracle.Sim(w)
    ref.set_ext_field(W.wall_field(w))
    for sid, (x, v, xi, wt) in enumerate(state):
        ref.add_species(w["species"][sid], wt, x, v, xi)
    ref.set_fields(*fields)
    return ref


def _compare(sim, ref, w, tol, label):
    for sid in range(len(w["species"])):
        xg, vg, _ = sim.particles(sid)
        xr, vr, _ = ref.particles(sid)
        ex = float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) if len(xg) else 0.0
        ev = _rel(vg, vr)
        print(f"{label} species {sid}: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
        assert ex < tol and ev < tol, (label, sid, ex, ev)
    eg, _ = sim.fields()
    er, _ = ref.fields()
    ee = _rel(eg, er)
    print(f"{label} fields: E rel {ee:.2e}", flush=True)
    assert ee < tol, (label, ee)


@pytest.mark.parametrize("name,steps", [("disk2d", 150), ("sphere3d", 30)])
def test_fp64_wall_matches_oracle(oracle, name, steps):
    from paper_2501_07465_amd import pic
    w = _walled(name)
    print(f"case fp64 wall {name} {steps} steps", flush=True)
    base = oracle.build_workload(w)
    st, fl = _outward(w, base.state()), base.fields()
    ref = _oracle_from(oracle, w, st, fl)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=fl, graphs=False)
    sim.step(steps)
    ref.step(steps)
    _compare(sim, ref, w, 1e-12, f"fp64 wall {name}")
    # the barrier acted: without it the electrons end elsewhere
    free = oracle.Sim({k: v for k, v in w.items() if k != "wall"})
    for sid, (x, v, xi, wt) in enumerate(st):
        free.add_species(w["species"][sid], wt, x, v, xi)
    free.set_fields(*fl)
    free.step(steps)
    dv = _rel(ref.particles(0)[1], free.particles(0)[1])
    print(f"with vs without the barrier: v rel {dv:.2e}", flush=True)
    assert dv > 1e-3
    # the field energy leaves the external field out
    assert abs(sim.field_energy() / ref.field_energy() - 1.0) < 1e-12


def test_fp32_wall_one_step(oracle):
    from paper_2501_07465_amd import pic
    w = _walled("disk2d", fp64=False)
    print("case fp32 wall one step", flush=True)
    base = oracle.build_workload(w)
    base.step(3)
    st = _outward(w, base.state())
    dx = np.array(w["dx"])
    st32 = []
    for x, v, xi, wt in st:
        X = x / dx
        c = np.floor(X)
        x32 = (c + (X - c).astype(np.float32).astype(np.float64)) * dx
        st32.append((x32, v.astype(np.float32).astype(np.float64),
                     None if xi is None else xi.astype(np.float32).astype(np.float64), wt))
    e, b = base.fields()
    fl = (e.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64))
    ref = _oracle_from(oracle, w, st32, fl)
    sim = pic.Simulation(w, precision="fp32", states=st32, fields=fl, graphs=False)
    sim.step(1)
    ref.step(1)
    for sid in range(len(w["species"])):
        xg, vg, _ = sim.particles(sid)
        xr, vr, _ = ref.particles(sid)
        vscale = np.max(np.linalg.norm(vr, axis=1))
        ev = float(np.max(np.abs(vg - vr)) / vscale)
        ex = float(np.max(np.abs(xg - xr) / dx))
        print(f"fp32 wall species {sid}: v err {ev:.2e}, x err {ex:.2e} cells", flush=True)
        assert ev <= 1e-6 and ex <= 1e-6, (sid, ev, ex)


def test_batch_mixes_wall_and_plain_members(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    wa = _walled("disk2d")
    wb = W.small("disk2d")
    print("case batch wall + plain", flush=True)
    base = oracle.build_workload(wa)
    sta, fla = _outward(wa, base.state()), base.fields()
    refa = _oracle_from(oracle, wa, sta, fla)
    refb = oracle.build_workload(wb)
    batch = pic.Batch(2, 2, "fp64")
    sa = pic.Simulation(wa, precision="fp64", states=sta, fields=fla, graphs=False, stream=batch.stream)
    sb = pic.Simulation(wb, precision="fp64", states=refb.state(), fields=refb.fields(), graphs=False,
                        stream=batch.stream)
    batch.add(sa)
    batch.add(sb)
    batch.step(60)
    refa.step(60)
    refb.step(60)
    batch.remove(sa)
    batch.remove(sb)
    _compare(sa, refa, wa, 1e-12, "batch wall")
    _compare(sb, refb, wb, 1e-12, "batch plain")


def test_ext_field_errors():
    from paper_2501_07465_amd import pic, workloads as W
    w = _walled("disk2d")
    sim = pic.Simulation(w, precision="fp64", graphs=False)
    e = W.wall_field(w)
    bad = e.copy()
    bad[0, 0, 3, 3] = np.inf
    with pytest.raises(pic.PicError) as err:
        pic.pic_load_ext_field(sim.h, bad)
    assert err.value.code == pic.PIC_EINVAL
    plain = pic.Simulation(W.small("disk2d"), precision="fp64", graphs=False)
    with pytest.raises(pic.PicError) as err:
        pic.pic_load_ext_field(plain.h, e)
    assert err.value.code == pic.PIC_EINVAL
