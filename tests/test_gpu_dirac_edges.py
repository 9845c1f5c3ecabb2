"""Diffusive ribbon edges for Dirac carriers on the device, through the C ABI, against the oracle.

A graphene ribbon (the sheet of the small sheet workload cut to x in [10, 90]) with diffusive ends:
a carrier that crosses an end is mirrored back and leaves along the in-sheet cosine law about the
inward normal, drawn from Philox4x32-10 with counter (slot, step, species id, 2^31) under the
species seed on both sides.  FP64 runs agree within 1e-12 of the oracle's scale, with the
species-constant and the per-carrier mass; FP32 one step from identical inputs within 1e-6.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if a.size else 0.0


def _ribbon(scatter="diffuse", mpp=False):
    from paper_2501_07465_amd import workloads as W
    w = W.small("sheet2d")
    sp = w["species"][0]
    lo, hi = list(sp["region"]["lo"]), list(sp["region"]["hi"])
    lo[0], hi[0] = 10.0, 90.0
    w["species"][0] = dict(sp, region={"kind": "box", "lo": lo, "hi": hi}, reflect=True, scatter=scatter,
                           mass_per_particle=mpp)
    return w


def _toward_ends(w, state, within, seed=7):
    """The state with every fourth Dirac carrier moved to within `within` cells of the nearer
    ribbon end (the rest of its position kept) and sent outward at an in-sheet angle below
    1.1 rad from the end's normal."""
    rng = np.random.default_rng(seed)
    dx = np.array(w["dx"])
    out = []
    for sid, (x, v, xi, wt) in enumerate(state):
        sp = w["species"][sid]
        if sp["kind"] == "dirac":
            X = x[:, 0] / dx[0]
            lo, hi = sp["region"]["lo"][0], sp["region"]["hi"][0]
            side = np.where(hi - X < X - lo, 1.0, -1.0)
            near = np.arange(len(X)) % 4 == 0
            gap = rng.uniform(0.05, 1.0, len(X)) * within
            x = x.copy()
            x[near, 0] = np.where(side > 0, hi - gap, lo + gap)[near] * dx[0]
            a = rng.uniform(-1.1, 1.1, len(X))
            vn = np.stack([side * np.cos(a), np.zeros(len(X)), np.sin(a)], axis=1) * sp["v_f"]
            v = v.copy()
            v[near] = vn[near]
        out.append((x, v, xi, wt))
    return out


def _oracle_from(oracle, w, state, fields):
    ref = oracle.Sim(w)
    for sid, (x, v, xi, wt) in enumerate(state):
        ref.add_species(w["species"][sid], wt, x, v, xi)
    ref.set_fields(*fields)
    return ref


def _compare(sim, ref, w, tol, label):
    for sid in range(len(w["species"])):
        xg, vg, _ = sim.particles(sid)
        xr, vr, _ = ref.particles(sid)
        ex = float(np.max(np.abs(xg - xr) / np.array(w["dx"])))
        ev = _rel(vg, vr)
        print(f"{label} species {sid}: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
        assert ex < tol and ev < tol, (label, sid, ex, ev)
    eg, _ = sim.fields()
    er, _ = ref.fields()
    ee = _rel(eg, er)
    print(f"{label} fields: E rel {ee:.2e}", flush=True)
    assert ee < tol


@pytest.mark.parametrize("mpp", [False, True])
def test_fp64_ribbon_matches_oracle(oracle, mpp):
    from paper_2501_07465_amd import pic
    w = _ribbon(mpp=mpp)
    steps = 120
    print(f"case fp64 dirac ribbon diffuse mpp={mpp} {steps} steps", flush=True)
    base = oracle.build_workload(w)
    st, fl = _toward_ends(w, base.state(), 0.25), base.fields()
    ref = _oracle_from(oracle, w, st, fl)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=fl, graphs=False)
    sim.step(steps)
    ref.step(steps)
    _compare(sim, ref, w, 1e-12, f"fp64 dirac ribbon mpp={mpp}")
    x, v, _ = sim.particles(0)
    X = x[:, 0] / w["dx"][0]
    assert np.all((X >= 10.0) & (X <= 90.0))
    assert np.all(v[:, 1] == 0.0)
    # the ends were hit: the specular ribbon ends elsewhere
    ws = {**w, "species": [dict(w["species"][0], scatter="specular"), w["species"][1]]}
    spec = _oracle_from(oracle, ws, st, fl)
    spec.step(steps)
    dv = _rel(ref.particles(0)[1], spec.particles(0)[1])
    print(f"diffuse vs specular ribbon oracle runs: v rel {dv:.2e}", flush=True)
    assert dv > 1e-2


def test_fp32_ribbon_one_step(oracle):
    from paper_2501_07465_amd import pic
    w = _ribbon()
    print("case fp32 dirac ribbon one step", flush=True)
    base = oracle.build_workload(w)
    base.step(3)
    st = _toward_ends(w, base.state(), 0.003)
    dx = np.array(w["dx"])
    x0, v0 = st[0][0], st[0][1]
    Xe = (x0[:, 0] + v0[:, 0] * w["dt"]) / dx[0]
    crossing = int(np.sum((Xe > 90.0) | (Xe < 10.0)))
    st32 = []
    for x, v, xi, wt in st:
        Xc = x / dx
        c = np.floor(Xc)
        x32 = (c + (Xc - c).astype(np.float32).astype(np.float64)) * dx
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
        print(f"fp32 dirac ribbon species {sid}: {crossing} crossing, v err {ev:.2e}, x err {ex:.2e} cells",
              flush=True)
        assert ev <= 1e-6 and ex <= 1e-6
    assert crossing > 5


def test_diffuse_refused_for_sheetless_dirac():
    from paper_2501_07465_amd import pic
    w = _ribbon()
    h = pic.pic_create(pic.grid_desc(w))
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_species(h, pic.species_desc(dict(w["species"][0], sheet_normal=-1)), 1)
    assert e.value.code == pic.PIC_EINVAL
    pic.pic_destroy(h)
