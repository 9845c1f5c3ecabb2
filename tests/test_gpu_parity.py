"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 form: element by element within 1e-12 of the oracle's scale (the oracle's
twin runs put the round-off floor near 3e-13 after 1000 steps).  Cell keys and
the sort order: bit-exact on identical inputs.  FP32 form: one step from
identical FP64 inputs rounded to FP32 within 1e-6 (velocity relative to the
species' largest speed, position relative to the cell size).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _small(name, fp64=True):
    from paper_2501_07465_amd import workloads as W
    w = W.small(name)
    if name == "sphere3d" and fp64:
        w["tile"] = [4, 4, 4]  # FP64 3D windows within 64 KiB of LDS
    return w


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if a.size else 0.0


def _compare(sim, ref, w, tol, label):
    for sid, sp in enumerate(w["species"]):
        xg, vg, xig = sim.particles(sid)
        xr, vr, xir = ref.particles(sid)
        assert xg.shape == xr.shape, label
        dx = np.array(w["dx"])
        ex = float(np.max(np.abs(xg - xr) / dx)) if len(xg) else 0.0
        ev = _rel(vg, vr)
        print(f"{label} species {sid}: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
        assert ex < tol, (label, sid, "x", ex)
        assert ev < tol, (label, sid, "v", ev)
        if sp["kind"] == "bound":
            exi = _rel(xig, xir)
            assert exi < tol, (label, sid, "xi", exi)
    eg, bg = sim.fields()
    er, br = ref.fields()
    ee, eb = _rel(eg, er), _rel(bg, br, max(np.max(np.abs(br)), np.max(np.abs(er)) / 3e8))
    print(f"{label} fields: E rel {ee:.2e}, B rel {eb:.2e}", flush=True)
    assert ee < tol and eb < tol, (label, ee, eb)


@pytest.mark.parametrize("name,steps,tile", [("slab1d", 60, None), ("disk2d", 40, None), ("sheet2d", 40, None),
                                            ("sphere3d", 20, None),
                                            # the FP64 tile shape compiled with constant window geometry
                                            ("sphere3d", 20, [4, 8, 4]),
                                            # tiles two cells wide: more tile columns reach a field
                                            # task than its column mask has bits, so it reads J on
                                            # every column
                                            ("disk2d", 40, [2, 8, 1]), ("sphere3d", 20, [2, 4, 4])])
def test_fp64_matches_oracle_from_same_state(oracle, name, steps, tile):
    from paper_2501_07465_amd import pic
    w = _small(name)
    if tile is not None:
        w["tile"] = list(tile)
    print(f"case fp64 {name} {steps} steps tile {w.get('tile')}", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False)
    sim.step(steps)
    ref.step(steps)
    _compare(sim, ref, w, 1e-12, f"fp64 {name}")
    # keys of the final state, bit-exact
    for sid in range(len(w["species"])):
        assert np.array_equal(sim.keys(sid), ref.keys(sid).astype(np.int64))
    # total current series
    sg, sr = sim.current_series(), ref.current_series()
    assert sg.shape == sr.shape
    assert _rel(sg, sr) < 1e-12


@pytest.mark.parametrize("periodic", [[0, 0, 1], [1, 1, 1]])
def test_fp64_2d_all_open_and_all_periodic(oracle, periodic):
    """The small disk with both in-plane axes open (Mur on every face and corner, source plane
    ending on open faces) or both periodic, FP64 GPU vs oracle over 60 steps."""
    from paper_2501_07465_amd import pic
    w = _small("disk2d")
    w["periodic"] = list(periodic)
    w["source"]["index"] = [6, 0, 0]
    print(f"case fp64 disk periodic {periodic}", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False)
    sim.step(60)
    ref.step(60)
    _compare(sim, ref, w, 1e-12, f"fp64 disk periodic {periodic}")


def test_fp64_slab_1000_steps(oracle):
    """The 1D slab at full size (256 cells, 64 ppc) for 1000 steps, FP64 GPU vs oracle."""
    from paper_2501_07465_amd import pic, workloads as W
    w = W.slab1d()
    print("case fp64 slab1d full 1000 steps", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields())
    sim.step(1000)
    ref.step(1000)
    _compare(sim, ref, w, 1e-12, "fp64 slab1d 1000")
    assert abs(sim.field_energy() / ref.field_energy() - 1) < 1e-12


@pytest.mark.parametrize("name", ["slab1d", "disk2d", "sheet2d", "sphere3d"])
def test_loader_matches_oracle_loader(oracle, name):
    """pic_init_species (device Fermi-Dirac loader, Philox) vs the oracle's loader, same seed."""
    from paper_2501_07465_amd import pic
    w = _small(name)
    print(f"case loader {name}", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", init_fields=False, graphs=False)
    for sid, sp in enumerate(w["species"]):
        xg, vg, xig = sim.particles(sid)
        xr, vr, xir = ref.particles(sid)
        assert xg.shape == xr.shape
        assert float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) < 1e-12
        if np.max(np.abs(vr)) > 0:
            assert _rel(vg, vr) < 1e-12
        else:
            assert np.all(vg == 0)
        if sp["kind"] == "bound":
            assert _rel(xig, xir) < 1e-12


def test_sort_order_bit_exact(oracle):
    """After a sort the particle order equals the stable order of the cell keys (oracle)."""
    from paper_2501_07465_amd import pic
    w = _small("disk2d")
    w["sort_every"] = 1
    ref = oracle.build_workload(w)
    rng = np.random.default_rng(3)
    st = ref.state()
    perm = [rng.permutation(len(s[0])) for s in st]
    st = [(x[p], v[p], None if xi is None else xi[p], wt) for (x, v, xi, wt), p in zip(st, perm)]
    print("case sort order", flush=True)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=ref.fields(), graphs=False)
    ref2 = oracle.Sim(w)
    for sid, (x, v, xi, wt) in enumerate(st):
        ref2.add_species(w["species"][sid], wt, x, v, xi)
    keys_before = [sim.keys(sid) for sid in range(len(st))]
    for sid in range(len(st)):
        assert np.array_equal(keys_before[sid], ref2.keys(sid).astype(np.int64))
    sim.step(1)
    ref2.set_ion_background(False)
    ref2.set_fields(*ref.fields())
    ref2.step(1)
    for sid in range(len(st)):
        xg, vg, _ = sim.particles(sid)
        xr, vr, _ = ref2.particles(sid)
        # same order: every particle matches its counterpart
        assert _rel(vg, vr) < 1e-12
        assert float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) < 1e-12


def test_sort_of_many_keys_is_stable():
    """A sort over many blocks with several rounds of keys each (9M particles in random order on a
    periodic 64^3 grid: 18-bit keys, three 8-bit passes) leaves the particles in the order of a
    stable argsort of their cell keys, bit for bit.  Velocities and fields are zero, so the step
    that follows the sort moves nothing."""
    from paper_2501_07465_amd import pic
    from paper_2501_07465_amd import workloads as W
    w = W.sphere3d(n=64, steps=1)
    w["periodic"] = [1, 1, 1]
    w.pop("source")
    w["species"] = [W.free_electrons(1, 5.5, 300.0, reflect=False)]
    w["sort_every"] = 1
    w["ion"] = "uniform"
    n = 9_000_000
    rng = np.random.default_rng(11)
    x = rng.random((n, 3)) * (np.array(w["n"]) * np.array(w["dx"]))
    zero = np.zeros((3, 64, 64, 64))
    print("case sort of 9M keys", flush=True)
    sim = pic.Simulation(w, states=[(x, np.zeros((n, 3)), None, 1.0)], fields=(zero, zero), graphs=False)
    assert sim.shape() == (64, 64, 64)
    x0, _, _ = sim.particles(0)
    k0 = sim.keys(0)
    assert k0.max() >= 2 ** 16  # the third pass has digits to sort
    order = np.argsort(k0, kind="stable")
    sim.step(1)
    x1, v1, _ = sim.particles(0)
    assert not np.any(v1)
    assert np.array_equal(sim.keys(0), k0[order])
    assert np.array_equal(x1, x0[order])


@pytest.mark.parametrize("name,tile", [("disk2d", None), ("sheet2d", None), ("sphere3d", None), ("slab1d", None),
                                       # the tile shapes compiled with constant window geometry
                                       ("disk2d", [32, 32, 1]), ("sphere3d", [4, 4, 4])])
def test_fp32_one_step_push(oracle, name, tile):
    """FP32 form, one step from identical inputs (FP64 values rounded to FP32) within 1e-6."""
    from paper_2501_07465_amd import pic
    w = _small(name, fp64=False)
    if tile is not None:
        w["tile"] = list(tile)
    print(f"case fp32 one step {name} tile {w.get('tile')}", flush=True)
    base = oracle.build_workload(w)
    base.step(3)  # a state with non-zero fields
    st32 = []
    for x, v, xi, wt in base.state():
        dx = np.array(w["dx"])
        X = x / dx
        c = np.floor(X)
        off32 = (X - c).astype(np.float32).astype(np.float64)
        x32 = (c + off32) * dx
        st32.append((x32, v.astype(np.float32).astype(np.float64),
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
        vscale = np.max(np.linalg.norm(vr, axis=1)) if len(vr) else 1.0
        ev = float(np.max(np.abs(vg - vr)) / vscale) if len(vr) else 0.0
        ex = float(np.max(np.abs(xg - xr) / np.array(w["dx"]))) if len(xr) else 0.0
        print(f"fp32 {name} species {sid}: v err {ev:.2e} (of max speed), x err {ex:.2e} cells", flush=True)
        assert ev <= 1e-6 and ex <= 1e-6, (name, sid, ev, ex)


def test_continuity_and_gauss_on_device(oracle):
    from paper_2501_07465_amd import pic
    w = _small("disk2d")
    print("case continuity fp64", flush=True)
    sim = pic.Simulation(w, precision="fp64", track_continuity=True, graphs=False)
    g0, sc0 = sim.gauss_residual()
    assert g0 <= 1e-12 * sc0
    for _ in range(5):
        sim.step(1)
        r, sc = sim.continuity_residual()
        assert r <= 1e-12 * sc, (r, sc)
    g1, sc1 = sim.gauss_residual()
    assert g1 <= 1e-11 * sc1, (g1, sc1)
    # the device current matches the oracle's for the same state
    ref = oracle.build_workload(w)
    sim2 = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), track_continuity=True,
                          graphs=False)
    sim2.step(1)
    ref.step(1)
    assert _rel(sim2.current(), ref.current()) < 1e-12


def test_graphs_match_plain_launches(oracle):
    from paper_2501_07465_amd import pic
    w = _small("disk2d")
    print("case graphs", flush=True)
    ref = oracle.build_workload(w)
    a = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=True)
    b = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False)
    a.step(40)
    b.step(40)
    ea, _ = a.fields()
    eb, _ = b.fields()
    assert _rel(ea, eb) < 1e-12
    assert a.steps_done == b.steps_done == 40


def test_overflow_path_long_sort_period(oracle):
    """Particles that leave their tile window between sorts take the global path and stay exact."""
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("slab1d")
    w["sort_every"] = 10000
    w["tile"] = [16, 1, 1]
    ref = oracle.build_workload(w)
    st = ref.state()
    x, v, xi, wt = st[0]
    v = v * 60.0  # ~0.2 cells per step: particles cross tiles within the run
    st = [(x, v, xi, wt)]
    ref = oracle.Sim(w)
    ref.add_species(w["species"][0], wt, x, v)
    ref.set_ion_background(True)
    ref.gauss_init_1d()
    print("case overflow", flush=True)
    sim = pic.Simulation(w, precision="fp64", states=st, fields=ref.fields(), graphs=False)
    sim.step(30)
    ref.step(30)
    assert sim.overflow() > 0
    _compare(sim, ref, w, 1e-12, "fp64 overflow")


@pytest.mark.parametrize("name,unit", [("disk2d", 64), ("disk2d", 200), ("sheet2d", 96), ("sphere3d", 128)])
def test_fp64_tiles_split_into_units(oracle, name, unit):
    """Tiles whose particles are split over several blocks (one current slot per unit) stay exact."""
    from paper_2501_07465_amd import pic
    w = _small(name)
    print(f"case fp64 units {name} unit {unit}", flush=True)
    ref = oracle.build_workload(w)
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=True, unit=unit)
    sim.step(40)
    ref.step(40)
    _compare(sim, ref, w, 1e-12, f"fp64 units {name}")
