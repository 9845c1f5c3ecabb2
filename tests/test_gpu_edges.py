"""Edge cases of the HIP path against the FP64 oracle: no species at all, an empty species,
hand-placed degenerate particles (offsets exactly 0 and just below 1, particles at rest, fast
diagonal movers that cross cell corners and periodic seams, reflections), and grids at the largest
extents the packed cell index holds (x = 65535 cells in 2D, 2047 in 3D, with a ragged last tile).
FP64 form, element by element within 1e-12 of the oracle's scale; keys bit-exact.
"""
import copy

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rel(a, b, scale=None):
    scale = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(scale, 1e-300)) if np.size(a) else 0.0


def _compare(sim, ref, w, tol, label):
    for sid, sp in enumerate(w["species"]):
        xg, vg, xig = sim.particles(sid)
        xr, vr, xir = ref.particles(sid)
        assert xg.shape == xr.shape, label
        if not len(xg):
            continue
        dx = np.array(w["dx"])
        ex = float(np.max(np.abs(xg - xr) / dx))
        ev = _rel(vg, vr)
        print(f"{label} species {sid}: x err {ex:.2e} cells, v rel {ev:.2e}", flush=True)
        assert ex < tol and ev < tol, (label, sid, ex, ev)
        if sp["kind"] == "bound":
            assert _rel(xig, xir) < tol, (label, sid)
    eg, bg = sim.fields()
    er, br = ref.fields()
    ee = _rel(eg, er)
    eb = _rel(bg, br, max(np.max(np.abs(br)), np.max(np.abs(er)) / 3e8, 1e-300))
    print(f"{label} fields: E rel {ee:.2e}, B rel {eb:.2e}", flush=True)
    assert ee < tol and eb < tol, (label, ee, eb)


def _run_pair(oracle, w, states, steps, label, unit=0):
    """Oracle and FP64 GPU from the same hand-placed state; returns both after `steps`."""
    from paper_2501_07465_amd import pic
    ref = oracle.Sim(w)
    for sp, (x, v, xi, wt) in zip(w["species"], states):
        ref.add_species(sp, wt, x, v, xi)
    ref.set_ion_background(w.get("ion", "local") == "uniform")
    sim = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=False, unit=unit)
    for sid in range(len(w["species"])):
        assert np.array_equal(sim.keys(sid), ref.keys(sid)), (label, "keys", sid)
    sim.step(steps)
    ref.step(steps)
    return sim, ref


def test_vacuum_without_species(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    w["species"] = []
    print("case vacuum", flush=True)
    ref = oracle.Sim(w)
    sim = pic.Simulation(w, precision="fp64", fields=ref.fields(), graphs=True)
    sim.step(60)
    ref.step(60)
    _compare(sim, ref, w, 1e-12, "vacuum")
    assert np.max(np.abs(ref.fields()[0])) > 0  # the source radiated


def test_empty_species_beside_a_full_one(oracle):
    from paper_2501_07465_amd import pic, workloads as W
    w = W.small("disk2d")
    w["species"][0]["region"] = {"kind": "ball", "center": [36.5, 33.5, 0.0], "radius": 0.4}  # holds no cell
    print("case empty species", flush=True)
    ref = oracle.build_workload(w)
    assert ref.count(0) == 0 and ref.count(1) > 0
    sim = pic.Simulation(w, precision="fp64", graphs=True)
    assert sim.count(0) == 0
    sim2 = pic.Simulation(w, precision="fp64", states=ref.state(), fields=ref.fields(), graphs=True)
    sim2.step(40)
    ref.step(40)
    _compare(sim2, ref, w, 1e-12, "empty species")


def _degenerate_particles(w, n_per, speed_cells, rng):
    """Positions on faces, just below faces, at seams; velocities zero or fast along diagonals."""
    dims, dx, dt = w["dims"], np.array(w["dx"]), w["dt"]
    centre = np.array(w["species"][0]["region"].get("center", [w["n"][0] / 2, w["n"][1] / 2, w["n"][2] / 2]))
    xs, vs = [], []
    below_one = 1.0 - 2.0 ** -40
    for i in range(n_per):
        base = np.floor(centre[:3]) + rng.integers(-6, 7, size=3)
        off = [0.0, below_one, 0.5, 0.25][i % 4]
        X = base + off
        if i % 5 == 0:
            v = np.zeros(3)
        else:
            d = rng.choice([-1.0, 1.0], size=3)
            v = d * speed_cells * dx / dt
        for a in range(dims, 3):
            X[a] = 0.0
        xs.append(X * dx)
        vs.append(v)
    return np.array(xs), np.array(vs)


def test_degenerate_positions_and_fast_corner_crossings(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("disk2d")
    w["species"][0]["region"]["radius"] = 12.5  # reflections happen within the run
    rng = np.random.default_rng(5)
    x, v = _degenerate_particles(w, 160, 0.31, rng)
    sp = w["species"][0]
    wt = 1e3
    w["species"] = [sp]
    print("case degenerate 2D", flush=True)
    sim, ref = _run_pair(oracle, w, [(x, v, None, wt)], 40, "degenerate 2D")
    _compare(sim, ref, w, 1e-12, "degenerate 2D")


def test_periodic_seam_and_zero_velocity_1d(oracle):
    from paper_2501_07465_amd import workloads as W
    w = W.small("slab1d")
    n, dx, dt = w["n"][0], w["dx"][0], w["dt"]
    x = np.zeros((64, 3))
    v = np.zeros((64, 3))
    seam = [n - 1 + (1.0 - 2.0 ** -40), 0.0, n - 1e-9 / dx, 0.5, 1.0, n - 1.0]
    for i in range(64):
        x[i, 0] = seam[i % len(seam)] * dx
        v[i] = [((-1) ** i) * 0.27 * dx / dt * (i % 3), 1e5 * (i % 2), -2e5 * (i % 4 == 0)]
    sp = copy.deepcopy(w["species"][0])
    w["species"] = [sp]
    w["ion"] = "uniform"
    print("case periodic seam 1D", flush=True)
    sim, ref = _run_pair(oracle, w, [(x, v, None, 1e4)], 50, "seam 1D")
    _compare(sim, ref, w, 1e-12, "seam 1D")


def test_dirac_carriers_hand_placed(oracle):
    """Dirac carriers on the sheet with in-plane velocities in every direction: |v| = v_F and a zero
    normal component on both sides, trajectories within 1e-12."""
    from paper_2501_07465_amd import workloads as W
    w = W.small("sheet2d")
    sp = copy.deepcopy(w["species"][0])
    normal = sp["sheet_normal"]
    ny = w["species"][0]["region"]["lo"][normal] if sp["region"]["kind"] == "box" else 30
    x = np.zeros((32, 3))
    v = np.zeros((32, 3))
    for i in range(32):
        x[i, 0] = (10 + 2.5 * i) * w["dx"][0]
        x[i, normal] = (ny + 0.5) * w["dx"][normal]
        ang = 2 * np.pi * i / 32
        plane = [a for a in range(3) if a != normal]
        v[i, plane[0]] = sp["v_f"] * np.cos(ang)
        v[i, plane[1]] = sp["v_f"] * np.sin(ang)
    w["species"] = [sp]
    print("case dirac", flush=True)
    sim, ref = _run_pair(oracle, w, [(x, v, None, 1e3)], 40, "dirac")
    _compare(sim, ref, w, 1e-12, "dirac")
    _, vg, _ = sim.particles(0)
    assert np.allclose(np.linalg.norm(vg, axis=1), sp["v_f"], rtol=1e-14)
    assert np.all(vg[:, normal] == 0.0)


EXTENTS = {
    "x2d": (2, [65535, 16, 1], [16, 8, 1]),
    "y2d": (2, [16, 65535, 1], [8, 16, 1]),
    "x3d": (3, [2047, 8, 8], [8, 4, 4]),
    "z3d": (3, [8, 8, 1023], [4, 4, 8]),
}


@pytest.mark.parametrize("case", sorted(EXTENTS))
def test_largest_packed_extents(oracle, case):
    """Cells at the top of every field of the packed cell index (16 + 16 bits in 2D, 11 + 11 + 10 in
    3D, so the top field reaches the sign bit) on a periodic seam, with a ragged last tile."""
    from paper_2501_07465_amd import workloads as W
    dims, n, tile = EXTENTS[case]
    big = int(np.argmax(n))
    dxv = 1e-9
    w = {"name": f"extent-{case}", "dims": dims, "n": n, "dx": [dxv] * 3, "dt": W.cfl_dt(dxv, dims),
         "periodic": [1, 1, 1], "tile": tile, "sort_every": 20, "ion": "uniform", "steps": 40,
         "species": [W.free_electrons(4, region={"kind": "all"}, reflect=False),
                     W.bound_electrons(4, 4.0, 0.1, 5.9e28, {"kind": "all"})]}
    rng = np.random.default_rng(3)
    m = 96
    X = np.zeros((m, 3))
    for a in range(dims):
        X[:, a] = rng.uniform(0, n[a], m)
    X[:, big] = np.concatenate([rng.uniform(n[big] - 3, n[big], m // 2), rng.uniform(0, 3, m - m // 2)])
    x = X * dxv
    v = rng.normal(0, 3e5, size=(m, 3))
    v[::4, big] = 0.3 * dxv / w["dt"]  # seam crossings along the long axis
    xi = rng.uniform(-1e-11, 1e-11, size=(m, 3))
    states = [(x, v, None, 1e2), (x.copy(), np.zeros((m, 3)), xi, 1e2)]
    print(f"case extent {case} n {n} tile {tile}", flush=True)
    sim, ref = _run_pair(oracle, w, states, 40, f"extent {case}")
    _compare(sim, ref, w, 1e-12, f"extent {case}")
    for sid in range(2):
        assert np.array_equal(sim.keys(sid), ref.keys(sid))
