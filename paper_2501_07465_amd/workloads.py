"""Seeded synthetic workloads shaped like the paper's condensed-matter runs.

This module only describes inputs: grid sizes, cell sizes, time steps, species
parameters as the workload states them, geometry, sources and seeds.  It holds
none of the method's arithmetic (no Fermi-energy/density relation, no Dirac
mass, no pusher, no deposit) and imports nothing else from this package, so the
oracle side and the HIP side can both be fed from it.

Physical inputs in SI.  Geometry (region centres, radii, boxes, source
positions) in cell units.

Workloads (seed of workload i is 1 + i; request j of the serving stream uses
1000 + j):

* ``slab1d``    1D3V periodic slab, 256 cells of 0.5 nm, 64 FD free electrons per
  cell at n = 5.9e28 m^-3 (E_F = 5.5 eV, 300 K), quiet start with a 1e-3 density
  perturbation, 2000 steps, FP64.
* ``disk2d``    2D3V 1024 x 1024 cells of 1 nm with a 200 nm metal disk: 16 ppc
  FD free electrons plus 16 ppc bound Lorentz electrons (hbar omega0 = 4 eV,
  hbar gamma = 0.1 eV, displacement < 0.01 nm), reflecting disk edge, 800 nm
  plane-wave pulse at 1e9 V/m from the left, 4000 steps.
* ``sphere3d``  3D3V 256^3 cells of 1 nm, nanosphere radius 100 cells, 8 + 8 ppc,
  dipole pulse, 2000 steps.
* ``sheet2d``   2D3V 2048 x 512 cells of 0.5 nm: a one-cell Dirac sheet (v_F =
  1e6 m/s, E_F = 0.2 eV, 64 ppc) on a 100-cell bound substrate (hbar omega0 = 6 eV,
  16 ppc), 1 THz pulse at 1e7 V/m, 5000 steps.
* ``stream``    512 uneven 2D3V nanostructure requests with Poisson arrivals.

Readings that fix what the workload text leaves open (bound density equal to
the free density for the disk, substrate density for a static permittivity of
2.1, source placement and envelope) are listed with the rest of the design
notes; the numbers below are the chosen inputs.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Input constants (CODATA 2018).  Used only to express the inputs in SI
# (electron-volt energies, the CFL time step, the source amplitude).
QE = 1.602176634e-19
ME = 9.1093837015e-31
CLIGHT = 299792458.0
EPS0 = 8.8541878128e-12
HBAR = 1.054571817e-34
EV = QE
KB = 1.380649e-23


def cfl_dt(dx: float, dims: int, frac: float = 0.95) -> float:
    """Time step at ``frac`` of the vacuum Courant limit for uniform cells."""
    return frac * dx / (CLIGHT * math.sqrt(dims))


def sheet_current_amplitude(e0: float, dx: float) -> float:
    """Current density of a one-cell soft sheet that radiates a wave of amplitude e0 each way."""
    return 2.0 * EPS0 * CLIGHT * e0 / dx


def _source(kind, comp, axis, index, e0, wavelength=None, freq=None, periods=2.0, dx=1e-9):
    if wavelength is not None:
        omega = 2.0 * math.pi * CLIGHT / wavelength
    else:
        omega = 2.0 * math.pi * freq
    period = 2.0 * math.pi / omega
    return {"kind": kind, "comp": comp, "axis": axis, "index": list(index),
            "j0": sheet_current_amplitude(e0, dx), "omega": omega, "tau": periods * period}


def free_electrons(ppc, e_fermi_ev=5.5, temperature=300.0, density=0.0, region=None, reflect=True, **kw):
    d = {"kind": "free", "q": -QE, "m": ME, "ppc": ppc, "momentum": "fd",
         "e_fermi": e_fermi_ev * EV, "temperature": temperature, "density": density,
         "region": region or {"kind": "all"}, "reflect": reflect}
    d.update(kw)
    return d


def bound_electrons(ppc, omega0_ev, gamma_ev, density, region, xi_radius=0.01e-9, b_weight=0.0):
    w0 = omega0_ev * EV / HBAR
    g = gamma_ev * EV / HBAR
    return {"kind": "bound", "q": -QE, "m": ME, "ppc": ppc, "momentum": "cold",
            "omega0": [w0, w0, w0], "gamma": [g, g, g], "density": density,
            "xi_radius": xi_radius, "b_weight": b_weight, "region": region, "reflect": False}


def dirac_carriers(ppc, e_fermi_ev, v_f, temperature, region, sheet_normal):
    return {"kind": "dirac", "q": -QE, "m": 0.0, "ppc": ppc, "momentum": "fd",
            "e_fermi": e_fermi_ev * EV, "temperature": temperature, "v_f": v_f,
            "sheet_normal": sheet_normal, "region": region, "reflect": False, "density": 0.0}


# ---------------------------------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------------------------------
def slab1d(n=256, ppc=64, steps=2000):
    dx = 0.5e-9
    return {"name": "slab1d", "dims": 1, "n": [n, 1, 1], "dx": [dx, dx, dx], "dt": cfl_dt(dx, 1),
            "periodic": [1, 1, 1], "tile": [64, 1, 1], "sort_every": 20,
            "species": [free_electrons(ppc, 5.5, 300.0, density=5.9e28, reflect=False,
                                       loading="quiet", pert_amp=1e-3, pert_mode=1)],
            "ion": "uniform", "gauss_init": True, "steps": steps, "seed": 1, "precision": "fp64"}


def disk2d(n=1024, radius=100.0, ppc_free=16, ppc_bound=16, steps=4000, tile=(16, 16), src_x=8):
    dx = 1e-9
    c = n / 2.0
    disk = {"kind": "ball", "center": [c, c, 0.0], "radius": radius}
    return {"name": "disk2d", "dims": 2, "n": [n, n, 1], "dx": [dx, dx, dx], "dt": cfl_dt(dx, 2),
            "periodic": [0, 1, 1], "tile": [tile[0], tile[1], 1], "sort_every": 20,
            "source": _source("sheet", 1, 0, [src_x, 0, 0], 1e9, wavelength=800e-9, dx=dx),
            "species": [free_electrons(ppc_free, 5.5, 300.0, region=disk, reflect=True),
                        bound_electrons(ppc_bound, 4.0, 0.1, 5.9e28, disk)],
            "ion": "local", "steps": steps, "seed": 2, "precision": "fp32"}


def sphere3d(n=256, radius=100.0, ppc_free=8, ppc_bound=8, steps=2000, tile=(8, 8, 4), src_gap=14):
    dx = 1e-9
    c = n / 2.0
    ball = {"kind": "ball", "center": [c, c, c], "radius": radius}
    src_z = int(c + radius + src_gap)
    return {"name": "sphere3d", "dims": 3, "n": [n, n, n], "dx": [dx, dx, dx], "dt": cfl_dt(dx, 3),
            "periodic": [0, 0, 0], "tile": list(tile), "sort_every": 20,
            "source": _source("point", 2, 2, [int(c), int(c), src_z], 1e9, wavelength=800e-9, dx=dx),
            "species": [free_electrons(ppc_free, 5.5, 300.0, region=ball, reflect=True),
                        bound_electrons(ppc_bound, 4.0, 0.1, 5.9e28, ball)],
            "ion": "local", "steps": steps, "seed": 3, "precision": "fp32"}


def sheet2d(nx=2048, ny=512, sheet_y=300, substrate=100, ppc_sheet=64, ppc_bound=16, steps=5000,
            tile=(16, 16), src_y=500):
    dx = 0.5e-9
    sheet = {"kind": "box", "lo": [0.0, float(sheet_y), 0.0], "hi": [float(nx), float(sheet_y + 1), 1.0]}
    slab = {"kind": "box", "lo": [0.0, float(sheet_y - substrate), 0.0], "hi": [float(nx), float(sheet_y), 1.0]}
    return {"name": "sheet2d", "dims": 2, "n": [nx, ny, 1], "dx": [dx, dx, dx], "dt": cfl_dt(dx, 2),
            "periodic": [1, 0, 1], "tile": [tile[0], tile[1], 1], "sort_every": 20,
            "source": _source("sheet", 0, 1, [0, src_y, 0], 1e7, freq=1e12, dx=dx),
            "species": [dirac_carriers(ppc_sheet, 0.2, 1e6, 300.0, sheet, sheet_normal=1),
                        bound_electrons(ppc_bound, 6.0, 0.1, 2.87e28, slab)],
            "ion": "local", "steps": steps, "seed": 4, "precision": "fp32"}


def stream_request(j: int, rng_seed_base: int = 1000, scale: float = 1.0):
    """Request j of the serving stream: a seeded uneven 2D3V nanostructure simulation.

    Grid side uniform in [128, 1024] cells (times ``scale``); disk, rod or slab
    geometry with seeded dimensions; 8-32 ppc free FD electrons plus 8-32 ppc bound
    electrons; 500-4000 steps (a multiple of the 20-step sort period).
    """
    rng = np.random.default_rng(rng_seed_base + j)
    n = int(rng.integers(128, 1025))
    n = max(32, int(round(n * scale)) // 16 * 16)
    geom = ["disk", "rod", "slab"][int(rng.integers(0, 3))]
    ppc_f = int(rng.integers(8, 33))
    ppc_b = int(rng.integers(8, 33))
    steps = 20 * int(rng.integers(25, 201))  # 500..4000, a whole number of sort periods
    c = n / 2.0
    if geom == "disk":
        d = float(rng.uniform(0.2, 0.6)) * n
        region = {"kind": "ball", "center": [c, c, 0.0], "radius": d / 2.0}
    elif geom == "rod":
        L = float(rng.uniform(0.3, 0.7)) * n
        W = float(rng.uniform(0.05, 0.2)) * n
        region = {"kind": "box", "lo": [c - L / 2, c - W / 2, 0.0], "hi": [c + L / 2, c + W / 2, 1.0]}
    else:
        t = float(rng.uniform(0.05, 0.3)) * n
        H = 0.8 * n
        region = {"kind": "box", "lo": [c - t / 2, c - H / 2, 0.0], "hi": [c + t / 2, c + H / 2, 1.0]}
    w = disk2d(n=n, ppc_free=ppc_f, ppc_bound=ppc_b, steps=steps)
    w["name"] = f"stream{j}"
    w["geometry"] = geom
    w["species"][0]["region"] = region
    w["species"][1]["region"] = copy.deepcopy(region)
    w["seed"] = rng_seed_base + j
    return w


def stream(n_requests=512, rate_hz=None, seed=7, scale=1.0):
    """Requests with Poisson arrival times (seconds); ``rate_hz`` None means all at t = 0."""
    rng = np.random.default_rng(seed)
    reqs = [stream_request(j, scale=scale) for j in range(n_requests)]
    if rate_hz:
        t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_requests))
    else:
        t = np.zeros(n_requests)
    for r, a in zip(reqs, t):
        r["arrival"] = float(a)
    return reqs


def with_dielectric(w: dict, eps, region=None) -> dict:
    """A copy of workload w with a constant background permittivity inside region (default: the
    region of the first species), vacuum elsewhere.  eps is [eps_x, eps_y, eps_z] (a diagonal
    tensor) or a 3x3 tensor (its inverse then has off-diagonal entries)."""
    w = copy.deepcopy(w)
    e = np.asarray(eps, dtype=float)
    w["dielectric"] = {"eps": e.tolist(),
                       "region": copy.deepcopy(region or w["species"][0]["region"])}
    w["name"] = w["name"] + "_eps"
    return w


def with_diffuse_walls(w: dict) -> dict:
    """A copy of workload w whose reflecting species scatter diffusively (cosine law) instead of
    specularly at their region boundary."""
    w = copy.deepcopy(w)
    for sp in w["species"]:
        if sp.get("reflect"):
            sp["scatter"] = "diffuse"
    w["name"] = w["name"] + "_diffuse"
    return w


def with_potential_wall(w: dict, height_ev: float, width: float, region=None) -> dict:
    """A copy of workload w whose free species are held by a static work-function barrier instead
    of reflecting walls: the potential energy of an electron rises by height_ev linearly over
    `width` cells outside region (default: the first species' region).  The grid becomes periodic
    on every axis (free particles without walls may reach any cell)."""
    w = copy.deepcopy(w)
    w["wall"] = {"height_ev": float(height_ev), "width": float(width),
                 "region": copy.deepcopy(region or w["species"][0]["region"])}
    for sp in w["species"]:
        if sp["kind"] == "free":
            sp["reflect"] = False
    w["periodic"] = [1, 1, 1]
    w["name"] = w["name"] + "_wall"
    return w


def wall_field(w: dict):
    """The barrier field at the E nodes ([3][L2][L1][L0], V/m): E = -grad phi on the grid, with the
    node potential phi = -height_ev * clamp(d / width, 0, 1) volts and d the distance (cells) of
    the node outside the region (so an electron's energy -e phi rises by height_ev eV).  Component
    c at node i holds -(phi(i + e_c) - phi(i)) / dx_c (wrapped on periodic axes, 0 on the padding
    index of an open axis and on inactive axes).  None without a wall."""
    d = w.get("wall")
    if d is None:
        return None
    L = field_extent(w)
    dims = w["dims"]
    kk, jj, ii = np.meshgrid(np.arange(L[2], dtype=float), np.arange(L[1], dtype=float),
                             np.arange(L[0], dtype=float), indexing="ij")
    pos = [ii, jj, kk]
    reg = d["region"]
    if reg["kind"] == "ball":
        dist = np.sqrt(sum((pos[a] - reg["center"][a]) ** 2 for a in range(dims))) - reg["radius"]
    elif reg["kind"] == "box":
        out = np.zeros_like(ii)
        for a in range(dims):
            g = np.maximum(np.maximum(reg["lo"][a] - pos[a], pos[a] - reg["hi"][a]), 0.0)
            out = out + g * g
        dist = np.sqrt(out)
    else:
        dist = np.full_like(ii, -1.0)
    phi = -d["height_ev"] * np.clip(dist / d["width"], 0.0, 1.0)
    e = np.zeros((3,) + phi.shape)
    for c in range(dims):
        ax = 2 - c  # arrays are [z, y, x]
        if w["periodic"][c]:
            e[c] = -(np.roll(phi, -1, axis=ax) - phi) / w["dx"][c]
        else:
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[ax] = slice(0, L[c] - 1)
            sl_hi[ax] = slice(1, L[c])
            e[c][tuple(sl_lo)] = -(phi[tuple(sl_hi)] - phi[tuple(sl_lo)]) / w["dx"][c]
    return e


def field_extent(w: dict):
    """Array extent per axis of a field component: n on periodic and inactive axes, n + 1 on open ones."""
    return [w["n"][a] + (1 if a < w["dims"] and not w["periodic"][a] else 0) for a in range(3)]


def _eps_inverse(d: dict):
    """The inverse permittivity tensor of a dielectric description (diagonal or 3x3)."""
    e = np.asarray(d["eps"], dtype=float)
    return np.diag(1.0 / e) if e.ndim == 1 else np.linalg.inv(e)


def _inside(w: dict, reg: dict, c: int):
    """Mask of the E_c nodes ([L2][L1][L0]) inside region reg."""
    L = field_extent(w)
    dims = w["dims"]
    kk, jj, ii = np.meshgrid(np.arange(L[2], dtype=float), np.arange(L[1], dtype=float),
                             np.arange(L[0], dtype=float), indexing="ij")
    pos = [ii, jj, kk]
    if c < dims:
        pos[c] = pos[c] + 0.5
    if reg["kind"] == "ball":
        r2 = sum((pos[a] - reg["center"][a]) ** 2 for a in range(dims))
        return r2 <= reg["radius"] ** 2
    if reg["kind"] == "box":
        inside = np.ones_like(ii, dtype=bool)
        for a in range(dims):
            inside &= (pos[a] >= reg["lo"][a]) & (pos[a] < reg["hi"][a])
        return inside
    return np.ones_like(ii, dtype=bool)


def eps_offdiag_map(w: dict):
    """Off-diagonal inverse permittivity ([6][L2][L1][L0], row a, column b != a at the E_a node, in
    the order 01 02 10 12 20 21) of a full-tensor dielectric inside its region.  Entries within two
    nodes of an open face are left zero (the media end before the absorbing faces).  None when the
    workload has no dielectric or a diagonal one."""
    d = w.get("dielectric")
    if d is None or np.asarray(d["eps"]).ndim == 1:
        return None
    inv = _eps_inverse(d)
    L = field_extent(w)
    keep = np.ones((L[2], L[1], L[0]), dtype=bool)
    for a in range(w["dims"]):
        if not w["periodic"][a]:
            idx = np.arange(L[a])
            ok = (idx >= 2) & (idx <= w["n"][a] - 2)
            shape = [1, 1, 1]
            shape[2 - a] = L[a]
            keep &= ok.reshape(shape)
    out = np.zeros((6, L[2], L[1], L[0]))
    m = 0
    for a in range(3):
        mask = _inside(w, d["region"], a) & keep
        for b in range(3):
            if b == a:
                continue
            out[m][mask] = inv[a, b]
            m += 1
    return out


def eps_inv_map(w: dict):
    """Inverse permittivity per E component at its Yee node ([3][L2][L1][L0]): the diagonal entry
    (eps^-1)_cc where the node (half-integer along c, integer along the other active axes, in cell
    units) lies in the dielectric region, 1 elsewhere.  None when the workload has no dielectric."""
    d = w.get("dielectric")
    if d is None:
        return None
    inv = _eps_inverse(d)
    out = np.ones([3] + field_extent(w)[::-1])
    for c in range(3):
        out[c][_inside(w, d["region"], c)] = inv[c, c]
    return out


# Fermi energies E_F = hbar^2 (3 pi^2 n)^(2/3) / (2 m_e) of the relaxation study's densities, stated
# here as inputs (eV; the tests check them against the closed form).
RELAX_EF_EV = {2e28: 2.6867273755, 4e28: 4.2649138622, 6e28: 5.5886181507}


def relax3d(density=6e28, ppc=128, n=16, box_nm=2.0, temperature_ev=0.0375, t_end_fs=20.0, tile=(8, 8, 4)):
    """The FD relaxation study (Sec. 2): a periodic 2 nm cube of bulk free electrons (fixed uniform
    ions), random positions, Fermi-Dirac momenta at 0.0375 eV with mu = E_F of the density, run for
    t_end_fs; the kinetic-energy tail is fitted to exp(-E / beta) along the run."""
    dx = box_nm * 1e-9 / n
    dt = cfl_dt(dx, 3)
    return {"name": "relax3d", "dims": 3, "n": [n, n, n], "dx": [dx, dx, dx], "dt": dt,
            "periodic": [1, 1, 1], "tile": list(tile), "sort_every": 20,
            "species": [free_electrons(ppc, RELAX_EF_EV[density], temperature_ev * EV / KB,
                                       density=density, reflect=False)],
            "ion": "uniform", "steps": int(round(t_end_fs * 1e-15 / dt / 20.0)) * 20, "seed": 5,
            "precision": "fp32", "relax": {"density": density, "temperature_ev": temperature_ev}}


WORKLOADS = {"slab1d": slab1d, "disk2d": disk2d, "sphere3d": sphere3d, "sheet2d": sheet2d, "relax3d": relax3d}


# ---------------------------------------------------------------------------------------------------
# Small variants for parity tests: several tiles and a ragged tail, oracle-fast.
# ---------------------------------------------------------------------------------------------------
def small(name: str):
    if name == "slab1d":
        return slab1d(n=64, ppc=16, steps=100)
    if name == "disk2d":
        w = disk2d(n=72, radius=20.5, ppc_free=6, ppc_bound=5, steps=40, tile=(16, 8), src_x=6)
        w["n"] = [72, 68, 1]
        w["species"][0]["region"]["center"] = [36.3, 33.7, 0.0]
        w["species"][1]["region"]["center"] = [36.3, 33.7, 0.0]
        return w
    if name == "sphere3d":
        w = sphere3d(n=40, radius=11.5, ppc_free=3, ppc_bound=2, steps=20, tile=(8, 8, 4), src_gap=3)
        w["n"] = [40, 36, 44]
        for sp in w["species"]:
            sp["region"]["center"] = [20.2, 18.1, 21.7]
        w["source"]["index"] = [20, 18, 37]
        return w
    if name == "relax3d":
        return relax3d(ppc=8, n=8, box_nm=1.0, t_end_fs=0.5, tile=(4, 4, 4))
    if name == "sheet2d":
        return sheet2d(nx=100, ny=60, sheet_y=30, substrate=10, ppc_sheet=8, ppc_bound=4, steps=40,
                       tile=(16, 8), src_y=50)
    raise KeyError(name)


def random_particles(w: dict, n: int, seed: int, speed: float = 1.4e6, region_margin: float = 3.0):
    """Seeded random positions (metres) and velocities (m/s) inside the domain, away from open faces."""
    rng = np.random.default_rng(seed)
    dims = w["dims"]
    x = np.zeros((n, 3))
    for a in range(dims):
        lo = 0.0 if w["periodic"][a] else region_margin
        hi = w["n"][a] - (0.0 if w["periodic"][a] else region_margin)
        x[:, a] = rng.uniform(lo, hi, size=n) * w["dx"][a]
    v = rng.normal(size=(n, 3))
    v *= speed / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.1, 1.0, size=(n, 1))
    return x, v
