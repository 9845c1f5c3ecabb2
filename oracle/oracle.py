"""ctypes wrapper of the plain FP64 CPU oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  The product path (the HIP library and
its binding) never imports this module.  From the product package this module
imports only ``workloads``, the seeded input generator shared by both sides,
which holds none of the method's arithmetic (it draws the inverse-permittivity
and wall-field inputs that both sides load).

Workloads arrive as plain dicts (see ``paper_2501_07465_amd.workloads``); every
derived quantity that belongs to the method (density from E_F, Dirac mass,
omega_b^2) is computed here through the oracle's own C functions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "libpic_oracle.so")

FREE, BOUND, DIRAC = 0, 1, 2
_KIND = {"free": FREE, "bound": BOUND, "dirac": DIRAC}
_REGION = {"all": 0, "ball": 1, "box": 2}
_SRC_KIND = {"none": 0, "sheet": 1, "point": 2}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", _LIB, _SRC, "-lm"],
            cwd=_HERE)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("dims", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3), ("dt", C.c_double),
                ("periodic", C.c_int * 3), ("tile", C.c_int * 3), ("sort_every", C.c_int),
                ("src_kind", C.c_int), ("src_comp", C.c_int), ("src_axis", C.c_int),
                ("src_index", C.c_int * 3), ("src_j0", C.c_double), ("src_omega", C.c_double),
                ("src_tau", C.c_double)]


class Species(C.Structure):
    _fields_ = [("kind", C.c_int), ("q", C.c_double), ("m", C.c_double), ("weight", C.c_double),
                ("omega0_sq", C.c_double * 3), ("gamma", C.c_double * 3), ("b_weight", C.c_double),
                ("v_f", C.c_double), ("sheet_normal", C.c_int), ("reflect", C.c_int),
                ("region", C.c_int), ("rc", C.c_double * 3), ("rr", C.c_double),
                ("rlo", C.c_double * 3), ("rhi", C.c_double * 3), ("seed", C.c_uint64),
                ("mass_per_particle", C.c_int)]


class Init(C.Structure):
    _fields_ = [("ppc", C.c_int), ("momentum", C.c_int), ("e_fermi", C.c_double),
                ("temperature", C.c_double), ("density", C.c_double), ("loading", C.c_int),
                ("pert_amp", C.c_double), ("pert_mode", C.c_int), ("xi_radius", C.c_double),
                ("seed", C.c_uint64)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.or_const.restype = C.c_double
        for name in ("or_fermi_energy", "or_density_from_fermi", "or_dirac_mass", "or_dirac_density2d"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double]
        L.or_dt_limit.restype = C.c_double
        L.or_dt_limit.argtypes = [C.c_double, C.c_double, _D, C.c_int]
        L.or_u53.restype = C.c_double
        L.or_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.or_push_free.argtypes = [C.c_double, C.c_double, _D, _D, _D]
        L.or_push_bound.argtypes = [C.c_double, C.c_double, _D, _D, C.c_double, _D, _D, _D, _D]
        L.or_push_dirac.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, _D, _D, _D]
        L.or_boris_matrix.argtypes = [_D, _D]
        L.or_gyro_matrix.argtypes = [_D, _D, _D]
        L.or_reflect.argtypes = [C.POINTER(Species), C.c_int, _D, _D]
        L.or_lambert.argtypes = [_D, _D, _D]
        L.or_lambert2d.argtypes = [_D, C.c_int, _D, _D]
        L.or_scatter_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _D]
        L.or_fd_sample_speeds.argtypes = [C.c_double, C.c_double, C.c_double, C.c_size_t, _D, _D]
        L.or_dirac_sample_energies.argtypes = [C.c_double, C.c_double, C.c_size_t, _D, _D]
        L.or_create.argtypes = [C.POINTER(Grid), C.POINTER(C.c_void_p)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_add_species.argtypes = [C.c_void_p, C.POINTER(Species), C.c_size_t, _D, _D, _D]
        L.or_init_species.argtypes = [C.c_void_p, C.POINTER(Species), C.POINTER(Init), C.POINTER(C.c_int)]
        L.or_species_weight.restype = C.c_double
        L.or_species_weight.argtypes = [C.c_void_p, C.c_int]
        L.or_count.restype = C.c_size_t
        L.or_count.argtypes = [C.c_void_p, C.c_int]
        L.or_get_particles.argtypes = [C.c_void_p, C.c_int, _D, _D, _D]
        L.or_keys.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int32)]
        L.or_field_len.restype = C.c_size_t
        L.or_field_len.argtypes = [C.c_void_p]
        L.or_field_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
        L.or_get_fields.argtypes = [C.c_void_p, _D, _D]
        L.or_set_fields.argtypes = [C.c_void_p, _D, _D]
        L.or_set_eps_inv.argtypes = [C.c_void_p, _D]
        L.or_set_eps_offdiag.argtypes = [C.c_void_p, _D]
        L.or_set_ext_field.argtypes = [C.c_void_p, _D]
        L.or_energy_histogram.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
        L.or_get_current.argtypes = [C.c_void_p, _D]
        L.or_get_rho.argtypes = [C.c_void_p, _D]
        L.or_gather_at.argtypes = [C.c_void_p, _D, _D, _D]
        L.or_set_ion_background.argtypes = [C.c_void_p, C.c_int]
        L.or_gauss_init_1d.argtypes = [C.c_void_p]
        L.or_step.argtypes = [C.c_void_p, C.c_int]
        L.or_track_continuity.argtypes = [C.c_void_p, C.c_int]
        L.or_sort.argtypes = [C.c_void_p]
        L.or_steps_done.restype = C.c_long
        L.or_steps_done.argtypes = [C.c_void_p]
        L.or_field_energy.restype = C.c_double
        L.or_field_energy.argtypes = [C.c_void_p]
        L.or_kinetic_energy.restype = C.c_double
        L.or_kinetic_energy.argtypes = [C.c_void_p, C.c_int]
        L.or_gauss_residual.restype = C.c_double
        L.or_gauss_residual.argtypes = [C.c_void_p, _D]
        L.or_current_series.argtypes = [C.c_void_p, _D, C.c_size_t, C.POINTER(C.c_size_t)]
        L.or_last_continuity_residual.restype = C.c_double
        L.or_last_continuity_residual.argtypes = [C.c_void_p, _D]
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _v3(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


def const(i: int) -> float:
    return lib().or_const(i)


# ---- single-particle building blocks -------------------------------------------------------------
def push_free(qm, dt, E, B, v):
    v = _v3(v).copy()
    lib().or_push_free(qm, dt, _dp(_v3(E)), _dp(_v3(B)), _dp(v))
    return v


def push_bound(qm, dt, w2, gam, bw, E, B, xi, v):
    v = _v3(v).copy()
    lib().or_push_bound(qm, dt, _dp(_v3(w2)), _dp(_v3(gam)), bw, _dp(_v3(E)), _dp(_v3(B)), _dp(_v3(xi)), _dp(v))
    return v


def push_dirac(qm, dt, v_f, normal, E, B, v):
    v = _v3(v).copy()
    lib().or_push_dirac(qm, dt, v_f, normal, _dp(_v3(E)), _dp(_v3(B)), _dp(v))
    return v


def lambert(n, u, v):
    n = _v3(n); u = np.ascontiguousarray(u, dtype=np.float64); v = _v3(v).copy()
    lib().or_lambert(_dp(n), _dp(u), _dp(v))
    return v


def lambert2d(n, normal, u, v):
    n = _v3(n); u = np.ascontiguousarray(u, dtype=np.float64); v = _v3(v).copy()
    lib().or_lambert2d(_dp(n), normal, _dp(u), _dp(v))
    return v


def scatter_uniforms(seed, p, step, sid):
    u = np.zeros(2)
    lib().or_scatter_uniforms(seed, p, step, sid, _dp(u))
    return u


def boris_matrix(b):
    R = np.zeros(9)
    lib().or_boris_matrix(_dp(_v3(b)), _dp(R))
    return R.reshape(3, 3)


def gyro_matrix(b, g):
    R = np.zeros(9)
    lib().or_gyro_matrix(_dp(_v3(b)), _dp(_v3(g)), _dp(R))
    return R.reshape(3, 3)


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def u53(a, b):
    return lib().or_u53(a, b)


def fd_speeds(e_fermi, kT, mass, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().or_fd_sample_speeds(e_fermi, kT, mass, u.size, _dp(u), _dp(out))
    return out


def dirac_energies(ef, kT, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    lib().or_dirac_sample_energies(ef, kT, u.size, _dp(u), _dp(out))
    return out


def fermi_energy(n, m):
    return lib().or_fermi_energy(n, m)


def density_from_fermi(ef, m):
    return lib().or_density_from_fermi(ef, m)


def dirac_mass(ef, vf):
    return lib().or_dirac_mass(ef, vf)


def dirac_density2d(ef, vf):
    return lib().or_dirac_density2d(ef, vf)


def dt_limit(omega_b, omega_p, dx, dims):
    d = np.ascontiguousarray(np.asarray(dx, dtype=np.float64).reshape(3))
    return lib().or_dt_limit(omega_b, omega_p, _dp(d), dims)


def make_species(sp: dict, dims: int) -> Species:
    """Species descriptor from a workload species dict (derived values via the oracle)."""
    s = Species()
    s.kind = _KIND[sp["kind"]]
    s.q = sp["q"]
    m = sp.get("m", 0.0)
    if s.kind == DIRAC and not m:
        m = dirac_mass(sp["e_fermi"], sp["v_f"])
    s.m = m
    s.weight = sp.get("weight", 0.0)
    w0 = sp.get("omega0", [0.0, 0.0, 0.0])
    g = sp.get("gamma", [0.0, 0.0, 0.0])
    for a in range(3):
        s.omega0_sq[a] = w0[a] * w0[a]
        s.gamma[a] = g[a]
    s.b_weight = sp.get("b_weight", 0.0)
    s.v_f = sp.get("v_f", 0.0)
    s.sheet_normal = sp.get("sheet_normal", -1)
    s.reflect = (2 if sp.get("scatter", "specular") == "diffuse" else 1) if sp.get("reflect", False) else 0
    s.mass_per_particle = int(bool(sp.get("mass_per_particle", False)))
    reg = sp.get("region", {"kind": "all"})
    s.region = _REGION[reg["kind"]]
    for a in range(3):
        s.rc[a] = reg.get("center", [0, 0, 0])[a]
        s.rlo[a] = reg.get("lo", [0, 0, 0])[a]
        s.rhi[a] = reg.get("hi", [0, 0, 0])[a]
    s.rr = reg.get("radius", 0.0)
    return s


def make_grid(w: dict) -> Grid:
    g = Grid()
    g.dims = w["dims"]
    for a in range(3):
        g.n[a] = w["n"][a]
        g.dx[a] = w["dx"][a]
        g.periodic[a] = int(w["periodic"][a])
        g.tile[a] = w["tile"][a]
    g.dt = w["dt"]
    g.sort_every = w.get("sort_every", 20)
    src = w.get("source", {"kind": "none"})
    g.src_kind = _SRC_KIND[src["kind"]]
    if g.src_kind:
        g.src_comp = src["comp"]
        g.src_axis = src.get("axis", 0)
        for a in range(3):
            g.src_index[a] = src["index"][a]
        g.src_j0 = src["j0"]
        g.src_omega = src["omega"]
        g.src_tau = src["tau"]
    return g


class Sim:
    """One oracle simulation."""

    def __init__(self, w: dict):
        self.w = w
        self.h = C.c_void_p()
        g = make_grid(w)
        r = lib().or_create(C.byref(g), C.byref(self.h))
        if r:
            raise RuntimeError(f"or_create failed ({r})")
        self.dims = w["dims"]
        self.species = []

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    # -- particles ------------------------------------------------------------------------------
    def init_species(self, sp: dict, seed: int) -> int:
        s = make_species(sp, self.dims)
        s.seed = seed
        ini = Init()
        ini.ppc = sp["ppc"]
        ini.momentum = 1 if sp.get("momentum", "fd") == "fd" else 0
        ini.e_fermi = sp.get("e_fermi", 0.0)
        ini.temperature = sp.get("temperature", 0.0)
        ini.density = sp.get("density", 0.0)
        ini.loading = 1 if sp.get("loading", "random") == "quiet" else 0
        ini.pert_amp = sp.get("pert_amp", 0.0)
        ini.pert_mode = sp.get("pert_mode", 1)
        ini.xi_radius = sp.get("xi_radius", 0.0)
        ini.seed = seed
        sid = C.c_int(-1)
        r = lib().or_init_species(self.h, C.byref(s), C.byref(ini), C.byref(sid))
        if r:
            raise RuntimeError(f"or_init_species failed ({r})")
        self.species.append(sp)
        return sid.value

    def add_species(self, sp: dict, weight: float, x, v, xi=None, seed: int | None = None) -> int:
        s = make_species(sp, self.dims)
        s.seed = self.w.get("seed", 1) if seed is None else seed
        s.weight = weight
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        xip = None
        if xi is not None:
            xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
            xip = _dp(xi)
        r = lib().or_add_species(self.h, C.byref(s), n, _dp(x), _dp(v), xip)
        if r < 0:
            raise RuntimeError(f"or_add_species failed ({r})")
        self.species.append(sp)
        return r

    def count(self, sid):
        return lib().or_count(self.h, sid)

    def weight(self, sid):
        return lib().or_species_weight(self.h, sid)

    def state(self):
        """(x, v, xi or None, weight) per species, for injecting the same state elsewhere."""
        out = []
        for sid, sp in enumerate(self.species):
            x, v, xi = self.particles(sid)
            keep = sp["kind"] == "bound" or (sp["kind"] == "dirac" and sp.get("mass_per_particle"))
            out.append((x, v, xi if keep else None, self.weight(sid)))
        return out

    def particles(self, sid):
        n = self.count(sid)
        x = np.zeros((n, 3)); v = np.zeros((n, 3)); xi = np.zeros((n, 3))
        lib().or_get_particles(self.h, sid, _dp(x), _dp(v), _dp(xi))
        return x, v, xi

    def keys(self, sid):
        n = self.count(sid)
        k = np.zeros(n, dtype=np.int32)
        lib().or_keys(self.h, sid, k.ctypes.data_as(C.POINTER(C.c_int32)))
        return k

    # -- fields ---------------------------------------------------------------------------------
    def shape(self):
        L = (C.c_int * 3)()
        lib().or_field_shape(self.h, L)
        return tuple(L)

    def fields(self):
        n = lib().or_field_len(self.h)
        e = np.zeros(3 * n); b = np.zeros(3 * n)
        lib().or_get_fields(self.h, _dp(e), _dp(b))
        L = self.shape()
        return e.reshape(3, L[2], L[1], L[0]), b.reshape(3, L[2], L[1], L[0])

    def set_fields(self, e, b):
        e = np.ascontiguousarray(e, dtype=np.float64).ravel()
        b = np.ascontiguousarray(b, dtype=np.float64).ravel()
        lib().or_set_fields(self.h, _dp(e), _dp(b))

    def energy_histogram(self, sid, e_max, nbins):
        """Macroparticle kinetic-energy histogram: nbins bins over [0, e_max) J, then the overflow."""
        out = np.zeros(nbins + 1, dtype=np.uint64)
        r = lib().or_energy_histogram(self.h, sid, e_max, nbins, out.ctypes.data_as(C.POINTER(C.c_uint64)))
        if r:
            raise ValueError("or_energy_histogram failed")
        return out

    def set_ext_field(self, e):
        """Static external field e[3][L] at the E_c nodes (Sec. 3 work-function barrier); None
        removes it."""
        if e is None:
            rc = lib().or_set_ext_field(self.h, None)
        else:
            e = np.ascontiguousarray(e, dtype=np.float64).ravel()
            rc = lib().or_set_ext_field(self.h, _dp(e))
        if rc != 0:
            raise ValueError("or_set_ext_field failed (%d)" % rc)

    def set_eps_inv(self, einv):
        """Diagonal inverse permittivity einv[3][L] at the E_c nodes (Sec. 4,
        eq:consteps); None restores the unit tensor."""
        if einv is None:
            rc = lib().or_set_eps_inv(self.h, None)
        else:
            einv = np.ascontiguousarray(einv, dtype=np.float64).ravel()
            rc = lib().or_set_eps_inv(self.h, _dp(einv))
        if rc != 0:
            raise ValueError("or_set_eps_inv failed (%d)" % rc)

    def set_eps_offdiag(self, eoff):
        """Off-diagonal inverse permittivity eoff[6][L] (row a, column b != a at the E_a node, order
        01 02 10 12 20 21; eq:consteps with a full tensor); None removes it."""
        if eoff is None:
            rc = lib().or_set_eps_offdiag(self.h, None)
        else:
            eoff = np.ascontiguousarray(eoff, dtype=np.float64).ravel()
            rc = lib().or_set_eps_offdiag(self.h, _dp(eoff))
        if rc != 0:
            raise ValueError("or_set_eps_offdiag failed (%d)" % rc)

    def current(self):
        n = lib().or_field_len(self.h)
        j = np.zeros(3 * n)
        lib().or_get_current(self.h, _dp(j))
        L = self.shape()
        return j.reshape(3, L[2], L[1], L[0])

    def rho(self):
        n = lib().or_field_len(self.h)
        r = np.zeros(n)
        lib().or_get_rho(self.h, _dp(r))
        L = self.shape()
        return r.reshape(L[2], L[1], L[0])

    def gather_at(self, x):
        E = np.zeros(3); B = np.zeros(3)
        lib().or_gather_at(self.h, _dp(_v3(x)), _dp(E), _dp(B))
        return E, B

    def set_ion_background(self, uniform: bool):
        lib().or_set_ion_background(self.h, int(uniform))

    def gauss_init_1d(self):
        r = lib().or_gauss_init_1d(self.h)
        if r:
            raise RuntimeError("or_gauss_init_1d failed")

    def track_continuity(self, on=True):
        lib().or_track_continuity(self.h, int(on))

    def step(self, n=1):
        r = lib().or_step(self.h, n)
        if r:
            raise RuntimeError(f"or_step failed ({r})")

    def sort(self):
        lib().or_sort(self.h)

    # -- diagnostics ----------------------------------------------------------------------------
    def field_energy(self):
        return lib().or_field_energy(self.h)

    def kinetic_energy(self, sid):
        return lib().or_kinetic_energy(self.h, sid)

    def gauss_residual(self):
        sc = C.c_double()
        r = lib().or_gauss_residual(self.h, C.byref(sc))
        return r, sc.value

    def continuity_residual(self):
        sc = C.c_double()
        r = lib().or_last_continuity_residual(self.h, C.byref(sc))
        return r, sc.value

    def current_series(self):
        n = C.c_size_t()
        lib().or_current_series(self.h, None, 0, C.byref(n))
        out = np.zeros(3 * n.value)
        lib().or_current_series(self.h, _dp(out), n.value, C.byref(n))
        return out.reshape(-1, 3)

    @property
    def steps_done(self):
        return lib().or_steps_done(self.h)


def build_workload(w: dict, seed: int | None = None) -> Sim:
    """Oracle simulation of a workload dict: species from the FD loader, ion background, fields."""
    s = Sim(w)
    seed = w.get("seed", 1) if seed is None else seed
    for sp in w["species"]:
        s.init_species(sp, seed)
    if w.get("dielectric") is not None or w.get("wall") is not None:
        # the inverse-permittivity map and the wall field are inputs, drawn by the shared input
        # generator
        from paper_2501_07465_amd import workloads as W
        if w.get("dielectric") is not None:
            s.set_eps_inv(W.eps_inv_map(w))
            off = W.eps_offdiag_map(w)
            if off is not None:
                s.set_eps_offdiag(off)
        if w.get("wall") is not None:
            s.set_ext_field(W.wall_field(w))
    s.set_ion_background(w.get("ion", "local") == "uniform")
    if w.get("gauss_init", False):
        s.gauss_init_1d()
    return s
