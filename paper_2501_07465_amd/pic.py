"""Thin ctypes binding of libpic (include/pic.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libpic.so``.  PyTorch supplies the device arena (one ``uint8`` tensor) and the
HIP stream.  Importing this module on a machine without the built library
raises; there is no fallback.

The module exposes the C entry points under their own names (``pic_create``,
``pic_init_species``, ``pic_step``, ``pic_diag``, ...) plus a small
``Simulation`` helper that builds a simulation from a workload dict of
``paper_2501_07465_amd.workloads``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ECFL, PIC_ENOMEM, PIC_ESTATE, PIC_EDEVICE, PIC_ENONFINITE, PIC_ETRUNC = 0, -1, -2, -3, -4, -5, -6, -7
PIC_FP32, PIC_FP64 = 0, 1
PIC_PERIODIC, PIC_OPEN = 0, 1
PIC_FREE, PIC_BOUND, PIC_DIRAC = 0, 1, 2
PIC_REGION_ALL, PIC_REGION_BALL, PIC_REGION_BOX = 0, 1, 2
PIC_MOM_COLD, PIC_MOM_FD = 0, 1
PIC_LOAD_RANDOM, PIC_LOAD_QUIET = 0, 1
PIC_SRC_NONE, PIC_SRC_SHEET, PIC_SRC_POINT = 0, 1, 2
(DIAG_FIELD_ENERGY, DIAG_KINETIC_ENERGY, DIAG_GAUSS_RESIDUAL, DIAG_CONTINUITY, DIAG_CURRENT_SERIES,
 DIAG_PARTICLE_COUNT, DIAG_STEP, DIAG_OVERFLOW, DIAG_EXPORT_PARTICLES, DIAG_EXPORT_FIELDS,
 DIAG_EXPORT_CURRENT, DIAG_KEYS, DIAG_NONFINITE_FLAG) = range(13)

EXPORTED = ["pic_create", "pic_init_species", "pic_footprint", "pic_bind", "pic_load_particles",
            "pic_load_fields", "pic_load_eps_inv", "pic_load_eps_offdiag", "pic_load_ext_field", "pic_field_shape", "pic_init_fields", "pic_step", "pic_use_graphs",
            "pic_diag", "pic_energy_histogram", "pic_energy_histogram_static", "pic_time_kernels", "pic_sync", "pic_set_stream", "pic_species_count", "pic_last_error", "pic_destroy",
            "pic_batch_footprint", "pic_batch_create", "pic_batch_add", "pic_batch_remove",
            "pic_batch_step", "pic_batch_size", "pic_batch_captures", "pic_batch_last_error", "pic_batch_destroy",
            "pic_measure_soa_copy"]


class GridDesc(C.Structure):
    _fields_ = [("dims", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3), ("dt", C.c_double),
                ("bc", C.c_int * 3), ("precision", C.c_int), ("tile", C.c_int * 3), ("block", C.c_int),
                ("unit", C.c_int),
                ("sort_every", C.c_int), ("series_cap", C.c_int), ("track_continuity", C.c_int),
                ("src_kind", C.c_int), ("src_comp", C.c_int), ("src_axis", C.c_int),
                ("src_index", C.c_int * 3), ("src_j0", C.c_double), ("src_omega", C.c_double),
                ("src_tau", C.c_double), ("eps_cells", C.c_int), ("ext_field", C.c_int)]


class SpeciesDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("q", C.c_double), ("m", C.c_double), ("density", C.c_double),
                ("weight", C.c_double), ("ppc", C.c_int), ("count", C.c_longlong), ("momentum", C.c_int),
                ("e_fermi", C.c_double), ("temperature", C.c_double), ("loading", C.c_int),
                ("pert_amp", C.c_double), ("pert_mode", C.c_int), ("omega0", C.c_double * 3),
                ("gamma", C.c_double * 3), ("b_weight", C.c_double), ("xi_radius", C.c_double),
                ("v_f", C.c_double), ("sheet_normal", C.c_int), ("reflect", C.c_int), ("region", C.c_int),
                ("rc", C.c_double * 3), ("rr", C.c_double), ("rlo", C.c_double * 3), ("rhi", C.c_double * 3),
                ("mass_per_particle", C.c_int)]


_lib = None
_D = C.POINTER(C.c_double)
_VP = C.c_void_p


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpic error {code}: {msg}")
        self.code = code


def lib():
    """Load libpic.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpic.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.pic_create.argtypes = [C.POINTER(GridDesc), C.POINTER(_VP)]
        L.pic_init_species.argtypes = [_VP, C.POINTER(SpeciesDesc), C.c_uint64, C.POINTER(C.c_int)]
        L.pic_footprint.argtypes = [_VP, C.POINTER(C.c_size_t)]
        L.pic_bind.argtypes = [_VP, _VP, C.c_size_t, _VP]
        L.pic_load_particles.argtypes = [_VP, C.c_int, _D, _D, _D, C.c_size_t]
        L.pic_load_fields.argtypes = [_VP, _D, _D]
        L.pic_load_eps_inv.argtypes = [_VP, _D]
        L.pic_load_eps_offdiag.argtypes = [_VP, _D]
        L.pic_load_ext_field.argtypes = [_VP, _D]
        L.pic_energy_histogram.argtypes = [_VP, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
        L.pic_energy_histogram_static.argtypes = [_VP, C.c_int, C.c_double, C.c_int, C.POINTER(C.c_uint64)]
        L.pic_field_shape.argtypes = [_VP, C.POINTER(C.c_int)]
        L.pic_init_fields.argtypes = [_VP, C.c_int]
        L.pic_step.argtypes = [_VP, C.c_int]
        L.pic_use_graphs.argtypes = [_VP, C.c_int]
        L.pic_diag.argtypes = [_VP, C.c_int, C.c_int, _D, C.c_size_t, C.POINTER(C.c_size_t)]
        L.pic_sync.argtypes = [_VP]
        L.pic_set_stream.argtypes = [_VP, _VP]
        L.pic_time_kernels.argtypes = [_VP, C.c_int, _D]
        L.pic_species_count.argtypes = [_VP, C.c_int]
        L.pic_species_count.restype = C.c_longlong
        L.pic_last_error.argtypes = [_VP]
        L.pic_last_error.restype = C.c_char_p
        L.pic_destroy.argtypes = [_VP]
        L.pic_destroy.restype = None
        L.pic_batch_footprint.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_size_t)]
        L.pic_batch_create.argtypes = [C.c_int, C.c_int, C.c_int, _VP, C.c_size_t, _VP, C.POINTER(_VP)]
        L.pic_batch_add.argtypes = [_VP, _VP]
        L.pic_batch_remove.argtypes = [_VP, _VP]
        L.pic_batch_step.argtypes = [_VP, C.c_int]
        L.pic_batch_size.argtypes = [_VP]
        L.pic_batch_captures.argtypes = [_VP]
        L.pic_batch_last_error.argtypes = [_VP]
        L.pic_batch_last_error.restype = C.c_char_p
        L.pic_batch_destroy.argtypes = [_VP]
        L.pic_batch_destroy.restype = None
        L.pic_measure_soa_copy.argtypes = [C.POINTER(_VP), C.POINTER(_VP), C.c_int, C.c_longlong, _VP]
        _lib = L
    return _lib


def _check(code, handle=None, batch=False):
    if code != PIC_OK:
        L = lib()
        msg = (L.pic_batch_last_error(handle) if batch else L.pic_last_error(handle)) or b""
        raise PicError(code, msg.decode())
    return code


# ---- entry points under their C names --------------------------------------------------------------
def pic_create(g: GridDesc):
    h = _VP()
    _check(lib().pic_create(C.byref(g), C.byref(h)))
    return h


def pic_init_species(h, d: SpeciesDesc, seed: int) -> int:
    sid = C.c_int(-1)
    _check(lib().pic_init_species(h, C.byref(d), seed, C.byref(sid)), h)
    return sid.value


def pic_footprint(h) -> int:
    b = C.c_size_t()
    _check(lib().pic_footprint(h, C.byref(b)), h)
    return b.value


def pic_bind(h, arena_ptr: int, nbytes: int, stream_ptr: int):
    _check(lib().pic_bind(h, C.c_void_p(arena_ptr), nbytes, C.c_void_p(stream_ptr)), h)


def pic_load_particles(h, sid, x, v, xi=None):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    xip = None
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
        xip = xi.ctypes.data_as(_D)
    _check(lib().pic_load_particles(h, sid, x.ctypes.data_as(_D), v.ctypes.data_as(_D), xip, x.shape[0]), h)


def pic_load_fields(h, e=None, b=None):
    ep = bp = None
    if e is not None:
        e = np.ascontiguousarray(e, dtype=np.float64)
        ep = e.ctypes.data_as(_D)
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.float64)
        bp = b.ctypes.data_as(_D)
    _check(lib().pic_load_fields(h, ep, bp), h)


def pic_load_eps_inv(h, einv):
    einv = np.ascontiguousarray(einv, dtype=np.float64)
    _check(lib().pic_load_eps_inv(h, einv.ctypes.data_as(_D)), h)


def pic_load_eps_offdiag(h, eoff):
    eoff = np.ascontiguousarray(eoff, dtype=np.float64)
    _check(lib().pic_load_eps_offdiag(h, eoff.ctypes.data_as(_D)), h)


def pic_load_ext_field(h, e):
    e = np.ascontiguousarray(e, dtype=np.float64)
    _check(lib().pic_load_ext_field(h, e.ctypes.data_as(_D)), h)


def pic_energy_histogram(h, sid, e_max, nbins):
    out = np.zeros(nbins + 1, dtype=np.uint64)
    _check(lib().pic_energy_histogram(h, sid, e_max, nbins, out.ctypes.data_as(C.POINTER(C.c_uint64))), h)
    return out


def pic_energy_histogram_static(h, sid, e_max, nbins):
    out = np.zeros(nbins + 1, dtype=np.uint64)
    _check(lib().pic_energy_histogram_static(h, sid, e_max, nbins, out.ctypes.data_as(C.POINTER(C.c_uint64))), h)
    return out


def pic_field_shape(h):
    L = (C.c_int * 3)()
    _check(lib().pic_field_shape(h, L), h)
    return tuple(L)


def pic_init_fields(h, mode: int):
    _check(lib().pic_init_fields(h, mode), h)


def pic_step(h, n: int):
    _check(lib().pic_step(h, n), h)


def pic_use_graphs(h, on: bool):
    _check(lib().pic_use_graphs(h, int(on)), h)


def pic_diag(h, kind: int, arg: int = -1) -> np.ndarray:
    n = C.c_size_t()
    r = lib().pic_diag(h, kind, arg, None, 0, C.byref(n))
    if r not in (PIC_OK, PIC_ETRUNC):
        _check(r, h)
    out = np.zeros(max(n.value, 1))
    _check(lib().pic_diag(h, kind, arg, out.ctypes.data_as(_D), out.size, C.byref(n)), h)
    return out[:n.value]


def pic_time_kernels(h, nsteps: int):
    """Average device ms per launch: particle kernel, field kernel, one sort, number of sorts."""
    out = np.zeros(4)
    _check(lib().pic_time_kernels(h, nsteps, out.ctypes.data_as(_D)), h)
    return out


def pic_sync(h):
    _check(lib().pic_sync(h), h)


def pic_set_stream(h, stream_ptr):
    _check(lib().pic_set_stream(h, C.c_void_p(stream_ptr)), h)


def pic_species_count(h, sid) -> int:
    return lib().pic_species_count(h, sid)


def pic_last_error(h=None) -> str:
    return (lib().pic_last_error(h) or b"").decode()


def pic_destroy(h):
    lib().pic_destroy(h)


def pic_batch_footprint(max_sims: int, dims: int) -> int:
    b = C.c_size_t()
    _check(lib().pic_batch_footprint(max_sims, dims, C.byref(b)))
    return b.value


def pic_batch_create(max_sims, dims, precision, arena_ptr, nbytes, stream_ptr):
    h = _VP()
    _check(lib().pic_batch_create(max_sims, dims, precision, C.c_void_p(arena_ptr), nbytes,
                                  C.c_void_p(stream_ptr), C.byref(h)))
    return h


def pic_batch_add(b, s):
    _check(lib().pic_batch_add(b, s), b, batch=True)


def pic_batch_remove(b, s):
    _check(lib().pic_batch_remove(b, s), b, batch=True)


def pic_batch_step(b, k):
    _check(lib().pic_batch_step(b, k), b, batch=True)


def pic_batch_size(b) -> int:
    return lib().pic_batch_size(b)


def pic_batch_captures(b) -> int:
    return lib().pic_batch_captures(b)


def pic_batch_destroy(b):
    lib().pic_batch_destroy(b)


def pic_measure_soa_copy(src_ptrs, dst_ptrs, n, stream_ptr):
    """Counter-calibration copy: dst[k][:n] = src[k][:n] for device float arrays (pointers)."""
    k = len(src_ptrs)
    S, D = (_VP * k)(*src_ptrs), (_VP * k)(*dst_ptrs)
    _check(lib().pic_measure_soa_copy(S, D, k, n, C.c_void_p(stream_ptr)))


# ---- workload dicts -> descriptors -----------------------------------------------------------------
_KIND = {"free": PIC_FREE, "bound": PIC_BOUND, "dirac": PIC_DIRAC}
_REGION = {"all": PIC_REGION_ALL, "ball": PIC_REGION_BALL, "box": PIC_REGION_BOX}
_SRC = {"none": PIC_SRC_NONE, "sheet": PIC_SRC_SHEET, "point": PIC_SRC_POINT}


def grid_desc(w: dict, precision: str | None = None, track_continuity: bool = False, block: int = 256,
              series_cap: int | None = None, unit: int | None = None) -> GridDesc:
    g = GridDesc()
    g.dims = w["dims"]
    for a in range(3):
        g.n[a] = w["n"][a]
        g.dx[a] = w["dx"][a]
        g.bc[a] = PIC_PERIODIC if w["periodic"][a] else PIC_OPEN
        g.tile[a] = w["tile"][a]
    g.dt = w["dt"]
    prec = precision or w.get("precision", "fp32")
    g.precision = PIC_FP64 if prec == "fp64" else PIC_FP32
    g.block = block
    g.unit = int(w.get("unit", 0) if unit is None else unit)
    g.sort_every = w.get("sort_every", 20)
    g.series_cap = series_cap or max(1, int(w.get("steps", 1000)) + 64)
    g.track_continuity = int(track_continuity)
    d = w.get("dielectric")
    g.eps_cells = 0 if d is None else (1 if np.asarray(d["eps"]).ndim == 1 else 2)
    g.ext_field = int(w.get("wall") is not None)
    src = w.get("source", {"kind": "none"})
    g.src_kind = _SRC[src["kind"]]
    if g.src_kind:
        g.src_comp = src["comp"]
        g.src_axis = src.get("axis", 0)
        for a in range(3):
            g.src_index[a] = src["index"][a]
        g.src_j0 = src["j0"]
        g.src_omega = src["omega"]
        g.src_tau = src["tau"]
    return g


def species_desc(sp: dict, count: int = 0, weight: float = 0.0) -> SpeciesDesc:
    d = SpeciesDesc()
    d.kind = _KIND[sp["kind"]]
    d.q = sp["q"]
    d.m = sp.get("m", 0.0)
    d.density = sp.get("density", 0.0)
    d.weight = weight
    d.ppc = sp.get("ppc", 0)
    d.count = count
    d.momentum = PIC_MOM_FD if sp.get("momentum", "fd") == "fd" else PIC_MOM_COLD
    d.e_fermi = sp.get("e_fermi", 0.0)
    d.temperature = sp.get("temperature", 0.0)
    d.loading = PIC_LOAD_QUIET if sp.get("loading", "random") == "quiet" else PIC_LOAD_RANDOM
    d.pert_amp = sp.get("pert_amp", 0.0)
    d.pert_mode = sp.get("pert_mode", 1)
    for a in range(3):
        d.omega0[a] = sp.get("omega0", [0.0] * 3)[a]
        d.gamma[a] = sp.get("gamma", [0.0] * 3)[a]
    d.b_weight = sp.get("b_weight", 0.0)
    d.xi_radius = sp.get("xi_radius", 0.0)
    d.v_f = sp.get("v_f", 0.0)
    d.sheet_normal = sp.get("sheet_normal", -1)
    d.reflect = (2 if sp.get("scatter", "specular") == "diffuse" else 1) if sp.get("reflect", False) else 0
    d.mass_per_particle = int(bool(sp.get("mass_per_particle", False)))
    reg = sp.get("region", {"kind": "all"})
    d.region = _REGION[reg["kind"]]
    for a in range(3):
        d.rc[a] = reg.get("center", [0, 0, 0])[a]
        d.rlo[a] = reg.get("lo", [0, 0, 0])[a]
        d.rhi[a] = reg.get("hi", [0, 0, 0])[a]
    d.rr = reg.get("radius", 0.0)
    return d


def _ion_mode(w: dict) -> int:
    if w.get("gauss_init"):
        return 2
    return 1 if w.get("ion", "local") == "uniform" else 0


class Simulation:
    """One device-resident simulation: descriptors from a workload dict, arena and stream from torch."""

    def __init__(self, w: dict, precision: str | None = None, states=None, fields=None, init_fields=True,
                 track_continuity=False, graphs=True, stream=None, block=256, series_cap=None, unit=None):
        import torch
        self.w = w
        self.h = None
        g = grid_desc(w, precision, track_continuity, block, series_cap, unit)
        self.h = pic_create(g)
        self.species = []
        for i, sp in enumerate(w["species"]):
            if states is not None:
                x, v, xi, weight = states[i]
                d = species_desc(sp, count=len(x), weight=weight)
            else:
                d = species_desc(sp)
            self.species.append(pic_init_species(self.h, d, w.get("seed", 1)))
        self.nbytes = pic_footprint(self.h)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        # a stream of its own (the legacy default stream cannot be captured into a graph)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        pic_bind(self.h, self.arena.data_ptr(), self.nbytes, self.stream.cuda_stream)
        if states is not None:
            for sid, (x, v, xi, _) in zip(self.species, states):
                pic_load_particles(self.h, sid, x, v, xi)
        if w.get("dielectric") is not None:
            from . import workloads
            pic_load_eps_inv(self.h, workloads.eps_inv_map(w))
            off = workloads.eps_offdiag_map(w)
            if off is not None:
                pic_load_eps_offdiag(self.h, off)
        if w.get("wall") is not None:
            from . import workloads
            pic_load_ext_field(self.h, workloads.wall_field(w))
        if fields is not None:
            pic_load_fields(self.h, fields[0], fields[1])
        if init_fields:
            pic_init_fields(self.h, _ion_mode(w) if fields is None else (1 if w.get("ion") == "uniform" else 0))
        pic_use_graphs(self.h, graphs)

    def __del__(self):
        h = getattr(self, "h", None)
        if not h:
            return
        self.h = None
        try:
            pic_sync(h)
        except Exception:
            pass
        try:
            pic_destroy(h)
        except TypeError:
            pass  # at interpreter exit this module's functions may already be gone; the process frees it

    def step(self, n=1):
        pic_step(self.h, n)

    def sync(self):
        pic_sync(self.h)

    def set_stream(self, stream):
        """Enqueue later work on ``stream`` (a torch stream), ordered after the work so far."""
        pic_set_stream(self.h, stream.cuda_stream)
        self.stream = stream

    def count(self, sid):
        return pic_species_count(self.h, sid)

    def shape(self):
        return pic_field_shape(self.h)

    def particles(self, sid):
        n = self.count(sid)
        a = pic_diag(self.h, DIAG_EXPORT_PARTICLES, sid)
        return a[:3 * n].reshape(n, 3), a[3 * n:6 * n].reshape(n, 3), a[6 * n:].reshape(n, 3)

    def fields(self):
        L = self.shape()
        a = pic_diag(self.h, DIAG_EXPORT_FIELDS).reshape(6, L[2], L[1], L[0])
        return a[:3], a[3:]

    def current(self):
        L = self.shape()
        return pic_diag(self.h, DIAG_EXPORT_CURRENT).reshape(3, L[2], L[1], L[0])

    def keys(self, sid):
        return pic_diag(self.h, DIAG_KEYS, sid).astype(np.int64)

    def field_energy(self):
        return float(pic_diag(self.h, DIAG_FIELD_ENERGY)[0])

    def kinetic_energy(self, sid):
        return float(pic_diag(self.h, DIAG_KINETIC_ENERGY, sid)[0])

    def gauss_residual(self):
        r = pic_diag(self.h, DIAG_GAUSS_RESIDUAL)
        return float(r[0]), float(r[1])

    def continuity_residual(self):
        r = pic_diag(self.h, DIAG_CONTINUITY)
        return float(r[0]), float(r[1])

    def current_series(self):
        return pic_diag(self.h, DIAG_CURRENT_SERIES).reshape(-1, 3)

    def overflow(self):
        return int(pic_diag(self.h, DIAG_OVERFLOW)[0])

    def nonfinite(self):
        return int(pic_diag(self.h, DIAG_NONFINITE_FLAG)[0])

    @property
    def steps_done(self):
        return int(pic_diag(self.h, DIAG_STEP)[0])


class Batch:
    """Several simulations of the same dimensionality and precision stepped by one persistent particle
    launch and one field launch per step (one captured graph per sort period).  Members must be
    bound to the batch's stream."""

    def __init__(self, max_sims: int, dims: int, precision: str = "fp32", stream=None):
        import torch
        self.b = None
        self.max_sims = max_sims
        self.dims = dims
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.Stream()
        nb = pic_batch_footprint(max_sims, dims)
        self.table = torch.empty(nb, dtype=torch.uint8, device="cuda")
        self.b = pic_batch_create(max_sims, dims, PIC_FP64 if precision == "fp64" else PIC_FP32,
                                  self.table.data_ptr(), nb, self.stream.cuda_stream)
        self.members = []

    def add(self, sim: "Simulation"):
        pic_batch_add(self.b, sim.h)
        self.members.append(sim)

    def remove(self, sim: "Simulation"):
        pic_batch_remove(self.b, sim.h)
        self.members.remove(sim)

    def step(self, k: int):
        pic_batch_step(self.b, k)

    def __len__(self):
        return pic_batch_size(self.b)

    @property
    def captures(self) -> int:
        """How many times the step graph was captured."""
        return pic_batch_captures(self.b)

    def __del__(self):
        b = getattr(self, "b", None)
        if not b:
            return
        for s in list(getattr(self, "members", [])):
            try:
                pic_batch_remove(b, s.h)
            except Exception:
                pass
        self.b = None
        try:
            pic_batch_destroy(b)
        except TypeError:
            pass  # at interpreter exit this module's functions may already be gone; the process frees it


def footprint_of(w: dict, precision: str | None = None, block: int = 256, series_cap: int | None = None,
                 unit: int | None = None) -> int:
    """Device bytes a simulation of workload ``w`` needs (host-only planning, nothing allocated)."""
    h = pic_create(grid_desc(w, precision, False, block, series_cap, unit))
    try:
        for sp in w["species"]:
            pic_init_species(h, species_desc(sp), w.get("seed", 1))
        return pic_footprint(h)
    finally:
        pic_destroy(h)
