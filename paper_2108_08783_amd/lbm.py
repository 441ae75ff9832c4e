"""Thin ctypes binding of ``liblbm.so`` (C ABI in ``include/lbm.h``).

Functions keep the C names (``lbm_create_geometry``, ``lbm_set_wall_params``,
``lbm_step``, ``lbm_read_fields``, ...); they only marshal arguments, turn
status codes into exceptions and return outputs.  Every step of the method
runs in the HIP library: there is no fallback, and importing a function
raises if the library has not been built.  ``Lattice`` bundles the calls for
one context.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
DTYPES = {"f64": F64, "f32": F32, "f16": F16DEV, "bf16": BF16DEV}
BOUNCEBACK, ELASTIC = 0, 1
DENSITY, VELOCITY = 0, 1

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5

# Every symbol declared in include/lbm.h (checked by the CPU test-suite).
EXPORTS = [
    "lbm_create_geometry", "lbm_destroy", "lbm_last_error", "lbm_set_wall_params",
    "lbm_set_iolet", "lbm_init_fields", "lbm_init_fields_device", "lbm_step", "lbm_sync",
    "lbm_get_stream", "lbm_time_steps", "lbm_read_fields", "lbm_read_populations",
    "lbm_write_populations", "lbm_cycle_delta", "lbm_get_info", "lbm_instance_sites",
    "lbm_set_launch", "lbm_autotune", "lbm_plan_export", "lbm_copy_probe",
    "lbm_plan_compressed", "lbm_set_wall_F", "lbm_fast_axis", "lbm_create_geometry_ex",
    "lbm_uses_caller_resources", "lbm_read_fields_noalloc",
]

# Staging limit of lbm_read_fields_noalloc (LBM_NOALLOC_SCRATCH_BYTES and
# LBM_NOALLOC_MAX_SITES in include/lbm.h).
NOALLOC_SCRATCH_BYTES = 96 << 20
NOALLOC_MAX_SITES = (NOALLOC_SCRATCH_BYTES - 256) // 44


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Diverged(LbmError):
    pass


class InstanceDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("labels", ctypes.c_void_p), ("segment", ctypes.c_void_p),
                ("normal", ctypes.c_void_p), ("iolet_weight", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int64), ("n_boundary", ctypes.c_int64),
                ("n_wall_sites", ctypes.c_int64), ("n_wall_links", ctypes.c_int64),
                ("n_iolet_links", ctypes.c_int64), ("step", ctypes.c_int64),
                ("n_instances", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("index_bits", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("nontemporal", ctypes.c_int32), ("boundary_fused", ctypes.c_int32),
                ("sites_per_lane", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bytes_per_site_algorithmic", ctypes.c_double),
                ("bytes_per_site_model", ctypes.c_double), ("device_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Resources(ctypes.Structure):
    """lbm_resources: caller's device allocator and stream."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p),
                ("use_stream", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class TorchResources:
    """torch's caching allocator and torch's current stream on the current
    device, handed to lbm_create_geometry_ex: the library's device memory
    then comes from torch's pool and its work is ordered with torch's work
    on that stream.  Keep the object alive as long as the context."""

    def __init__(self):
        import torch
        self.device = torch.cuda.current_device()
        self.torch_stream = torch.cuda.current_stream(self.device)
        alloc_impl = torch.cuda.caching_allocator_alloc
        free_impl = torch.cuda.caching_allocator_delete
        dev, stream = self.device, self.torch_stream

        def alloc(nbytes, user):
            try:
                return alloc_impl(int(nbytes), dev, stream)
            except Exception:   # out of memory: the library reports LBM_ENOMEM
                return None

        def free(ptr, user):
            try:
                free_impl(ptr)
            except Exception:
                pass

        self._alloc, self._free = _ALLOC_FN(alloc), _FREE_FN(free)
        self.struct = Resources(self._alloc, self._free, None, 1, self.torch_stream.cuda_stream)


_lib = None


def load():
    """Opens liblbm.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run paper_2108_08783_amd/build.py first")
    # torch ships its own HIP runtime; load it first so that the library and
    # torch share one runtime in the process (the library's dependency is
    # then resolved to the already-loaded copy).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, L = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "lbm_create_geometry": [P, P, I, I, D],
        "lbm_create_geometry_ex": [P, P, I, I, D, P],
        "lbm_uses_caller_resources": [P, P, P],
        "lbm_destroy": [P],
        "lbm_set_wall_params": [P, I, I, D, D, P, I],
        "lbm_set_wall_F": [P, I, P, I],
        "lbm_fast_axis": [P, I, P],
        "lbm_set_iolet": [P, I, I, I, D, D, D, D, P],
        "lbm_init_fields": [P, I, P, P],
        "lbm_init_fields_device": [P, I, P],
        "lbm_step": [P, L],
        "lbm_sync": [P],
        "lbm_get_stream": [P, P],
        "lbm_time_steps": [P, L, P],
        "lbm_read_fields": [P, I, P, P, P, P],
        "lbm_read_fields_noalloc": [P, I, P, P, P, P],
        "lbm_read_populations": [P, I, P],
        "lbm_write_populations": [P, I, P],
        "lbm_cycle_delta": [P, I, P, P],
        "lbm_get_info": [P, P],
        "lbm_instance_sites": [P, I, P],
        "lbm_set_launch": [P, I, I, I, I, I, I, I],
        "lbm_autotune": [P, I, P],
        "lbm_plan_export": [P, I, P, P, P, P, P],
        "lbm_plan_compressed": [P, I, P, P],
        "lbm_copy_probe": [P, P, ctypes.c_size_t, I, I, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lbm_last_error.argtypes = [P]
    lib.lbm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, ctx=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(ctx).decode()
        raise (Diverged if rc == LBM_EDIVERGED else LbmError)(rc, msg)


def _descs(geoms):
    keep = []
    arr = (InstanceDesc * len(geoms))()
    for d, g in zip(arr, geoms):
        lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
        nz, ny, nx = lab.shape
        seg = None if g.segment is None else np.ascontiguousarray(g.segment, dtype=np.uint16)
        nrm = None if g.normal is None else np.ascontiguousarray(g.normal, dtype=np.float32)
        iw = None if g.iolet_weight is None else np.ascontiguousarray(g.iolet_weight, np.float32)
        keep += [lab, seg, nrm, iw]
        d.nx, d.ny, d.nz = nx, ny, nz
        d.labels, d.segment, d.normal, d.iolet_weight = _p(lab), _p(seg), _p(nrm), _p(iw)
    return arr, keep


# ------------------------------------------------------------------ C names --
def lbm_create_geometry(geoms, dtype="f32", tau=0.8):
    """Returns an opaque context handle (int)."""
    lib = load()
    arr, keep = _descs(geoms)
    out = ctypes.c_void_p()
    rc = lib.lbm_create_geometry(ctypes.byref(out), arr, len(geoms), DTYPES.get(dtype, dtype),
                                 float(tau))
    _check(rc, None)
    return out.value


def lbm_create_geometry_ex(geoms, dtype="f32", tau=0.8, resources=None):
    """As lbm_create_geometry with a Resources structure (or None)."""
    lib = load()
    arr, keep = _descs(geoms)
    out = ctypes.c_void_p()
    res = None if resources is None else ctypes.byref(resources)
    rc = lib.lbm_create_geometry_ex(ctypes.byref(out), arr, len(geoms), DTYPES.get(dtype, dtype),
                                    float(tau), res)
    _check(rc, None)
    return out.value


def lbm_uses_caller_resources(ctx):
    """(allocator, stream): whether ctx uses the caller's allocator / stream."""
    a, st = ctypes.c_int(), ctypes.c_int()
    _check(load().lbm_uses_caller_resources(ctx, ctypes.byref(a), ctypes.byref(st)), ctx)
    return bool(a.value), bool(st.value)


def lbm_destroy(ctx):
    _check(load().lbm_destroy(ctx), None)


def lbm_set_wall_params(ctx, inst, mode, F, P0, k):
    k = np.ascontiguousarray(np.atleast_1d(k), dtype=np.float64)
    _check(load().lbm_set_wall_params(ctx, inst, mode, float(F), float(P0), _p(k), len(k)), ctx)


def lbm_set_wall_F(ctx, inst, F):
    F = np.ascontiguousarray(np.atleast_1d(F), dtype=np.float64)
    _check(load().lbm_set_wall_F(ctx, inst, _p(F), len(F)), ctx)


def lbm_set_iolet(ctx, inst, iolet_id, kind, a0, amp=0.0, period=1.0, phase=0.0, direction=None):
    d = None if direction is None else np.ascontiguousarray(direction, dtype=np.float64)
    _check(load().lbm_set_iolet(ctx, inst, iolet_id, kind, float(a0), float(amp), float(period),
                                float(phase), _p(d)), ctx)


def lbm_init_fields(ctx, inst, rho=None, u=None):
    r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    _check(load().lbm_init_fields(ctx, inst, _p(r), _p(v)), ctx)


def lbm_init_fields_device(ctx, inst, rho_u_ptr):
    _check(load().lbm_init_fields_device(ctx, inst, ctypes.c_void_p(rho_u_ptr)), ctx)


def lbm_step(ctx, n):
    _check(load().lbm_step(ctx, int(n)), ctx)


def lbm_sync(ctx):
    _check(load().lbm_sync(ctx), ctx)


def lbm_get_stream(ctx):
    s = ctypes.c_void_p()
    _check(load().lbm_get_stream(ctx, ctypes.byref(s)), ctx)
    return s.value or 0


def lbm_time_steps(ctx, n):
    ms = ctypes.c_double()
    _check(load().lbm_time_steps(ctx, int(n), ctypes.byref(ms)), ctx)
    return ms.value


def lbm_instance_sites(ctx, inst):
    n = ctypes.c_int64()
    _check(load().lbm_instance_sites(ctx, inst, ctypes.byref(n)), ctx)
    return n.value


def lbm_read_fields(ctx, inst, wss=True, wall_dr=True):
    """(rho[n], u[n,3], wss[n] or None, wall_dr[n] or None)."""
    n = lbm_instance_sites(ctx, inst)
    rho = np.zeros(n)
    u = np.zeros((n, 3))
    w = np.zeros(n) if wss else None
    dr = np.zeros(n, np.float32) if wall_dr else None
    _check(load().lbm_read_fields(ctx, inst, _p(rho), _p(u), _p(w), _p(dr)), ctx)
    return rho, u, w, dr


def lbm_read_fields_noalloc(ctx, inst, rho, u, wss=None, wall_dr=None):
    """lbm_read_fields into caller-owned host arrays (rho[n], u[n,3] float64,
    optional wss[n] float64, wall_dr[n] float32), with no allocation by the
    library; any array may be None."""
    for a, dt in ((rho, np.float64), (u, np.float64), (wss, np.float64), (wall_dr, np.float32)):
        if a is not None and (a.dtype != dt or not a.flags.c_contiguous):
            raise TypeError("output arrays must be C-contiguous float64 (float32 for wall_dr)")
    _check(load().lbm_read_fields_noalloc(ctx, inst, _p(rho), _p(u), _p(wss), _p(wall_dr)), ctx)


def lbm_read_populations(ctx, inst):
    n = lbm_instance_sites(ctx, inst)
    f = np.zeros((n, 19))
    _check(load().lbm_read_populations(ctx, inst, _p(f)), ctx)
    return f


def lbm_write_populations(ctx, inst, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().lbm_write_populations(ctx, inst, _p(f)), ctx)


def lbm_cycle_delta(ctx, inst):
    du, dp = ctypes.c_double(), ctypes.c_double()
    _check(load().lbm_cycle_delta(ctx, inst, ctypes.byref(du), ctypes.byref(dp)), ctx)
    return du.value, dp.value


def lbm_get_info(ctx):
    info = Info()
    _check(load().lbm_get_info(ctx, ctypes.byref(info)), ctx)
    return info.as_dict()


def lbm_set_launch(ctx, block_size=-1, index_bits=-1, use_graph=-1, xcd_remap=-1,
                   nontemporal=-1, boundary_fused=-1, sites_per_lane=-1):
    _check(load().lbm_set_launch(ctx, block_size, index_bits, use_graph, xcd_remap, nontemporal,
                                 boundary_fused, sites_per_lane), ctx)


def lbm_autotune(ctx, steps_per_trial=64):
    r = ctypes.c_double()
    _check(load().lbm_autotune(ctx, int(steps_per_trial), ctypes.byref(r)), ctx)
    return r.value


def lbm_copy_probe(dst_ptr, src_ptr, nbytes, nontemporal=False, reps=20, stream=0):
    """Average milliseconds of a plain device copy (diagnostic)."""
    ms = ctypes.c_double()
    _check(load().lbm_copy_probe(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes),
                                 int(nontemporal), int(reps), ctypes.c_void_p(stream),
                                 ctypes.byref(ms)), None)
    return ms.value


def lbm_plan_export(geoms, wall_modes=None, tables=True):
    """Host-only geometry plan (no GPU).  Returns a dict with the counts and,
    if ``tables``, the neighbour table [18, N], boundary sites and masks."""
    lib = load()
    arr, keep = _descs(geoms)
    wm = None if wall_modes is None else np.ascontiguousarray(wall_modes, dtype=np.int32)
    counts = np.zeros(6, np.int64)
    _check(lib.lbm_plan_export(arr, len(geoms), _p(wm), _p(counts), None, None, None), None)
    out = dict(n_sites=int(counts[0]), n_boundary=int(counts[1]), n_wall_sites=int(counts[2]),
               n_wall_links=int(counts[3]), n_iolet_links=int(counts[4]),
               max_abs_offset=int(counts[5]))
    if tables:
        nbr = np.zeros((18, counts[0]), np.int32)
        bs = np.zeros(max(1, counts[1]), np.int32)
        bm = np.zeros(max(1, counts[1]), np.uint32)
        _check(lib.lbm_plan_export(arr, len(geoms), _p(wm), _p(counts), _p(nbr), _p(bs), _p(bm)),
               None)
        out.update(nbr=nbr, boundary=bs[:counts[1]], bmask=bm[:counts[1]])
    return out


def lbm_plan_compressed(geoms, wall_modes=None):
    """Host-only build (and self-check) of the update kernel's compressed
    addressing: dict with stretches, irregular, exceptional and records."""
    lib = load()
    arr, keep = _descs(geoms)
    wm = None if wall_modes is None else np.ascontiguousarray(wall_modes, np.int32)
    st = np.zeros(4, np.int64)
    _check(lib.lbm_plan_compressed(arr, len(geoms), _p(wm), _p(st)), None)
    del keep
    return dict(stretches=int(st[0]), irregular=int(st[1]), exceptional=int(st[2]),
                records=int(st[3]))


def lbm_fast_axis(geoms):
    """Host-only: the axis each instance's sites are ordered along on the
    device (0 x, 1 y, 2 z; see lbm_create_geometry)."""
    lib = load()
    arr, keep = _descs(geoms)
    out = np.zeros(len(geoms), np.int32)
    _check(lib.lbm_fast_axis(arr, len(geoms), _p(out)), None)
    del keep
    return [int(v) for v in out]


# ------------------------------------------------------------------ wrapper --
class Lattice:
    """One library context holding one or more vessel instances.

    resources: "torch" (default) hands torch's caching allocator and torch's
    current stream to the library (lbm_create_geometry_ex), so its device
    memory comes from torch's pool and its work is ordered with torch's on
    that stream; "library" lets the library call hipMalloc and create its
    own stream (lbm_create_geometry)."""

    def __init__(self, geoms, dtype="f32", tau=0.8, resources="torch"):
        if not isinstance(geoms, (list, tuple)):
            geoms = [geoms]
        self.geoms = list(geoms)
        self.tau = float(tau)
        self.dtype = dtype
        if resources == "torch":
            self._res = TorchResources()
            self.ctx = lbm_create_geometry_ex(self.geoms, dtype, tau, self._res.struct)
        elif resources == "library":
            self._res = None
            self.ctx = lbm_create_geometry(self.geoms, dtype, tau)
        else:
            raise ValueError(f"resources must be 'torch' or 'library', not {resources!r}")

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None
        self._res = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def n_sites(self, inst=0):
        return lbm_instance_sites(self.ctx, inst)

    def set_wall(self, inst, mode, F=0.0, P0=1.0 / 3.0, k=(1.0,)):
        lbm_set_wall_params(self.ctx, inst, mode, F, P0, k)

    def set_wall_F(self, inst, F):
        """Slip ratio per wall segment of instance inst (after set_wall)."""
        lbm_set_wall_F(self.ctx, inst, F)

    def set_iolet(self, inst, iolet_id, kind, a0, amp=0.0, period=1.0, phase=0.0, direction=None):
        lbm_set_iolet(self.ctx, inst, iolet_id, kind, a0, amp, period, phase, direction)

    def init_fields(self, inst, rho=None, u=None):
        lbm_init_fields(self.ctx, inst, rho, u)

    def init_fields_device(self, inst, rho_u):
        """rho_u: a torch CUDA float32 tensor [n, 4] (device memory)."""
        assert rho_u.is_cuda and rho_u.dtype.itemsize == 4 and rho_u.is_contiguous()
        assert tuple(rho_u.shape) == (self.n_sites(inst), 4)
        lbm_init_fields_device(self.ctx, inst, rho_u.data_ptr())

    def step(self, n=1):
        lbm_step(self.ctx, n)

    def sync(self):
        lbm_sync(self.ctx)

    def time_steps(self, n):
        return lbm_time_steps(self.ctx, n)

    def read_fields(self, inst=0, wss=True, wall_dr=True):
        return lbm_read_fields(self.ctx, inst, wss, wall_dr)

    def read_populations(self, inst=0):
        return lbm_read_populations(self.ctx, inst)

    def write_populations(self, inst, f):
        lbm_write_populations(self.ctx, inst, f)

    def cycle_delta(self, inst=0):
        return lbm_cycle_delta(self.ctx, inst)

    def info(self):
        return lbm_get_info(self.ctx)

    def set_launch(self, **kw):
        lbm_set_launch(self.ctx, **kw)

    def autotune(self, steps_per_trial=64):
        return lbm_autotune(self.ctx, steps_per_trial)

    @property
    def stream(self):
        return lbm_get_stream(self.ctx)
