"""FP64 CPU oracle for the elastic-wall D3Q19 lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  The arithmetic
lives in ``lbm_oracle.c`` (plain C, FP64, OpenMP over sites); this module only
builds it with gcc and marshals arguments through ctypes.

Which part of the paper each oracle function follows is stated in the C file;
closed forms used to pin it are in ``oracle.closed_forms``, the brute-force
single-site transcription in ``oracle.brute`` and the MLP reference in
``oracle.mlp``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [ctypes.c_int] * 3 + [P, P, P, P, ctypes.c_double]
    lib.orc_destroy.argtypes = [P]
    lib.orc_n_sites.argtypes = [P]
    lib.orc_n_sites.restype = ctypes.c_int
    lib.orc_site_coords.argtypes = [P, P]
    lib.orc_velocity_set.argtypes = [P, P]
    lib.orc_feq.argtypes = [ctypes.c_double] * 4 + [P]
    lib.orc_set_wall.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, ctypes.c_int]
    lib.orc_set_wall_F.argtypes = [P, P, ctypes.c_int]
    lib.orc_set_iolet.argtypes = [P, ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4 + [P]
    lib.orc_init_fields.argtypes = [P, P, P]
    lib.orc_set_populations.argtypes = [P, P]
    lib.orc_get_populations.argtypes = [P, P]
    lib.orc_step.argtypes = [P, ctypes.c_long]
    lib.orc_read.argtypes = [P, P, P, P, P]
    lib.orc_time.argtypes = [P]
    lib.orc_time.restype = ctypes.c_long
    lib.orc_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def velocity_set():
    """(c[19,3] int, w[19] float64) in the oracle's order."""
    lib = _load()
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19, np.float64)
    lib.orc_velocity_set(_ptr(c), _ptr(w))
    return c, w


def feq(rho, u):
    lib = _load()
    out = np.zeros(19, np.float64)
    lib.orc_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _ptr(out))
    return out


def num_threads() -> int:
    return int(_load().orc_num_threads())


class Oracle:
    """One vessel instance on the CPU in FP64.

    Arguments mirror the GPU library: ``labels`` is a (nz, ny, nx) uint8 array
    (x fastest; 0 wall, 1 fluid, 2.. iolet id+2), ``segment`` (uint16),
    ``normal`` (float32, (nz,ny,nx,3)) and ``iolet_weight`` (float32) are
    optional per-voxel arrays.  Sites are in raster order of fluid voxels.
    """

    def __init__(self, labels, tau, segment=None, normal=None, iolet_weight=None):
        lib = _load()
        labels = np.ascontiguousarray(labels, dtype=np.uint8)
        nz, ny, nx = labels.shape
        self._keep = [labels]
        seg = None if segment is None else np.ascontiguousarray(segment, dtype=np.uint16)
        nrm = None if normal is None else np.ascontiguousarray(normal, dtype=np.float32)
        iw = None if iolet_weight is None else np.ascontiguousarray(iolet_weight, dtype=np.float32)
        self._h = lib.orc_create(nx, ny, nz, _ptr(labels), _ptr(seg), _ptr(nrm), _ptr(iw),
                                 float(tau))
        if not self._h:
            raise ValueError("invalid geometry: no fluid voxel or fluid voxel on the array border")
        self.n = lib.orc_n_sites(self._h)
        self.shape = (nz, ny, nx)
        self.tau = float(tau)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_destroy(h)
            self._h = None

    def coords(self):
        xyz = np.zeros((self.n, 3), np.int32)
        _load().orc_site_coords(self._h, _ptr(xyz))
        return xyz

    def set_wall(self, mode, F=0.0, P0=1.0 / 3.0, k=(1.0,)):
        k = np.ascontiguousarray(k, dtype=np.float64)
        _load().orc_set_wall(self._h, int(mode), float(F), float(P0), _ptr(k), len(k))

    def set_wall_F(self, F):
        """Slip ratio per wall segment, replacing the single F of set_wall
        (one value per segment given to set_wall)."""
        F = np.ascontiguousarray(F, dtype=np.float64)
        if _load().orc_set_wall_F(self._h, _ptr(F), len(F)) != 0:
            raise ValueError("one F per wall segment is required")

    def set_iolet(self, iolet_id, kind, a0, amp=0.0, period=1.0, phase=0.0, direction=(0, 0, 0)):
        d = np.ascontiguousarray(direction, dtype=np.float64)
        _load().orc_set_iolet(self._h, int(iolet_id), int(kind), float(a0), float(amp),
                              float(period), float(phase), _ptr(d))

    def init_fields(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        _load().orc_init_fields(self._h, _ptr(r), _ptr(v))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.n, 19)
        _load().orc_set_populations(self._h, _ptr(f))

    def populations(self):
        f = np.zeros((self.n, 19), np.float64)
        _load().orc_get_populations(self._h, _ptr(f))
        return f

    def step(self, n=1):
        _load().orc_step(self._h, int(n))

    @property
    def time(self):
        return int(_load().orc_time(self._h))

    def read(self):
        """(rho[N], u[N,3], wss[N], wall_dr[N]) from f(t)."""
        rho = np.zeros(self.n)
        u = np.zeros((self.n, 3))
        wss = np.zeros(self.n)
        dr = np.zeros(self.n)
        _load().orc_read(self._h, _ptr(rho), _ptr(u), _ptr(wss), _ptr(dr))
        return rho, u, wss, dr
