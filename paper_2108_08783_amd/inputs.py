"""Seeded synthetic vessel geometries and drive parameters.

This module produces INPUTS only (voxel labels, segment ids, outward normals,
inlet profile weights, seeded perturbations and parameter draws).  It holds
none of the lattice Boltzmann arithmetic, so the GPU path and the CPU oracle
can both be fed from it without sharing any of the method's code.

Voxel arrays are indexed ``[z, y, x]`` (x fastest in memory).  Labels:
0 wall/solid, 1 fluid, 2.. iolet with id = label - 2.

The paper's own geometries (a 4 cm cylinder at R = 50/100/200 lattice units,
Sec. 2.4 and Table A1; a patient forearm, Sec. 3) are stood in for by the
synthetic shapes below; the forearm data is not available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

WALL, FLUID, IOLET0 = 0, 1, 2


@dataclasses.dataclass
class Geometry:
    labels: np.ndarray                      # uint8 [nz, ny, nx]
    segment: Optional[np.ndarray] = None    # uint16 [nz, ny, nx]
    normal: Optional[np.ndarray] = None     # float32 [nz, ny, nx, 3], outward unit
    iolet_weight: Optional[np.ndarray] = None  # float32 [nz, ny, nx]
    n_seg: int = 1
    iolets: List[dict] = dataclasses.field(default_factory=list)  # id, role, direction
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return self.labels.shape

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.labels == FLUID))


def cylinder(R: float, L: int, margin: int = 2, with_normals: bool = True) -> Geometry:
    """Straight z-aligned tube of radius R (strict r < R about an axis through
    voxel centres), fluid for z = 1..L, inlet plane z = 0 (iolet 0), outlet
    plane z = L + 1 (iolet 1).  Parabolic inlet weights 2 (1 - r^2/R^2)."""
    n = int(2 * math.ceil(R) + 2 * margin + 1)
    nx = ny = n
    nz = L + 2
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r2 = (x - c) ** 2 + (y - c) ** 2
    disk = r2 < R * R
    labels = np.zeros((nz, ny, nx), np.uint8)
    labels[1:L + 1][:, disk] = FLUID
    labels[0, :, :] = IOLET0 + 0
    labels[nz - 1, :, :] = IOLET0 + 1
    geo = Geometry(labels=labels)
    r = np.sqrt(r2)
    w = np.where(disk, 2.0 * (1.0 - r2 / (R * R)), 0.0).astype(np.float32)
    geo.iolet_weight = np.broadcast_to(w, (nz, ny, nx)).copy()
    if with_normals:
        nrm = np.zeros((ny, nx, 3), np.float32)
        rr = np.where(r > 0, r, 1.0)
        nrm[..., 0] = (x - c) / rr
        nrm[..., 1] = (y - c) / rr
        geo.normal = np.broadcast_to(nrm, (nz, ny, nx, 3)).copy()
    geo.segment = np.zeros((nz, ny, nx), np.uint16)
    geo.iolets = [dict(id=0, role="inlet", direction=(0.0, 0.0, 1.0)),
                  dict(id=1, role="outlet", direction=(0.0, 0.0, -1.0))]
    geo.info = dict(kind="cylinder", R=R, L=L, centre=c)
    return geo


def duct(W: int, H: int, L: int) -> Geometry:
    """Rectangular duct: fluid x = 1..W, y = 1..H, z = 1..L; walls around it,
    inlet plane z = 0 (iolet 0) and outlet plane z = L + 1 (iolet 1)."""
    nx, ny, nz = W + 2, H + 2, L + 2
    labels = np.zeros((nz, ny, nx), np.uint8)
    labels[1:L + 1, 1:H + 1, 1:W + 1] = FLUID
    labels[0] = IOLET0 + 0
    labels[nz - 1] = IOLET0 + 1
    geo = Geometry(labels=labels, segment=np.zeros_like(labels, dtype=np.uint16))
    geo.iolets = [dict(id=0, role="inlet", direction=(0.0, 0.0, 1.0)),
                  dict(id=1, role="outlet", direction=(0.0, 0.0, -1.0))]
    geo.info = dict(kind="duct", W=W, H=H, L=L)
    return geo


def closed_box(nx: int, ny: int, nz: int) -> Geometry:
    """Fluid box enclosed by one layer of wall voxels on every side."""
    labels = np.zeros((nz + 2, ny + 2, nx + 2), np.uint8)
    labels[1:nz + 1, 1:ny + 1, 1:nx + 1] = FLUID
    return Geometry(labels=labels, info=dict(kind="box"))


def random_labels(shape, rng: np.random.Generator, p_fluid=0.7, n_iolets=2) -> Geometry:
    """Tiny box of random labels (fluid, wall and iolet voxels mixed) with a
    one-voxel non-fluid border, for brute-force checks of every link type."""
    nz, ny, nx = shape
    lab = np.where(rng.random(shape) < p_fluid, FLUID, WALL).astype(np.uint8)
    io = rng.integers(0, n_iolets, size=shape) + IOLET0
    lab = np.where((lab == WALL) & (rng.random(shape) < 0.4), io, lab).astype(np.uint8)
    border = np.ones(shape, bool)
    border[1:-1, 1:-1, 1:-1] = False
    lab[border] = np.where(rng.random(int(border.sum())) < 0.5, WALL,
                           rng.integers(0, n_iolets, int(border.sum())) + IOLET0)
    seg = rng.integers(0, 3, size=shape).astype(np.uint16)
    w = rng.uniform(0.0, 2.0, size=shape).astype(np.float32)
    geo = Geometry(labels=lab, segment=seg, iolet_weight=w, n_seg=3)
    geo.iolets = [dict(id=i, role="any", direction=tuple(d)) for i, d in
                  enumerate(_unit_rows(rng, n_iolets))]
    return geo


def separate_iolets(geo: Geometry) -> Geometry:
    """Turns iolet voxels into wall voxels until no fluid voxel has upstream
    neighbours in two different iolets (the GPU library allows one iolet per
    site).  Deterministic: the higher id loses."""
    lab = geo.labels
    nz, ny, nx = lab.shape
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if 0 < dx * dx + dy * dy + dz * dz <= 2]
    changed = True
    while changed:
        changed = False
        for z, y, x in zip(*np.nonzero(lab == FLUID)):
            seen = {}
            for dx, dy, dz in offs:
                v = int(lab[z - dz, y - dy, x - dx])
                if v >= IOLET0:
                    seen.setdefault(v, []).append((z - dz, y - dy, x - dx))
            if len(seen) > 1:
                for v in sorted(seen)[1:]:
                    for zz, yy, xx in seen[v]:
                        lab[zz, yy, xx] = WALL
                changed = True
    return geo


def _unit_rows(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def mirror_x(geo: Geometry) -> Geometry:
    """The same geometry reflected in x (normals and directions reflected)."""
    g = Geometry(labels=geo.labels[:, :, ::-1].copy(), n_seg=geo.n_seg, info=dict(geo.info))
    if geo.segment is not None:
        g.segment = geo.segment[:, :, ::-1].copy()
    if geo.iolet_weight is not None:
        g.iolet_weight = geo.iolet_weight[:, :, ::-1].copy()
    if geo.normal is not None:
        n = geo.normal[:, :, ::-1].copy()
        n[..., 0] *= -1
        g.normal = n
    g.iolets = [dict(io, direction=(-io["direction"][0], io["direction"][1], io["direction"][2]))
                for io in geo.iolets]
    return g


def density_perturbation(n: int, seed: int, amplitude: float = 1e-6) -> np.ndarray:
    """rho_0 = 1 + U(-amplitude, amplitude) per site (seeded)."""
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amplitude, amplitude, size=n)


def log_uniform(rng: np.random.Generator, lo: float, hi: float, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))
