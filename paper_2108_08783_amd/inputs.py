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
    segments: Optional[list] = None         # tube segments the shape was built from
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


# ------------------------------------------------------ branching vessels --
@dataclasses.dataclass
class Segment:
    p0: np.ndarray          # start point (x, y, z) in voxel units
    p1: np.ndarray          # end point
    r0: float               # radius at p0
    r1: float               # radius at p1
    gen: int = 0            # generation (root 0)
    outlet: bool = False    # flat end with an outlet cap
    inlet: bool = False     # flat start on the inlet plane
    sid: int = 0


def _rot(v, axis, ang):
    """Rotate v about unit axis by ang (Rodrigues)."""
    axis = axis / np.linalg.norm(axis)
    return (v * math.cos(ang) + np.cross(axis, v) * math.sin(ang)
            + axis * np.dot(axis, v) * (1 - math.cos(ang)))


def _perp(d):
    a = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    p = np.cross(d, a)
    return p / np.linalg.norm(p)


def voxelise(segments: List[Segment], shape, iolet_of_segment=None) -> Geometry:
    """Union of tapered round-ended tubes.  Outlet segments end flat at p1
    with an outlet cap (one voxel layer beyond the end plane); the inlet
    segment starts flat on the inlet plane x = 0.  Segment id = first
    segment containing the voxel.  Inlet weights are parabolic in the
    distance from the inlet segment's axis."""
    nz, ny, nx = shape
    lab = np.zeros(shape, np.uint8)
    seg = np.zeros(shape, np.uint16)
    claimed = np.zeros(shape, bool)
    iw = np.zeros(shape, np.float32)
    iolets = []
    next_io = 1  # 0 is the inlet

    def bbox(pts, pad):
        lo = np.floor(np.min(pts, 0) - pad).astype(int)
        hi = np.ceil(np.max(pts, 0) + pad).astype(int) + 1
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, [nx, ny, nz])
        return lo, hi

    def local(s, lo, hi):
        z, y, x = np.ogrid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        d = s.p1 - s.p0
        dd = float(d @ d)
        rx, ry, rz = x - s.p0[0], y - s.p0[1], z - s.p0[2]
        t = (rx * d[0] + ry * d[1] + rz * d[2]) / dd
        return rx, ry, rz, t, d, dd

    # outlet caps first (fluid overrides them)
    for s in segments:
        if not s.outlet:
            continue
        io = next_io
        next_io += 1
        lo, hi = bbox([s.p1], s.r1 + 3)
        rx, ry, rz, t, d, dd = local(s, lo, hi)
        L = math.sqrt(dd)
        ax = t * L
        px, py, pz = rx - t * d[0], ry - t * d[1], rz - t * d[2]
        rad2 = px * px + py * py + pz * pz
        cap = (ax > L) & (ax <= L + 1.8) & (rad2 < (s.r1 + 1.8) ** 2)
        sub = lab[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[cap] = IOLET0 + io
        iolets.append(dict(id=io, role="outlet", direction=tuple(-d / L), segment=s.sid,
                           box=(lo, hi)))
    for s in segments:
        r_max = max(s.r0, s.r1)
        lo, hi = bbox([s.p0, s.p1], r_max + 2)
        rx, ry, rz, t, d, dd = local(s, lo, hi)
        tc = np.clip(t, 0.0, 1.0)
        px, py, pz = rx - tc * d[0], ry - tc * d[1], rz - tc * d[2]
        rad2 = px * px + py * py + pz * pz
        r = s.r0 + tc * (s.r1 - s.r0)
        inside = rad2 < r * r
        if s.outlet:
            inside &= t <= 1.0
        z0, y0, x0 = lo[2], lo[1], lo[0]
        sl = (slice(z0, hi[2]), slice(y0, hi[1]), slice(x0, hi[0]))
        if s.inlet:
            xs = np.arange(lo[0], hi[0])[None, None, :]
            inside &= xs >= 1
            w = np.where(inside, 2.0 * (1.0 - rad2 / (s.r0 * s.r0)), 0.0)
            iw[sl] = np.maximum(iw[sl], np.clip(w, 0.0, None).astype(np.float32))
        new = inside & ~claimed[sl]
        seg[sl][new] = s.sid
        claimed[sl] |= inside
        lab[sl][inside] = FLUID
    # inlet plane x = 0 (around the inlet segment)
    for s in segments:
        if s.inlet:
            lo, hi = bbox([s.p0], s.r0 + 3)
            y, z = np.ogrid[lo[1]:hi[1], lo[2]:hi[2]]
            disk = (y - s.p0[1]) ** 2 + (z - s.p0[2]) ** 2 < (s.r0 + 1.8) ** 2
            plane = lab[lo[2]:hi[2], lo[1]:hi[1], 0]
            plane[disk.T] = IOLET0 + 0
            iolets.insert(0, dict(id=0, role="inlet", direction=tuple((s.p1 - s.p0) /
                                                                      np.linalg.norm(s.p1 - s.p0))))
    _resolve_iolet_conflicts(lab)
    # an outlet whose cap lost every voxel next to fluid to another iolet is
    # closed: drop it from the list and from its segment
    segments = list(segments)
    kept = []
    for io in iolets:
        if io["role"] == "outlet":
            lo, hi = io.pop("box")
            if not _touches_fluid(lab, IOLET0 + io["id"], lo, hi):
                k = next(i for i, q in enumerate(segments) if q.sid == io["segment"])
                segments[k] = dataclasses.replace(segments[k], outlet=False)
                continue
        kept.append(io)
    g = Geometry(labels=lab, segment=seg, iolet_weight=iw, n_seg=len(segments))
    g.iolets = kept
    g.segments = segments
    return g


def _touches_fluid(lab, code, lo, hi):
    """Whether a voxel labelled `code` inside the box [lo, hi) (x, y, z
    order) has a fluid voxel among its 18 neighbours."""
    nz, ny, nx = lab.shape
    z0, y0, x0 = max(lo[2] - 1, 0), max(lo[1] - 1, 0), max(lo[0] - 1, 0)
    z1, y1, x1 = min(hi[2] + 1, nz), min(hi[1] + 1, ny), min(hi[0] + 1, nx)
    sub = lab[z0:z1, y0:y1, x0:x1]
    mine = sub == code
    if not mine.any():
        return False
    fl = np.pad(sub == FLUID, 1)
    Z, Y, X = sub.shape
    for dx, dy, dz in _OFFS18:
        if (mine & fl[1 + dz:1 + dz + Z, 1 + dy:1 + dy + Y, 1 + dx:1 + dx + X]).any():
            return True
    return False


_OFFS18 = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
           if 0 < dx * dx + dy * dy + dz * dz <= 2]


def _resolve_iolet_conflicts(lab):
    """A fluid voxel whose upstream
    neighbours lie in two different iolets loses the higher-id iolet voxels
    (they become wall).  Only the neighbourhoods of iolet voxels are
    examined."""
    zz, yy, xx = np.nonzero(lab >= IOLET0)
    if len(zz) == 0:
        return
    nz, ny, nx = lab.shape
    ids = lab[zz, yy, xx]
    for v in np.unique(ids):
        sel = ids == v
        lo = np.maximum([zz[sel].min() - 3, yy[sel].min() - 3, xx[sel].min() - 3], 0)
        hi = np.minimum([zz[sel].max() + 4, yy[sel].max() + 4, xx[sel].max() + 4], [nz, ny, nx])
        _resolve_region(lab[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]])


def _resolve_region(lab):
    for _ in range(8):
        if min(lab.shape) < 3:
            return
        inner = lab[1:-1, 1:-1, 1:-1]
        fl = inner == FLUID
        lo = np.full(inner.shape, 255, np.uint8)
        hi = np.zeros(inner.shape, np.uint8)
        nz, ny, nx = lab.shape
        for dx, dy, dz in _OFFS18:
            nb = lab[1 - dz:nz - 1 - dz, 1 - dy:ny - 1 - dy, 1 - dx:nx - 1 - dx]
            io = nb >= IOLET0
            np.minimum(lo, np.where(io, nb, 255), out=lo)
            np.maximum(hi, np.where(io, nb, 0), out=hi)
        bad = fl & (hi > lo) & (lo < 255)
        if not bad.any():
            return
        zz, yy, xx = np.nonzero(bad)
        for z, y, x in zip(zz + 1, yy + 1, xx + 1):
            h = hi[z - 1, y - 1, x - 1]
            for dx, dy, dz in _OFFS18:
                if lab[z - dz, y - dy, x - dx] == h:
                    lab[z - dz, y - dy, x - dx] = WALL


def murray_tree(seed: int, scale: float = 1.0, generations: int = 4, root_radius: float = 40.0,
                box=(1200, 400, 400), angle_range=(30.0, 70.0), length_factor: float = 8.9,
                stubs_per_leaf: int = 3, max_tries: int = 50, pull: float = 1.0):
    """Bifurcating tapered tree with Murray's-law radii, r_g = r_root 2^(-g/3)
    (each segment tapers by 2^(-1/6) along its length), segment lengths
    length_factor r_g U(0.9, 1.1), branch angle (between daughters)
    U(angle_range) about a downstream bisector pulled toward the box axis,
    bifurcation planes turned 90 degrees per generation, and
    at every leaf end a trifurcation into stubs of radius r 3^(-1/3) and length
    4 r, each ending in a fixed-density outlet.  The root runs along +x from
    the inlet plane x = 0.  Everything is scaled by ``scale``.  Returns the
    Geometry with one segment id per tube; redraws until the tree fits the
    box with a 4-voxel margin."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(round(b * scale)) for b in box)
    R0 = root_radius * scale
    for _ in range(max_tries):
        segs: List[Segment] = []
        c = np.array([0.0, (ny - 1) / 2.0, (nz - 1) / 2.0])

        def grow(p0, d, gen, normal):
            r = R0 * 2.0 ** (-gen / 3.0)
            L = length_factor * r * rng.uniform(0.9, 1.1)
            r_end = r * 2.0 ** (-1.0 / 6.0)
            p1 = p0 + d * L
            s = Segment(p0=p0, p1=p1, r0=r, r1=r_end, gen=gen, inlet=(gen == 0),
                        sid=len(segs))
            segs.append(s)
            if gen + 1 < generations + 1:
                half = math.radians(rng.uniform(*angle_range)) / 2.0
                # daughters at +-half about a bisector that runs downstream
                # (+x) and is pulled back toward the box axis
                lat = p1 - c
                lat[0] = 0.0
                b = np.array([1.0, 0.0, 0.0]) - pull * lat / (0.5 * min(ny, nz))
                b /= np.linalg.norm(b)
                nrm = _rot(normal, d, math.pi / 2.0)
                nrm = nrm - (nrm @ b) * b
                nrm /= np.linalg.norm(nrm)
                for sgn in (+1, -1):
                    grow(p1, _rot(b, nrm, sgn * half), gen + 1, nrm)
            else:
                rs = r_end * 3.0 ** (-1.0 / 3.0)
                for k in range(stubs_per_leaf):
                    ang = 2 * math.pi * k / stubs_per_leaf
                    off = _rot(normal, d, ang)
                    ds = d * math.cos(math.radians(35)) + off * math.sin(math.radians(35))
                    ds /= np.linalg.norm(ds)
                    segs.append(Segment(p0=p1, p1=p1 + ds * 4.0 * rs, r0=rs, r1=rs, gen=gen + 1,
                                        outlet=True, sid=len(segs)))

        grow(c, np.array([1.0, 0.0, 0.0]), 0, np.array([0.0, 1.0, 0.0]))
        pts = np.array([s.p1 for s in segs] + [s.p0 for s in segs])
        rad = max(s.r0 for s in segs[1:])
        lo = pts.min(0) - rad - 4
        hi = pts.max(0) + rad + 4
        if lo[1] >= 0 and lo[2] >= 0 and hi[0] <= nx - 1 and hi[1] <= ny - 1 and hi[2] <= nz - 1:
            break
    else:
        raise RuntimeError("tree does not fit the box")
    # the root starts on the inlet plane: extend it back so x = 1 is inside
    segs[0].p0 = segs[0].p0 - np.array([2.0, 0.0, 0.0])
    g = voxelise(segs, (nz, ny, nx))
    g.info = dict(kind="murray_tree", seed=seed, scale=scale, generations=generations,
                  n_segments=len(segs), box=(nx, ny, nz))
    return g


def bifurcation(r: float, length: float, angle_deg: float, margin: int = 3) -> Geometry:
    """Single bifurcation: a parent tube of radius r and length length/2
    along +x from the inlet plane, two daughters of radius r 2^(-1/3) and
    length length/2 at +-angle/2, each ending in a fixed-density outlet."""
    rc = r * 2.0 ** (-1.0 / 3.0)
    half = math.radians(angle_deg) / 2.0
    Lp, Lc = length / 2.0, length / 2.0
    p_end = np.array([Lp, 0.0, 0.0])
    ends = [p_end + Lc * np.array([math.cos(half), s * math.sin(half), 0.0]) for s in (1, -1)]
    ymax = max(abs(e[1]) for e in ends) + rc + margin + 2
    nx = int(math.ceil(max(e[0] for e in ends) + rc + margin + 3))
    ny = int(math.ceil(2 * max(ymax, r + margin + 2))) + 1
    nz = int(math.ceil(2 * (r + margin + 2))) + 1
    c = np.array([0.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    segs = [Segment(p0=c - np.array([2.0, 0, 0]), p1=c + p_end, r0=r, r1=r, inlet=True, sid=0)]
    for k, e in enumerate(ends):
        segs.append(Segment(p0=c + p_end, p1=c + e, r0=rc, r1=rc, gen=1, outlet=True, sid=k + 1))
    g = voxelise(segs, (nz, ny, nx))
    g.info = dict(kind="bifurcation", r=r, length=length, angle=angle_deg)
    return g


def straight_tube_x(r: float, length: float, margin: int = 3) -> Geometry:
    """Straight tube along +x from the inlet plane x = 0, radius r, flat
    outlet cap at the far end."""
    n = int(math.ceil(2 * (r + margin + 2))) + 1
    nx = int(math.ceil(length + margin + 4))
    c = np.array([0.0, (n - 1) / 2.0, (n - 1) / 2.0])
    segs = [Segment(p0=c - np.array([2.0, 0, 0]), p1=c + np.array([length, 0.0, 0.0]), r0=r,
                    r1=r, inlet=True, outlet=True, sid=0)]
    g = voxelise(segs, (n, n, nx))
    g.info = dict(kind="tube", r=r, length=length)
    return g


def batch(seed: int, n: int = 64, target_sites: float = 20e6, r_range=(6.0, 24.0),
          lr_range=(8.0, 16.0), angle_range=(30.0, 70.0), k_range=(1e-3, 1e-1),
          u0_range=(0.01, 0.03), tol: float = 0.05):
    """Uneven batch: half straight tubes, half single bifurcations, radius
    U(r_range), length/radius U(lr_range); all lengths are then scaled by
    one common factor so that the total site count is target_sites within
    tol (the stated radius and length distributions alone give about 12M
    sites for 64 instances).  Per instance: stiffness log-uniform in
    k_range, inlet amplitude U(u0_range).  Returns (geometries, params)."""
    rng = np.random.default_rng(seed)
    kinds = ["tube"] * (n // 2) + ["bif"] * (n - n // 2)
    rng.shuffle(kinds)
    r = rng.uniform(*r_range, size=n)
    lr = rng.uniform(*lr_range, size=n)
    ang = rng.uniform(*angle_range, size=n)
    k = log_uniform(rng, *k_range, size=n)
    u0 = rng.uniform(*u0_range, size=n)

    def est(kind, ri, Li):  # volume estimate
        if kind == "tube":
            return math.pi * ri * ri * Li
        rc = ri * 2 ** (-1 / 3)
        return math.pi * ri * ri * Li / 2 + 2 * math.pi * rc * rc * Li / 2

    base = sum(est(kd, ri, ri * li) for kd, ri, li in zip(kinds, r, lr))
    s = target_sites / base if target_sites else 1.0
    for _ in range(6):
        geos = []
        for kd, ri, li, ai in zip(kinds, r, lr, ang):
            L = ri * li * s
            geos.append(straight_tube_x(ri, L) if kd == "tube" else bifurcation(ri, L, ai))
        tot = sum(g.n_fluid for g in geos)
        if not target_sites or abs(tot / target_sites - 1) <= tol:
            break
        s *= target_sites / tot
    params = [dict(kind=kd, r=float(ri), length=float(ri * li * s), angle=float(ai), k=float(ki),
                   u0=float(ui)) for kd, ri, li, ai, ki, ui in zip(kinds, r, lr, ang, k, u0)]
    return geos, params
