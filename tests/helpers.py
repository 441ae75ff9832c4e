"""Shared set-up for parity tests: the same seeded problem is handed to the
GPU library and to the FP64 oracle (which share no code)."""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

import oracle
from paper_2108_08783_amd import inputs
from paper_2108_08783_amd import lbm


@dataclasses.dataclass
class Problem:
    geo: inputs.Geometry
    tau: float = 0.8
    mode: int = lbm.BOUNCEBACK
    F: float = 0.0
    P0: float = 1.0 / 3.0
    k: List[float] = dataclasses.field(default_factory=lambda: [1.0])
    iolets: Dict[int, dict] = dataclasses.field(default_factory=dict)
    rho0: Optional[np.ndarray] = None
    u0: Optional[np.ndarray] = None
    F_seg: Optional[List[float]] = None     # slip ratio per segment


def make_oracle(p: Problem) -> oracle.Oracle:
    g = p.geo
    o = oracle.Oracle(g.labels, p.tau, segment=g.segment, normal=g.normal,
                      iolet_weight=g.iolet_weight)
    o.set_wall(p.mode, F=p.F, P0=p.P0, k=p.k)
    if p.F_seg is not None:
        o.set_wall_F(p.F_seg)
    for i, q in p.iolets.items():
        o.set_iolet(i, q["kind"], q["a0"], q.get("amp", 0.0), q.get("period", 1.0),
                    q.get("phase", 0.0), q.get("direction", (0.0, 0.0, 0.0)))
    o.init_fields(p.rho0, p.u0)
    return o


def configure(lat: lbm.Lattice, inst: int, p: Problem, init=True):
    lat.set_wall(inst, p.mode, F=p.F, P0=p.P0, k=p.k)
    if p.F_seg is not None:
        lat.set_wall_F(inst, p.F_seg)
    for i, q in p.iolets.items():
        lat.set_iolet(inst, i, q["kind"], q["a0"], q.get("amp", 0.0), q.get("period", 1.0),
                      q.get("phase", 0.0), q.get("direction"))
    if init:
        lat.init_fields(inst, p.rho0, p.u0)


def make_lattice(problems: List[Problem], dtype: str, resources: str = "torch") -> lbm.Lattice:
    taus = {p.tau for p in problems}
    assert len(taus) == 1
    lat = lbm.Lattice([p.geo for p in problems], dtype=dtype, tau=problems[0].tau,
                      resources=resources)
    # all wall modes first (a mode change rebuilds the tables once), then
    # the initial states
    for k, p in enumerate(problems):
        configure(lat, k, p, init=False)
    for k, p in enumerate(problems):
        lat.init_fields(k, p.rho0, p.u0)
    return lat


def rel_linf(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def errors(gpu, ref, P0=1.0 / 3.0):
    """Relative L-infinity errors stated separately per result."""
    rho_g, u_g, w_g, d_g = gpu
    rho_r, u_r, w_r, d_r = ref
    out = dict(u=rel_linf(u_g, u_r), p=rel_linf(rho_g / 3, rho_r / 3),
               dp=rel_linf(rho_g / 3 - P0, rho_r / 3 - P0))
    if w_g is not None:
        out["wss"] = rel_linf(w_g, w_r)
    if d_g is not None:
        out["dr"] = rel_linf(d_g, d_r)
    return out


def tube_problem(R, L, *, seed=0, mode=lbm.ELASTIC, pulsatile=True, period=400.0, F=0.85):
    """Elastic straight tube with a pulsatile parabolic velocity inlet and a
    fixed-density outlet (the shape of the 1.65M-site tube workload)."""
    g = inputs.cylinder(R, L)
    rng = np.random.default_rng(seed)
    k = float(inputs.log_uniform(rng, 1e-3, 1e-1))
    io = {0: dict(kind=lbm.VELOCITY, a0=0.02, amp=0.5 if pulsatile else 0.0, period=period,
                  direction=(0.0, 0.0, 1.0)),
          1: dict(kind=lbm.DENSITY, a0=1.0, direction=(0.0, 0.0, -1.0))}
    return Problem(geo=g, tau=0.8, mode=mode, F=F, P0=1.0 / 3.0, k=[k], iolets=io)


def poiseuille_problem(mode, seed=0):
    """Steady density-driven R=8, L=64 tube (12,352 sites), tau = 0.8, inlet
    1.001 / outlet 0.999, rho0 = 1 + U(-1e-6, 1e-6)."""
    g = inputs.cylinder(8, 64)
    rho0 = inputs.density_perturbation(g.n_fluid, seed)
    io = {0: dict(kind=lbm.DENSITY, a0=1.001, direction=(0.0, 0.0, 1.0)),
          1: dict(kind=lbm.DENSITY, a0=0.999, direction=(0.0, 0.0, -1.0))}
    return Problem(geo=g, tau=0.8, mode=mode, F=0.85, P0=0.999 / 3.0, k=[1e-2], iolets=io,
                   rho0=rho0)


def one_iolet_per_site(geo: inputs.Geometry) -> inputs.Geometry:
    """The library's limit (a fluid site may touch one iolet only), applied
    to a random geometry for the GPU tests: iolet voxels become wall until
    no fluid voxel has upstream neighbours in two different iolets (the
    higher id loses).  The shared generator itself is not restricted; the
    oracle accepts any labels, and a CPU test checks that the library
    rejects the unrestricted boxes."""
    lab = geo.labels
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if 0 < dx * dx + dy * dy + dz * dz <= 2]
    changed = True
    while changed:
        changed = False
        for z, y, x in zip(*np.nonzero(lab == inputs.FLUID)):
            seen = {}
            for dx, dy, dz in offs:
                v = int(lab[z - dz, y - dy, x - dx])
                if v >= inputs.IOLET0:
                    seen.setdefault(v, []).append((z - dz, y - dy, x - dx))
            if len(seen) > 1:
                for v in sorted(seen)[1:]:
                    for zz, yy, xx in seen[v]:
                        lab[zz, yy, xx] = inputs.WALL
                changed = True
    return geo


def random_box_problem(seed, mode=lbm.ELASTIC, shape=(9, 10, 11)):
    rng = np.random.default_rng(seed)
    g = one_iolet_per_site(inputs.random_labels(shape, rng))
    io = {0: dict(kind=lbm.DENSITY, a0=1.002, amp=0.3, period=17.0, phase=0.4),
          1: dict(kind=lbm.VELOCITY, a0=0.03, amp=0.5, period=11.0, phase=-1.0,
                  direction=g.iolets[1]["direction"])}
    # only iolets that some fluid site links to (a label with no fluid
    # neighbour is rejected by the library as a mis-set iolet)
    hi = g.labels.shape[::-1]
    present = {i for i in (0, 1) if inputs._touches_fluid(g.labels, 2 + i, (0, 0, 0), hi)}
    io = {k: v for k, v in io.items() if k in present}
    n = g.n_fluid
    u0 = 0.02 * rng.uniform(-1, 1, (n, 3))
    rho0 = 1 + 0.01 * rng.uniform(-1, 1, n)
    return Problem(geo=g, tau=0.7, mode=mode, F=0.6, P0=0.331, k=[0.02, 0.005, 1e-3],
                   iolets=io, rho0=rho0, u0=u0)
