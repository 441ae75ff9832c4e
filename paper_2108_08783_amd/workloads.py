"""Named synthetic workloads: geometries plus per-instance wall and drive
parameters, applied to a ``lbm.Lattice``.

  tube32   elastic straight cylinder R=32, L=512 (1,640,960 sites), pulsatile
           parabolic velocity inlet u(t) = 0.02 (1 + 0.5 sin(2 pi t/4000)),
           fixed-density outlet, stiffness log-uniform [1e-3, 1e-1], F=0.85;
  tree     4-generation Murray tree in a 1200x400x400 box (~7.5M sites),
           per-segment stiffness, the same pulsatile inlet, 48 fixed-density
           outlets, F=0.5;
  sweep    64 uneven tubes and single bifurcations (~20M sites), per-instance
           stiffness and inlet amplitude u0 in [0.01, 0.03], F=0.5.

All use D3Q19 BGK with tau = 0.8 and lattice units.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

from . import inputs
from . import lbm

PERIOD = 4000.0


@dataclasses.dataclass
class InstanceParams:
    mode: int
    F: float
    P0: float
    k: List[float]
    iolets: Dict[int, dict]
    F_seg: Optional[List[float]] = None     # slip ratio per segment (else F)


@dataclasses.dataclass
class Workload:
    name: str
    geoms: List[inputs.Geometry]
    params: List[InstanceParams]
    tau: float = 0.8
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n_sites(self):
        return sum(g.n_fluid for g in self.geoms)


def _drive(g, u0, period=PERIOD, amp=0.5):
    io = {0: dict(kind=lbm.VELOCITY, a0=u0, amp=amp, period=period,
                  direction=tuple(g.iolets[0]["direction"]))}
    for d in g.iolets[1:]:
        # fixed-density outlets with their inward normal (only the velocity
        # along it enters the outlet node)
        io[d["id"]] = dict(kind=lbm.DENSITY, a0=1.0, direction=tuple(d["direction"]))
    return io


def tube32(seed=1, R=32, L=512, period=PERIOD):
    g = inputs.cylinder(R, L)
    rng = np.random.default_rng(seed)
    k = float(inputs.log_uniform(rng, 1e-3, 1e-1))
    p = InstanceParams(lbm.ELASTIC, 0.85, 1.0 / 3.0, [k], _drive(g, 0.02, period))
    return Workload(f"tube R={R} L={L}", [g], [p], info=dict(seed=seed, k=k))


def tree(seed=3, scale=1.0, period=PERIOD):
    g = inputs.murray_tree(seed, scale=scale)
    rng = np.random.default_rng(seed)
    k = list(map(float, inputs.log_uniform(rng, 1e-3, 1e-1, size=g.n_seg)))
    p = InstanceParams(lbm.ELASTIC, 0.5, 1.0 / 3.0, k, _drive(g, 0.02, period))
    return Workload(f"murray tree seed {seed} scale {scale}", [g], [p],
                    info=dict(seed=seed, scale=scale))


def trees(seeds, scale=1.0, period=PERIOD):
    """Several Murray trees (as `tree`) as the instances of one workload."""
    wls = [tree(sd, scale, period) for sd in seeds]
    return Workload(f"{len(wls)} murray trees seeds {list(seeds)} scale {scale}",
                    [w.geoms[0] for w in wls], [w.params[0] for w in wls],
                    info=dict(seeds=list(seeds), scale=scale))


def sweep(seed=4, n=64, target_sites=20e6, period=PERIOD):
    geos, prm = inputs.batch(seed, n=n, target_sites=target_sites)
    params = [InstanceParams(lbm.ELASTIC, 0.5, 1.0 / 3.0, [q["k"]] * g.n_seg,
                             _drive(g, q["u0"], period)) for g, q in zip(geos, prm)]
    return Workload(f"sweep of {n} tubes/bifurcations seed {seed}", geos, params,
                    info=dict(seed=seed, instances=prm))


def apply(lat: lbm.Lattice, wl: Workload, init=True):
    # every wall mode first: a mode change rebuilds the tables of all
    # instances at the next initialisation or step, so initialise after
    for k, p in enumerate(wl.params):
        lat.set_wall(k, p.mode, F=p.F, P0=p.P0, k=p.k)
        if p.F_seg is not None:
            lat.set_wall_F(k, p.F_seg)
        for i, q in p.iolets.items():
            lat.set_iolet(k, i, q["kind"], q["a0"], q.get("amp", 0.0), q.get("period", 1.0),
                          q.get("phase", 0.0), q.get("direction"))
    if init:
        for k in range(len(wl.params)):
            lat.init_fields(k)


def lattice(wl: Workload, dtype="f32") -> lbm.Lattice:
    lat = lbm.Lattice(wl.geoms, dtype=dtype, tau=wl.tau)
    apply(lat, wl)
    return lat
