"""Rigid against elastic wall shear stress, site by site (Sec. 3, Fig. 11: the
paper's pointwise comparison of instantaneous wall shear stress in its
arterial geometry finds it generally higher with rigid walls), with the
elastic wall applied both with one global F and with a local F per vessel
from the Sec. 2.3 relation (the Sec. 4 discussion).

Each workload runs three times from rest to a periodic state (cycle-to-cycle
change of u and p below 1e-3): bounce-back walls, elastic walls with the
workload's F, elastic walls with F per segment (M calibrated so that the
relation gives the paper's F = 0.85 for its alpha = 3 cylinder of radius 50
spacings).  The drive is the same velocity inlet in all three, so the flow
through the vessels is the same.  During one further cycle the wall shear
stress at every site with a wall link is sampled at evenly spaced phases.

    python -m paper_2108_08783_amd.wall_shear --workloads tube tree --out r.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np

from . import inputs, lbm, slip, workloads
from .warmstart import run_to_periodic

# the paper's verification cylinder: F = 0.85 at alpha = 3, radius 50
CALIBRATION = dict(F=0.85, alpha=3.0, radius=50.0)


def wall_sites(geo: inputs.Geometry) -> np.ndarray:
    """Canonical indices of the fluid sites with at least one wall link
    (an upstream voxel x - c_i labelled wall)."""
    lab = geo.labels
    fl = lab == inputs.FLUID
    wall = np.pad(lab == inputs.WALL, 1)
    nz, ny, nx = lab.shape
    hit = np.zeros_like(fl)
    for dx, dy, dz in inputs._OFFS18:
        hit |= wall[1 - dz:1 - dz + nz, 1 - dy:1 - dy + ny, 1 - dx:1 - dx + nx]
    return np.flatnonzero((hit & fl)[fl])


def compare(a: np.ndarray, b: np.ndarray, floor: float) -> dict:
    """Pointwise statistics of a against b over the sites where b > floor."""
    sel = b > floor
    a, b = a[sel].astype(np.float64), b[sel].astype(np.float64)
    r = a / b
    return dict(sites=int(sel.sum()), frac_lower=float(np.mean(a < b)),
                median_ratio=float(np.median(r)), p10_ratio=float(np.percentile(r, 10)),
                p90_ratio=float(np.percentile(r, 90)),
                slope=float(np.dot(a, b) / np.dot(b, b)),
                corr=float(np.corrcoef(a, b)[0, 1]),
                mean_a=float(a.mean()), mean_b=float(b.mean()))


def sample_cycle(lat: lbm.Lattice, sites: np.ndarray, period: int, phases: int):
    """WSS at the given sites at `phases` evenly spaced phases of one cycle
    (float32 [phases, n]) and the extension Delta r there at each phase."""
    step = period // phases
    W = np.zeros((phases, len(sites)), np.float32)
    D = np.zeros((phases, len(sites)), np.float32)
    for j in range(phases):
        _, _, wss, dr = lat.read_fields(0)
        W[j] = wss[sites]
        D[j] = dr[sites]
        lat.step(step)
    lat.step(period - step * phases)
    return W, D


def study(wl: workloads.Workload, dtype="f32", phases=8, tol=1e-3, max_cycles=16,
          log=print) -> dict:
    g = wl.geoms[0]
    base = wl.params[0]
    period = int(base.iolets[0]["period"])
    nu = (wl.tau - 0.5) / 3.0
    M = slip.calibrate_M(CALIBRATION["F"], CALIBRATION["alpha"],
                         slip.dr_over_R(CALIBRATION["radius"]))
    F_loc = slip.segment_F(g, M, period, nu)
    runs = {"rigid": dataclasses.replace(base, mode=lbm.BOUNCEBACK, F_seg=None),
            "elastic_global": dataclasses.replace(base, F_seg=None),
            "elastic_local": dataclasses.replace(base, F_seg=list(F_loc))}
    sites = wall_sites(g)
    t0 = time.perf_counter()
    lat = lbm.Lattice(wl.geoms, dtype=dtype, tau=wl.tau)
    log(f"{wl.name}: {g.n_fluid} sites, {len(sites)} wall sites, context in "
        f"{time.perf_counter() - t0:.1f} s")
    out = dict(workload=wl.name, sites=g.n_fluid, wall_sites=int(len(sites)), dtype=dtype,
               period=period, phases=phases, M=M, F_global=base.F,
               F_local=dict(min=float(F_loc.min()), max=float(F_loc.max()),
                            mean=float(F_loc.mean())), runs={})
    W = {}
    for name, p in runs.items():
        one = dataclasses.replace(wl, params=[p])
        workloads.apply(lat, one)
        t0 = time.perf_counter()
        res = run_to_periodic(lat, 1, period, tol, max_cycles,
                              log=lambda s, n=name: log(f"  {n}: {s}"))
        W[name], D = sample_cycle(lat, sites, period, phases)
        out["runs"][name] = dict(cycles=res.cycles[0], seconds=time.perf_counter() - t0,
                                 wss_mean=float(W[name].mean()),
                                 dr_max=float(D.max()),
                                 dE_p99=float(np.percentile(np.maximum(D - 1, 0), 99)))
        log(f"  {name}: periodic after {res.cycles[0]} cycles, mean WSS "
            f"{W[name].mean():.3e}, max Delta r {D.max():.4f}")
    lat.close()
    peak = phases // 4                      # sin(2 pi t / T) = 1: peak inlet flow
    tawss = {k: v.mean(axis=0) for k, v in W.items()}
    floor = 1e-3 * float(tawss["rigid"].max())
    out["peak_phase"] = peak
    for a, b in (("elastic_global", "rigid"), ("elastic_local", "rigid"),
                 ("elastic_local", "elastic_global")):
        key = f"{a}_vs_{b}"
        out[key] = dict(peak=compare(W[a][peak], W[b][peak], floor),
                        time_mean=compare(tawss[a], tawss[b], floor))
        s = out[key]["peak"]
        log(f"  {key} at peak flow: lower at {100 * s['frac_lower']:.1f}% of sites, median "
            f"ratio {s['median_ratio']:.3f}, slope {s['slope']:.3f}, corr {s['corr']:.3f}, "
            f"means {s['mean_a']:.3e} / {s['mean_b']:.3e}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workloads", nargs="+", default=["tube", "tree"])
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--phases", type=int, default=8)
    ap.add_argument("--scale", type=float, default=1.0, help="tree scale")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = {}
    for name in a.workloads:
        wl = workloads.tube32() if name == "tube" else workloads.tree(scale=a.scale)
        res[name] = study(wl, a.dtype, a.phases, log=lambda s: print(s, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()
