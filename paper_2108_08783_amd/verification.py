"""The paper's verification cylinder (Sec. 2.4 with the Table A1 lattice
parameters) on one GPU.

* `womersley`: the R = 50 dx cylinder (3 mm radius, 4 cm long, lattice
  spacing 60 um, time step 11 us, tau 0.537, 5.2M sites) driven by an
  oscillating pressure gradient of amplitude |k_p| (period pi/2 s, Womersley
  number 3), with rigid (bounce-back) or elastic walls (F = 0.85, stiffness
  from Y = 20 kPa, h = 0.1 R, sigma = 0.5).  After the start-up transient
  the axial velocity in the centre plane is compared at 5 phases of a period
  with the rigid-tube Womersley solution for the gradient measured at that
  plane.  The paper's elastic analytical solution needs an elasticity
  factor and a wave speed that the paper does not define, so the elastic
  run is reported against the rigid solution (its near-wall slip is the
  difference).
* `timing`: walltime of 1000 iterations of the R = 50, 100 and 200 dx
  cylinders, elastic and rigid (the paper's Table 1 measures the same on
  3,072 - 12,000 CPU cores).

Unit conversions: lattice viscosity nu dt/dx^2 = (tau - 1/2)/3 (Sec. 2.1
eq. Viscosity); pressure unit rho dx^2/dt^2, so a gradient in Pa/m becomes
G dt^2/(rho dx) and the wall stiffness k = Y h/((1 - sigma^2) R^2) (Sec. 2.4)
becomes k dt^2/(rho dx).
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import inputs, slip
from . import lbm

# Sec. 2.4 (fluid and wall) and Table A1 (lattice spacing and time step)
R_M, LENGTH_M = 3.0e-3, 0.04
RHO, MU = 1000.0, 0.004
PERIOD_S = math.pi / 2
YOUNG, H_OVER_R, POISSON = 20.0e3, 0.1, 0.5
F_WALL = 0.85
RESOLUTIONS = {50: (6.0e-5, 1.10e-5), 100: (3.0e-5, 5.48e-6), 200: (1.5e-5, 2.74e-6)}
# Table 1: seconds per 1000 iterations (elastic, rigid) on 3,072 / 6,000 /
# 12,000 Skylake cores
PAPER_TABLE1 = {50: (0.9770, 0.9781), 100: (3.159, 3.385), 200: (10.656, 11.446)}


@dataclasses.dataclass
class Case:
    R: int                # radius in lattice units
    L: int                # fluid length in lattice units
    dx: float
    dt: float
    tau: float
    period: int           # steps per period of the pressure gradient
    k: float              # wall stiffness, lattice units
    G: float              # gradient amplitude, lattice units
    alpha: float          # Womersley number

    @property
    def nu(self):
        return (self.tau - 0.5) / 3.0


def case(R: int, kp: float = 50.0, tau: Optional[float] = None) -> Case:
    """Lattice parameters of the R dx cylinder for a gradient amplitude of
    kp Pa/m.  With `tau` given, the same dimensionless problem at another
    relaxation time: the time step changes so that the Womersley number, the
    lattice velocities (hence Reynolds and Mach numbers) and the lattice
    stiffness relative to the driving pressure stay the same."""
    dx, dt = RESOLUTIONS[R]
    nu = MU / RHO
    tau0 = 0.5 + 3.0 * nu * dt / (dx * dx)
    if tau is not None:
        dt = dt * (tau - 0.5) / (tau0 - 0.5) * 1.0
    else:
        tau = tau0
    k_phys = YOUNG * H_OVER_R * R_M / ((1.0 - POISSON ** 2) * R_M * R_M)
    omega = 2 * math.pi / PERIOD_S
    # with nu_lattice scaled by s = (tau - 1/2)/(tau0 - 1/2) the period in
    # steps scales by 1/s; the gradient (and the stiffness, a pressure per
    # length) scale by s so that velocities G R^2 / nu_lattice are unchanged
    s = (tau - 0.5) / (tau0 - 0.5)
    dt0 = RESOLUTIONS[R][1]
    return Case(R=R, L=int(round(LENGTH_M / dx)), dx=dx, dt=dt, tau=tau,
                period=int(round(PERIOD_S / dt0 / s)), k=k_phys * dt0 * dt0 / (RHO * dx) * s,
                G=abs(kp) * dt0 * dt0 / (RHO * dx) * s, alpha=R_M * math.sqrt(omega * RHO / MU))


def womersley_profile(r, R, omega, nu, G_hat):
    """Complex amplitude of the axial velocity of oscillating flow in a rigid
    pipe of radius R driven by -dp/dz = Re[G_hat e^{i omega t}] (density 1):
    G_hat/(i omega) (1 - J0(k r)/J0(k R)), k^2 = -i omega/nu."""
    from scipy.special import jv
    k = np.sqrt(-1j * omega / nu)
    return G_hat / (1j * omega) * (1.0 - jv(0, k * np.asarray(r, float)) / jv(0, k * R))


def _lattice(c: Case, mode: int, dtype: str, amp: float):
    g = inputs.cylinder(c.R, c.L, with_normals=False)
    lat = lbm.Lattice([g], dtype=dtype, tau=c.tau)
    lat.set_wall(0, mode, F=F_WALL if mode == lbm.ELASTIC else 0.0, P0=1.0 / 3.0, k=[c.k])
    # density iolets 1 +- amp sin(omega t) on the planes z = 0 and z = L + 1,
    # with their inward normals
    lat.set_iolet(0, 0, lbm.DENSITY, 1.0, amp, float(c.period), 0.0, (0.0, 0.0, 1.0))
    lat.set_iolet(0, 1, lbm.DENSITY, 1.0, amp, float(c.period), math.pi, (0.0, 0.0, -1.0))
    lat.init_fields(0)
    return g, lat


def womersley(R: int = 50, mode: int = lbm.BOUNCEBACK, kp: float = 50.0, settle: int = 3,
              dtype: str = "f32", samples: int = 40, tau: Optional[float] = None, log=None) -> Dict:
    """Runs `settle` periods, then samples one more period (`samples` evenly
    spaced times) and compares the centre-plane axial velocity at 5 phases
    with the rigid Womersley solution for the measured centre-plane gradient.
    Errors per phase: max over the plane of |u - u_a| / max |u_a| at that
    phase, and the same normalised by the amplitude of the centre velocity."""
    c = case(R, kp, tau)
    amp = 1.5 * c.G * (c.L + 1)          # density amplitude: gradient c.G over L + 1
    g, lat = _lattice(c, mode, dtype, amp)
    lat.autotune(32)
    n = lat.n_sites(0)
    t0 = time.perf_counter()
    lat.step(settle * c.period)
    lat.sync()
    t_settle = time.perf_counter() - t0
    if log:
        log(f"R={R} {'elastic' if mode == lbm.ELASTIC else 'rigid'}: {settle} periods "
            f"({settle * c.period} steps, {n} sites) in {t_settle:.1f} s")
    zz, yy, xx = np.nonzero(g.labels == inputs.FLUID)     # canonical (raster) order
    xyz = np.stack([xx, yy, zz], 1)
    zc = (c.L + 1) // 2
    mid, up, dn = (xyz[:, 2] == zc), (xyz[:, 2] == zc + 1), (xyz[:, 2] == zc - 1)
    ctr = g.info["centre"]
    r = np.hypot(xyz[mid, 0] - ctr, xyz[mid, 1] - ctr)
    R_eff = math.sqrt(mid.sum() / math.pi)
    axis = np.hypot(xyz[:, 0] - ctr, xyz[:, 1] - ctr) < 0.75
    z_axis = xyz[axis, 2]
    central = np.abs(z_axis - zc) <= c.L // 4
    omega = 2 * math.pi / c.period
    stride = c.period // samples
    G_t, u_t, ts, cl = [], [], [], []
    start = lat.info()["step"]
    for s in range(samples):
        rho, u, _, _ = lat.read_fields(0, wss=False, wall_dr=False)
        t = lat.info()["step"] - start
        G_t.append(-(rho[up].mean() - rho[dn].mean()) / 6.0)
        u_t.append(u[mid, 2].copy())
        cl.append(u[axis, 2].copy())
        ts.append(t)
        lat.step(stride)
    lat.close()
    ts = np.asarray(ts, float)
    e = np.exp(-1j * omega * ts)
    G_hat = 2.0 * np.mean(np.asarray(G_t) * e)
    u_hat_a = womersley_profile(r, R_eff, omega, c.nu, G_hat)
    centre_amp = abs(womersley_profile([0.0], R_eff, omega, c.nu, G_hat)[0])
    phases = []
    for k in range(5):
        j = k * samples // 5
        ua = np.real(u_hat_a * np.exp(1j * omega * ts[j]))
        err = np.abs(u_t[j] - ua)
        phases.append(dict(phase=round(ts[j] / c.period, 3),
                           u_centre_sim=float(u_t[j][np.argmin(r)]), u_centre_ana=float(ua[np.argmin(r)]),
                           err_rel_phase=float(err.max() / max(np.abs(ua).max(), 1e-30)),
                           err_rel_amplitude=float(err.max() / centre_amp),
                           err_rms_amplitude=float(np.sqrt((err ** 2).mean()) / centre_amp)))
    # shape fits (the paper's elastic comparison): the first harmonic of the
    # simulated centre-plane profile against 1 - M J0(Lambda r/R)/J0(Lambda)
    # with one fitted complex amplitude; M from the Sec. 2.3 relation at the
    # paper's F for this cylinder (reading: extended wall R = r + 1/2), and
    # the rigid shape (M = 1, wall at the equal-area radius) for contrast
    u_arr = np.asarray(u_t)
    u_hat_sim = 2.0 * (u_arr * e[:, None]).mean(axis=0)
    fits = {}
    M_el = slip.calibrate_M(F_WALL, c.alpha, slip.dr_over_R(c.R))
    for name, M, Rw in (("elastic_model", M_el, c.R + 0.5), ("rigid_model", 1.0, R_eff)):
        al = Rw * math.sqrt(omega / c.nu)
        phi = slip.womersley_shape(M, al, r / Rw)
        A = complex(np.vdot(phi, u_hat_sim) / np.vdot(phi, phi))
        amp_f = float(np.abs(A * phi).max())
        per = []
        for k in range(5):
            j = k * samples // 5
            err = np.abs(u_t[j] - np.real(A * phi * np.exp(1j * omega * ts[j])))
            per.append(float(err.max() / amp_f))
        res = np.abs(u_hat_sim - A * phi)
        fits[name] = dict(M=float(M), R_wall=float(Rw), alpha=float(al),
                          err_max_rel_amplitude=max(per), phase_err_rel_amplitude=per,
                          harmonic_rms_rel=float(np.sqrt((res ** 2).mean()) / amp_f))
    # centreline: axis sites of the central half of the tube against the
    # analytic centre value, same phases; and the axial profile of the
    # deviation in eight bins over the whole length (entrance effects)
    cl_err, cl_bins = [], []
    edges = np.linspace(1, c.L + 1, 9)
    for k in range(5):
        j = k * samples // 5
        ua0 = np.real(womersley_profile([0.0], R_eff, omega, c.nu, G_hat)[0] * np.exp(1j * omega * ts[j]))
        dev = np.abs(cl[j] - ua0) / centre_amp
        cl_err.append(float(dev[central].max()))
        cl_bins.append([float(dev[(z_axis >= edges[b]) & (z_axis < edges[b + 1])].max()) for b in range(8)])
    return dict(R=R, L=c.L, sites=int(n), tau=c.tau, period=c.period, alpha=c.alpha, k_lattice=c.k,
                G_lattice=c.G, G_measured=abs(G_hat), R_eff=R_eff,
                mode="elastic" if mode == lbm.ELASTIC else "rigid", dtype=dtype, settle_periods=settle,
                seconds_settle=t_settle, glups=n * settle * c.period / t_settle / 1e9,
                phases=phases, shape_fits=fits, centreline_central_half_err_rel_amplitude=cl_err,
                centreline_err_by_length_eighth=cl_bins)


def timing(radii=(50, 100, 200), dtype: str = "f32", steps: int = 1000, log=None) -> List[Dict]:
    """Seconds per `steps` iterations, elastic and rigid, per radius (graph
    replay, HIP events on the library stream, after autotuning and 100
    warm-up steps), beside the paper's Table 1."""
    out = []
    for R in radii:
        c = case(R)
        t0 = time.perf_counter()
        g, lat = _lattice(c, lbm.ELASTIC, dtype, 1e-4)
        t_build = time.perf_counter() - t0
        n = lat.n_sites(0)
        del g
        row = dict(R=R, L=c.L, sites=int(n), dtype=dtype, seconds_build=t_build)
        if log:
            log(f"R={R}: {n} sites built in {t_build:.1f} s")
        for name, mode in (("elastic", lbm.ELASTIC), ("rigid", lbm.BOUNCEBACK)):
            lat.set_wall(0, mode, F=F_WALL if mode == lbm.ELASTIC else 0.0, P0=1.0 / 3.0, k=[c.k])
            lat.init_fields(0)
            lat.autotune(16)
            lat.step(100)
            ms = lat.time_steps(steps)
            row[name + "_s"] = ms / 1e3 * 1000.0 / steps
            row[name + "_glups"] = n * steps / (ms * 1e-3) / 1e9
            if log:
                log(f"R={R} {name}: {row[name + '_s']:.4f} s per 1000 iterations")
        row["paper_elastic_s"], row["paper_rigid_s"] = PAPER_TABLE1[R]
        lat.close()
        if log:
            log(f"R={R}: {n} sites, elastic {row['elastic_s']:.4f} s, rigid {row['rigid_s']:.4f} s "
                f"per 1000 iterations (paper: {PAPER_TABLE1[R][0]} s, {PAPER_TABLE1[R][1]} s)")
        out.append(row)
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="the paper's verification cylinder on one GPU")
    ap.add_argument("--womersley", type=int, nargs="*", default=[], help="radii to run")
    ap.add_argument("--modes", nargs="+", default=["rigid", "elastic"])
    ap.add_argument("--kp", type=float, default=50.0)
    ap.add_argument("--settle", type=int, default=3)
    ap.add_argument("--tau", type=float, default=None,
                    help="run the Womersley case at this relaxation time (same dimensionless problem)")
    ap.add_argument("--timing", type=int, nargs="*", default=[], help="radii to time")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    res = dict(womersley=[], timing=[])
    for R in a.womersley:
        for m in a.modes:
            r = womersley(R, lbm.ELASTIC if m == "elastic" else lbm.BOUNCEBACK, a.kp, a.settle,
                          a.dtype, tau=a.tau, log=log)
            log(json.dumps(r))
            res["womersley"].append(r)
    if a.timing:
        res["timing"] = timing(a.timing, a.dtype, log=log)
        log(json.dumps(res["timing"]))
    if a.out:
        with open(a.out, "w") as f:
            f.write(json.dumps(res) + "\n")


if __name__ == "__main__":
    main()
