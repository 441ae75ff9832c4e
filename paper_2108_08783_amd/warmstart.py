"""Learned warm start of the periodic state.

A per-site network predicts density and velocity of the periodic
(cycle-to-cycle converged) flow from local geometry and drive features; the
prediction initialises the populations at equilibrium (Sec. 2.1 eq. feq),
after which the ordinary update runs unchanged.  The zero-velocity start is
the fallback and the reference: both starts must converge to the same periodic
state, and the figure of merit is the number of cardiac cycles needed.

Features (16 per site, host-side, from the generator's segment list), in
one of three sets that differ in slots 1, 2, 4-10:
  0  (r(t) - |x - q|) / r(t): wall distance relative to the local radius
  1  absolute: r(t) / 24, the local radius;
     scale_free: r(t) / r_ref, the radius relative to the parent segment's
     end radius (the segment's own start radius for the root), about 0.79
     at every Murray branching
  2  absolute: r(t) / r_inlet;
     scale_free: the generation of the owning segment (0 for the root)
  3  t: position along the owning segment (0 at its start)
  4  path position: distance from the inlet along the tree over the
     (mean) inlet-to-outlet path length through the segment
  5  the prior's density output (below)
  6  downstream path length over r_inlet, scaled by 1/40
  7-9 absolute: generation one-hot (0, 1, deeper); the deeper slot starts
     at zero weight, so generations absent from the training data
     contribute nothing; scale_free: zero
  10 the prior's axial velocity over u0
  11 the prior's slip factor at the local mean pressure
  12 log10(k) + 2: wall stiffness of the segment
  13 u0 / 0.02: inlet amplitude
  14, 15 sin and cos of 2 pi (phase of the predicted state in the cycle)
The local set keeps every input local and dimensionless: slot 1 as in the
scale-free set, 2 the local Womersley number r sqrt(omega / nu) / 3, 4 and
6 the distances to the segment's start and end in local radii (/ 16,
capped at 1), 5 zero, 7 and 8 whether the segment starts and ends at a
junction, 9 zero, 10 the prior's axial velocity in units of the section's
mean-flow velocity; its outputs are corrections in that velocity too.
Outputs (4): (rho - 1) / (10 u0), and the velocity / u0 in the segment's
frame (axial, radial, azimuthal), each as a correction to a physics prior
(`network_prior`): a linear one-dimensional model of the segment tree with
slip-Poiseuille mean flow and, at the drive frequency, a transmission line
per segment with the slip Womersley impedance and the lattice's
compressibility.  The correction is applied only at sites whose features
all lie inside the range seen in training (with a 5 % margin); elsewhere
the start is the prior.  The training instances (tubes and single
bifurcations, radii 6-24) hold generations 0 and 1 only.  With the absolute
set the held-out Murray trees (radii up to 40, generations to 4) fall
outside that range at every site, so the trees start from the prior; the
scale-free set puts about 70 % of their sites inside it (the generation
gate keeps generations 2 and deeper out), and the correction learned on
single bifurcations then makes the trees' starts worse than the prior.
The local set puts half of the tree sites inside the range (the root and
first-generation vessels are wider than any training tube) and does not
help the trees either.  The absolute set is the default.  Trained on
branching trees instead (`train_trees`), the same network with the
absolute set does help held-out trees; that network is TREE_NET_FILE.
"""
from __future__ import annotations

import dataclasses
import math
import os
import time
from typing import List, Optional, Sequence

import numpy as np

from . import inputs
from . import lbm
from . import workloads

N_FEAT, N_OUT = 16, 4


# ------------------------------------------------------------- features --
@dataclasses.dataclass
class SiteFrame:
    static: np.ndarray   # [n, 12] float32, features 0..11
    r: np.ndarray        # [n] local radius r(t) of the owning segment
    seg: np.ndarray      # [n] owning segment
    axis: np.ndarray     # [n, 3]
    radial: np.ndarray   # [n, 3]
    azim: np.ndarray     # [n, 3]
    kind: str = "absolute"   # the feature set the static part belongs to


def _topology(segs):
    """Parent of every segment (-1 for the root) and the children lists;
    a segment's parent is the one whose end point is its start point."""
    n = len(segs)
    parent = [-1] * n
    for j, s in enumerate(segs):
        for i, q in enumerate(segs):
            if i != j and np.allclose(q.p1, s.p0):
                parent[j] = i
                break
    children = [[j for j in range(n) if parent[j] == i] for i in range(n)]
    return parent, children


def _path_lengths(segs):
    """Per segment: distance from the inlet to its start, its length, the
    mean inlet-to-outlet path length through it and the mean remaining
    length beyond its end."""
    n = len(segs)
    parent, children = _topology(segs)
    lengths = [float(np.linalg.norm(s.p1 - s.p0)) for s in segs]
    start = [0.0] * n
    for j in range(n):            # parents precede children in the lists
        if parent[j] >= 0:
            start[j] = start[parent[j]] + lengths[parent[j]]
    rem = [0.0] * n
    for i in range(n - 1, -1, -1):
        if children[i]:
            rem[i] = float(np.mean([lengths[c] + rem[c] for c in children[i]]))
    total = [start[i] + lengths[i] + rem[i] for i in range(n)]
    return start, lengths, total, rem


FEATURE_SETS = ("absolute", "scale_free", "local")


def site_frames(geo: inputs.Geometry, feature_set: str = "absolute") -> SiteFrame:
    if feature_set not in FEATURE_SETS:
        raise ValueError(f"feature_set must be one of {FEATURE_SETS}")
    segs = geo.segments
    assert segs, "geometry needs its segment list"
    zz, yy, xx = np.nonzero(geo.labels == inputs.FLUID)
    pos = np.stack([xx, yy, zz], 1).astype(np.float64)
    n_id = max(s.sid for s in segs) + 1
    # per-segment constants, gathered per site (segments are few)
    parent, children = _topology(segs)
    RREF = np.ones(n_id)
    UPJ = np.zeros(n_id)
    DNJ = np.zeros(n_id)
    for j, sg in enumerate(segs):
        RREF[sg.sid] = segs[parent[j]].r1 if parent[j] >= 0 else sg.r0
        UPJ[sg.sid] = parent[j] >= 0
        DNJ[sg.sid] = len(children[j]) > 0
    P0 = np.zeros((n_id, 3))
    A = np.zeros((n_id, 3))
    Ls = np.ones(n_id)
    R0 = np.zeros(n_id)
    R1 = np.zeros(n_id)
    G = np.zeros(n_id, np.int64)
    FB = np.zeros((n_id, 3))
    for sg in segs:
        d = np.asarray(sg.p1, np.float64) - np.asarray(sg.p0, np.float64)
        L = float(np.linalg.norm(d))
        ax = d / L
        fb = np.cross(ax, [0, 0, 1.0] if abs(ax[2]) < 0.9 else [0, 1.0, 0])
        P0[sg.sid], A[sg.sid], Ls[sg.sid] = sg.p0, ax, L
        R0[sg.sid], R1[sg.sid], G[sg.sid] = sg.r0, sg.r1, sg.gen
        FB[sg.sid] = fb / np.linalg.norm(fb)
    sid = geo.segment[zz, yy, xx].astype(np.int64)
    del xx, yy, zz
    n = len(sid)
    a = A[sid]
    rv = pos - P0[sid]
    del pos
    s_ax = np.einsum("ij,ij->i", rv, a)
    t = np.clip(s_ax / Ls[sid], 0.0, 1.0)
    rv -= (t * Ls[sid])[:, None] * a
    dist = np.sqrt(np.einsum("ij,ij->i", rv, rv))
    r = R0[sid] + t * (R1[sid] - R0[sid])
    gen = G[sid]
    ok = dist > 1e-9
    radial = rv
    np.divide(rv, dist[:, None], out=radial, where=ok[:, None])
    bad = np.nonzero(~ok)[0]
    radial[bad] = FB[sid[bad]]
    azim = np.empty_like(a)
    azim[:, 0] = a[:, 1] * radial[:, 2] - a[:, 2] * radial[:, 1]
    azim[:, 1] = a[:, 2] * radial[:, 0] - a[:, 0] * radial[:, 2]
    azim[:, 2] = a[:, 0] * radial[:, 1] - a[:, 1] * radial[:, 0]
    ids = [sg.sid for sg in segs]
    by_id = []
    for v in _path_lengths(segs):
        w = np.zeros(n_id)
        w[ids] = v
        by_id.append(w[sid])
    start, lengths, total, rem = by_id
    path = (start + t * lengths) / total
    r_in = segs[0].r0
    static = np.zeros((n, 12), np.float32)
    static[:, 0] = np.clip((r - dist) / r, -0.5, 1.0)
    if feature_set == "scale_free":
        static[:, 1] = r / RREF[sid]
        static[:, 2] = gen
    elif feature_set == "local":
        # slot 2 (the local Womersley number) is set with the drive
        static[:, 1] = r / RREF[sid]
        static[:, 7] = UPJ[sid]
        static[:, 8] = DNJ[sid]
    else:
        static[:, 1] = r / 24.0
        static[:, 2] = r / r_in
        static[:, 7] = gen == 0
        static[:, 8] = gen == 1
        static[:, 9] = gen >= 2
    static[:, 3] = t
    if feature_set == "local":
        # distances to the segment's start and end in local radii
        static[:, 4] = np.minimum(t * lengths / r, 16.0) / 16.0
        static[:, 6] = np.minimum((1.0 - t) * lengths / r, 16.0) / 16.0
    else:
        static[:, 4] = path
        static[:, 6] = (lengths * (1.0 - t) + rem) / r_in / 40.0
    return SiteFrame(static, r, sid, a, radial, azim, feature_set)


def features(frame: SiteFrame, k_seg: Sequence[float], u0: float, phase: float,
             prior: "Prior") -> np.ndarray:
    """Network inputs (listed in the module docstring); `prior` is
    `network_prior`'s estimate for the same sites and phase."""
    n = frame.static.shape[0]
    X = np.empty((n, N_FEAT), np.float32)
    X[:, :12] = frame.static
    if frame.kind == "local":
        X[:, 2] = frame.r * prior.kappa / 3.0          # local Womersley number / 3
        X[:, 5] = 0.0
        X[:, 10] = prior.Y[:, 1] / prior.scale         # in the local flow velocity
    else:
        X[:, 5] = prior.Y[:, 0]
        X[:, 10] = prior.Y[:, 1]
    X[:, 11] = prior.slip
    X[:, 12] = np.log10(np.asarray(k_seg, np.float64)[frame.seg]) + 2.0
    X[:, 13] = u0 / 0.02
    X[:, 14] = math.sin(2 * math.pi * phase)
    X[:, 15] = math.cos(2 * math.pi * phase)
    return X


def _b2(R, s):
    """b^2 of the parabola A (b^2 - y^2) whose value at the wall node R_w =
    R + 1/2 is s times its value at R_w - 1 (the slip condition of the wall
    rule, Sec. 2.3); large for s -> 1 (plug flow)."""
    Rw = R + 0.5
    return (Rw * Rw - s * (Rw - 1.0) ** 2) / np.maximum(1.0 - s, 1e-9)


def _slip(p, k, F, P0):
    """Slip factor of the elastic rule at pressure p (Sec. 2.3 and 2.4):
    s = (F + Delta E)/(1 + Delta E), Delta E = max(0, (p - P0)/k)."""
    dE = np.maximum(0.0, (p - P0) / k)
    return (F + dE) / (1.0 + dE)


def _womersley(r, s, kw):
    """Oscillatory profile u(y) = C0 (1 + beta J0(kw y)) of a tube of radius
    r whose wall node R_w = r + 1/2 carries s times the velocity of the node
    inside it; kw^2 = -i omega / nu.  Returns (beta, m) with m the mean of
    the profile over the disk y < r divided by C0."""
    from scipy.special import jv
    Rw = r + 0.5
    beta = -(1.0 - s) / (jv(0, kw * Rw) - s * jv(0, kw * (Rw - 1.0)))
    m = 1.0 + beta * 2.0 * jv(1, kw * r) / (kw * r)
    return beta, m


@dataclasses.dataclass
class Prior:
    Y: np.ndarray        # [n, 4] estimate in output units
    slip: np.ndarray     # [n] slip factor at the mean pressure
    scale: Optional[np.ndarray] = None   # [n] mean-flow velocity of the section / u0
    kappa: float = 0.0   # sqrt(omega / nu): r kappa is the local Womersley number


def network_prior(geo: inputs.Geometry, frame: SiteFrame, k_seg, F: float, P0: float, u0: float,
                  phase: float, nu: float = 0.1, amp: float = 0.5, period: float = 4000.0,
                  n_sub: int = 16, iters: int = 4) -> Prior:
    """Linear one-dimensional model of the segment tree, evaluated at every
    site.  Inlet flow Q(t) = pi r_in^2 u0 (1 + amp sin(omega t)); pressure
    P0 at the outlets.

    Mean part: slip Poiseuille flow in each piece (n_sub pieces per
    segment), -dp/dx = 4 nu Q / (pi r^2 (b^2 - r^2/2)) with b^2 from the
    slip factor at the local mean pressure; flows split at junctions by the
    downstream resistances, iterated with the pressures.
    Oscillating part: a transmission line per piece at the drive frequency,
    series impedance i omega / (pi r^2 m) from the slip Womersley profile
    and shunt admittance i omega pi r^2 / c_s^2 from the lattice's
    compressibility (c_s^2 = 1/3); input impedances from the outlets up,
    then pressure and flow from the inlet down."""
    segs = geo.segments
    n = len(segs)
    parent, children = _topology(segs)
    omega = 2.0 * math.pi / period
    kw = np.sqrt(-1j * omega / nu)
    r_in = segs[0].r0
    L = np.array([float(np.linalg.norm(sg.p1 - sg.p0)) for sg in segs])
    k = np.asarray(k_seg, np.float64)[[sg.sid for sg in segs]]
    tm = (np.arange(n_sub) + 0.5) / n_sub                      # piece mid-points
    rp = np.array([sg.r0 + tm * (sg.r1 - sg.r0) for sg in segs])          # [n, n_sub]
    lp = (L / n_sub)[:, None]
    A = math.pi * rp * rp
    Q0 = math.pi * r_in * r_in * u0

    # ---- mean flow: pressures from the outlets up, flow split by resistance
    # (a subtree without an outlet carries no mean flow)
    opened = [False] * n
    for i in range(n - 1, -1, -1):
        opened[i] = segs[i].outlet or any(opened[c] for c in children[i])
    kids = [[c for c in children[i] if opened[c]] for i in range(n)]
    Q = np.zeros(n)
    Q[0] = Q0
    for i in range(n):                       # Murray split to start
        if kids[i]:
            w = np.array([segs[c].r0 ** 3 for c in kids[i]])
            Q[kids[i]] = Q[i] * w / w.sum()
    pst = np.zeros((n, n_sub + 1))
    slp = np.zeros((n, n_sub))
    for _ in range(iters):
        for i in range(n - 1, -1, -1):
            if not opened[i]:
                continue
            p = P0 if not kids[i] else float(np.mean([pst[c, 0] for c in kids[i]]))
            pst[i, n_sub] = p
            for m in range(n_sub - 1, -1, -1):
                sl = float(_slip(p, k[i], F, P0))
                b2 = float(_b2(rp[i, m], sl))
                G = 4.0 * nu * Q[i] / (A[i, m] * max(b2 - 0.5 * rp[i, m] ** 2, 1e-9))
                p += G * lp[i, 0]
                pst[i, m] = p
                slp[i, m] = sl
        Rseg = (pst[:, 0] - pst[:, n_sub]) / np.maximum(Q, 1e-30)
        Req = np.zeros(n)
        for i in range(n - 1, -1, -1):
            down = 1.0 / sum(1.0 / Req[c] for c in kids[i]) if kids[i] else 0.0
            Req[i] = Rseg[i] + down
        for i in range(n):
            if kids[i]:
                g = np.array([1.0 / Req[c] for c in kids[i]])
                Q[kids[i]] = Q[i] * g / g.sum()
    for i in range(n):                       # dead ends: the junction's pressure
        if not opened[i] and parent[i] >= 0:
            pst[i, :] = pst[parent[i], n_sub]
            slp[i, :] = _slip(pst[i, 0], k[i], F, P0)

    # ---- oscillating flow at the drive frequency
    beta, mfac = _womersley(rp, slp, kw)
    Z = 1j * omega / (A * mfac)              # series impedance per length
    Y = 1j * omega * A * 3.0                 # shunt admittance per length
    gam = np.sqrt(Z * Y)
    Zc = np.sqrt(Z / Y)
    th = np.tanh(gam * lp)
    Zst = np.zeros((n, n_sub + 1), complex)  # impedance looking downstream
    for i in range(n - 1, -1, -1):
        if children[i]:
            ZL = 1.0 / sum(1.0 / Zst[c, 0] for c in children[i])
        elif segs[i].outlet:
            ZL = 0.0
        else:
            ZL = np.inf
        Zst[i, n_sub] = ZL
        for m in range(n_sub - 1, -1, -1):
            if np.isinf(ZL):
                ZL = Zc[i, m] / th[i, m]
            else:
                ZL = Zc[i, m] * (ZL + Zc[i, m] * th[i, m]) / (Zc[i, m] + ZL * th[i, m])
            Zst[i, m] = ZL
    ph = np.zeros((n, n_sub + 1), complex)
    qh = np.zeros((n, n_sub + 1), complex)
    for i in range(n):
        if parent[i] < 0:
            qh[i, 0] = -1j * amp * Q0            # amp sin = Re(-i amp e^{i omega t})
            ph[i, 0] = Zst[i, 0] * qh[i, 0]
        else:
            ph[i, 0] = ph[parent[i], n_sub]
            qh[i, 0] = ph[i, 0] / Zst[i, 0]
        for m in range(n_sub):
            ch, sh = np.cosh(gam[i, m] * lp[i, 0]), np.sinh(gam[i, m] * lp[i, 0])
            ph[i, m + 1] = ph[i, m] * ch - Zc[i, m] * qh[i, m] * sh
            qh[i, m + 1] = qh[i, m] * ch - ph[i, m] / Zc[i, m] * sh

    # ---- evaluate at the sites
    st = frame.static
    seg = frame.seg
    idx = np.array([sg.sid for sg in segs])
    row = np.empty(int(idx.max()) + 1, np.int64)
    row[idx] = np.arange(n)
    g = row[seg]
    r = frame.r.astype(np.float64)
    t = st[:, 3].astype(np.float64)
    dist = np.maximum(r * (1.0 - st[:, 0]), 0.0)
    pos = t * n_sub
    s0 = np.clip(np.floor(pos).astype(np.int64), 0, n_sub - 1)
    fr = pos - s0
    p_mean = pst[g, s0] * (1 - fr) + pst[g, s0 + 1] * fr
    p_osc = ph[g, s0] * (1 - fr) + ph[g, s0 + 1] * fr
    q_osc = qh[g, s0] * (1 - fr) + qh[g, s0 + 1] * fr
    sl = _slip(p_mean, k[g], F, P0)
    b2 = _b2(r, sl)
    area = math.pi * r * r
    prof = np.clip((b2 - dist * dist) / np.maximum(b2 - 0.5 * r * r, 1e-9), 0.0, None)
    # beta and m at the piece mid-points, J0(kw y) from a fine table
    sm = np.clip(np.floor(pos - 0.5).astype(np.int64), 0, n_sub - 2) if n_sub > 1 else 0 * s0
    fm = np.clip(pos - 0.5 - sm, 0.0, 1.0) if n_sub > 1 else 0.0 * fr
    bet = beta[g, sm] * (1 - fm) + beta[g, np.minimum(sm + 1, n_sub - 1)] * fm
    mf = mfac[g, sm] * (1 - fm) + mfac[g, np.minimum(sm + 1, n_sub - 1)] * fm
    from scipy.special import jv
    h = 1.0 / 64.0
    ytab = np.arange(0.0, float(dist.max()) + 2 * h, h)
    j0 = jv(0, kw * ytab)
    yi = np.minimum((dist / h).astype(np.int64), len(ytab) - 2)
    yf = dist / h - yi
    shape = (1.0 + bet * (j0[yi] * (1 - yf) + j0[yi + 1] * yf)) / mf
    e = np.exp(1j * 2.0 * math.pi * phase)
    u_ax = Q[g] / area * prof + np.real(q_osc / area * shape * e)
    p = p_mean + np.real(p_osc * e)
    P = np.zeros((len(seg), N_OUT), np.float32)
    P[:, 0] = (3.0 * p - 1.0) / (10.0 * u0)
    P[:, 1] = u_ax / u0
    scale = np.maximum(Q[g] / area / u0, 0.05).astype(np.float32)
    return Prior(P, sl.astype(np.float32), scale, math.sqrt(omega / nu))


def targets(frame: SiteFrame, rho, u, u0) -> np.ndarray:
    T = np.empty((len(rho), N_OUT), np.float32)
    T[:, 0] = (rho - 1.0) / (10.0 * u0)
    T[:, 1] = (u * frame.axis).sum(1) / u0
    T[:, 2] = (u * frame.radial).sum(1) / u0
    T[:, 3] = (u * frame.azim).sum(1) / u0
    return T


def assemble(frame: SiteFrame, Y: np.ndarray, u0: float):
    """Network output -> (rho, u) in the global frame."""
    Y = np.asarray(Y, np.float64)
    rho = 1.0 + 10.0 * u0 * Y[:, 0]
    u = u0 * (Y[:, 1:2] * frame.axis + Y[:, 2:3] * frame.radial + Y[:, 3:4] * frame.azim)
    return rho, u


# ---------------------------------------------------- periodic runs -------
@dataclasses.dataclass
class PeriodicResult:
    cycles: List[int]           # cycles to periodicity per instance (-1: not reached)
    deltas: List[List[float]]   # per instance, max(du, dp) after each cycle
    seconds: float
    du: List[List[float]] = dataclasses.field(default_factory=list)
    dp: List[List[float]] = dataclasses.field(default_factory=list)


def run_to_periodic(lat: lbm.Lattice, n_inst: int, period: int, tol: float = 1e-3,
                    max_cycles: int = 20, on_converged=None, log=None) -> PeriodicResult:
    """Steps the context cycle by cycle.  After each cycle the monitor
    compares every instance's u and p with the previous cycle; an instance is
    periodic at the first cycle whose change is below tol.  on_converged(k)
    is called once per instance when it converges (e.g. to sample it)."""
    t0 = time.perf_counter()
    cycles = [-1] * n_inst
    deltas = [[] for _ in range(n_inst)]
    dus = [[] for _ in range(n_inst)]
    dps = [[] for _ in range(n_inst)]
    for k in range(n_inst):
        lat.cycle_delta(k)                       # snapshot at t = 0
    for c in range(1, max_cycles + 1):
        lat.step(period)
        for k in range(n_inst):
            if cycles[k] >= 0:
                continue
            du, dp = lat.cycle_delta(k)
            deltas[k].append(max(du, dp))
            dus[k].append(du)
            dps[k].append(dp)
            if max(du, dp) < tol:
                cycles[k] = c
                if on_converged:
                    on_converged(k, c)
        if log:
            done = sum(1 for x in cycles if x >= 0)
            log(f"cycle {c}: {done}/{n_inst} periodic, "
                f"median delta {np.median([d[-1] for d in deltas if d]):.2e}")
        if all(x >= 0 for x in cycles):
            break
    return PeriodicResult(cycles, deltas, time.perf_counter() - t0, dus, dps)


# ----------------------------------------------------------- training ----
def collect_batch(wl: workloads.Workload, dtype="f16", phases=8, sites_per_phase=2048,
                  tol=1e-3, max_cycles=20, seed=0, log=None, feature_set="absolute"):
    """Runs a batch of instances cold to periodicity, then samples every
    instance at `phases` phases of one further cycle.  Returns (X, T,
    PeriodicResult).  All instances share the drive period."""
    rng = np.random.default_rng(seed)
    period = int(wl.params[0].iolets[0]["period"])
    nu = (wl.tau - 0.5) / 3.0
    lat = workloads.lattice(wl, dtype)
    lat.autotune(64)
    res = run_to_periodic(lat, len(wl.geoms), period, tol, max_cycles, log=log)
    subs = []
    for k, g in enumerate(wl.geoms):
        fr = site_frames(g, feature_set)
        n = fr.static.shape[0]
        idx = np.sort(rng.choice(n, min(sites_per_phase, n), replace=False))
        subs.append((idx, SiteFrame(fr.static[idx], fr.r[idx], fr.seg[idx], fr.axis[idx],
                                    fr.radial[idx], fr.azim[idx], fr.kind)))
    Xs, Ts = [], []
    step = period // phases
    for ph in range(phases):
        # every instance was initialised at t = 0, so its drive phase is
        # (steps so far mod period) / period
        phase = (lat.info()["step"] % period) / period
        for k, p in enumerate(wl.params):
            if res.cycles[k] < 0:
                continue
            rho, u, _, _ = lat.read_fields(k, wss=False, wall_dr=False)
            idx, sub = subs[k]
            u0 = p.iolets[0]["a0"]
            pr = network_prior(wl.geoms[k], sub, p.k, p.F, p.P0, u0, phase, nu=nu,
                               amp=p.iolets[0]["amp"], period=period)
            Xs.append(features(sub, p.k, u0, phase, pr))
            Ts.append((targets(sub, rho[idx], u[idx], u0) - pr.Y) / out_scale(sub, pr)[:, None])
        lat.step(step)
    lat.close()
    return np.concatenate(Xs), np.concatenate(Ts), res


GEN_SLOTS = range(7, 10)
TRUST = 1.0


def out_scale(frame: SiteFrame, prior: Prior) -> np.ndarray:
    """Unit of the network's correction per site, in output units: 1 (u0,
    and 10 u0 for the density), or for the local feature set the prior's
    mean-flow velocity of the site's section."""
    if frame.kind == "local":
        return prior.scale.astype(np.float32)
    return np.ones(frame.static.shape[0], np.float32)


def new_net(seed=0, width=128, depth=4, feature_set="absolute"):
    """Network with the standard shape for the given feature set; the
    first-layer weights of the generation one-hot inputs (absolute set)
    start at zero, so generations absent from the training data contribute
    nothing at inference."""
    from . import mlp
    p = mlp.init_params(N_FEAT, width, depth, N_OUT, seed=seed)
    W0 = p[:N_FEAT * width].reshape(width, N_FEAT)
    if feature_set == "absolute":
        W0[:, list(GEN_SLOTS)] = 0.0
    net = mlp.Net(N_FEAT, width, depth, N_OUT, params=p)
    net.feature_set = feature_set
    return net


def feature_range(X: np.ndarray, margin: float = 0.05) -> np.ndarray:
    """[2, N_FEAT] bounds of the training features, widened by `margin` of
    each feature's span (features constant in training stay exact)."""
    lo, hi = X.min(0).astype(np.float64), X.max(0).astype(np.float64)
    pad = margin * (hi - lo)
    return np.stack([lo - pad, hi + pad])


def in_range(X: np.ndarray, rng: Optional[np.ndarray]) -> np.ndarray:
    """Per site: every feature inside the training range."""
    if rng is None:
        return np.ones(X.shape[0], bool)
    return np.all((X >= rng[0]) & (X <= rng[1]), axis=1)


def train(net, X: np.ndarray, T: np.ndarray, epochs=30, batch=8192, lr=2e-3, seed=0,
          weights=(1.0, 1.0, 1.0, 1.0), log=None):
    """Adam on the weighted MSE with a cosine learning-rate decay; records
    the training features' range on the network (`feature_range`);
    returns the per-epoch mean losses."""
    import torch
    rng = np.random.default_rng(seed)
    net.feature_range = feature_range(X)
    Xt = net.to_bf16(torch.tensor(X, dtype=torch.float32, device="cuda"))
    Tt = torch.tensor(T, dtype=torch.float32, device="cuda")
    w = torch.tensor(weights, dtype=torch.float32, device="cuda")
    n = X.shape[0]
    nb = max(1, n // batch)
    losses = []
    total = epochs * nb
    it = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device="cuda")
        acc = torch.zeros(1, device="cuda")
        for b in range(nb):
            sel = perm[b * batch:(b + 1) * batch]
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / total))
            acc += net.train_step(Xt[sel].contiguous(), Tt[sel].contiguous(), w, lr=lr_t)
            it += 1
        losses.append(acc.item() / nb)
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses


def instance_prior(geo, frame: SiteFrame, params, phase, nu=0.1) -> Prior:
    io = params.iolets[0]
    return network_prior(geo, frame, params.k, params.F, params.P0, io["a0"], phase, nu=nu,
                         amp=io["amp"], period=io["period"])


# Outside the training range: "gate" applies no correction at a site with
# any feature outside it; "clamp" moves every feature into the range first
# (the network is then used everywhere, saturating at the range boundary).
OUT_OF_RANGE = "gate"


def predict(net, geo, frame: SiteFrame, params, phase, nu=0.1, chunk=1 << 20, use_net=True,
            prior: Optional[Prior] = None, out_of_range: Optional[str] = None):
    """(rho, u) of every site of one instance: the network prior plus the
    network's correction (clipped to the trust region; sites with features
    outside the training range handled by `out_of_range`, default
    OUT_OF_RANGE)."""
    import torch
    u0 = params.iolets[0]["a0"]
    pr = prior if prior is not None else instance_prior(geo, frame, params, phase, nu)
    Y = pr.Y.copy()
    if use_net:
        X = features(frame, params.k, u0, phase, pr)
        fr = getattr(net, "feature_range", None)
        mode = out_of_range or OUT_OF_RANGE
        if mode == "clamp" and fr is not None:
            X = np.clip(X, fr[0].astype(np.float32), fr[1].astype(np.float32))
            ok = np.ones(X.shape[0], bool)
        else:
            ok = in_range(X, fr)
        unit = out_scale(frame, pr)
        for s in range(0, X.shape[0], chunk):
            xb = net.to_bf16(torch.tensor(X[s:s + chunk], device="cuda"))
            # trust region: the correction to the prior is at most one output
            # unit (u0 in velocity, 10 u0 in density), and none at sites
            # whose features lie outside the training range
            dY = np.clip(net.infer_fused(xb).cpu().numpy(), -TRUST, TRUST)
            Y[s:s + chunk] += dY * (ok[s:s + chunk] * unit[s:s + chunk])[:, None]
    return assemble(frame, Y, u0)


def compare_starts(net, wl: workloads.Workload, dtype="f32", tol=1e-3, max_cycles=20, log=None,
                   modes=("cold", "prior", "warm")):
    """Starts the same instances from rest ("cold"), from the physics prior
    alone ("prior") and from the network ("warm") on one lattice
    (re-initialised per start), runs each to periodicity and returns the
    PeriodicResult per mode plus, per instance, the largest difference of
    each periodic state from the cold one (max |du| / max |u| at the same
    phase)."""
    period = int(wl.params[0].iolets[0]["period"])
    nu = (wl.tau - 0.5) / 3.0
    out = {"state_diff": []}
    fields = {}
    lat = workloads.lattice(wl, dtype)
    lat.autotune(64)
    frames, priors = {}, {}
    if any(m != "cold" for m in modes):
        for k, (g, p) in enumerate(zip(wl.geoms, wl.params)):
            frames[k] = site_frames(g, getattr(net, "feature_set", "absolute"))
            priors[k] = instance_prior(g, frames[k], p, 0.0, nu)
    try:
        for mode in modes:
            for k, (g, p) in enumerate(zip(wl.geoms, wl.params)):
                if mode == "cold":
                    lat.init_fields(k)
                else:
                    rho, u = predict(net, g, frames[k], p, 0.0, nu=nu, use_net=(mode == "warm"),
                                     prior=priors[k])
                    lat.init_fields(k, rho, u)
            try:
                res = run_to_periodic(lat, len(wl.geoms), period, tol, max_cycles, log=log)
                # periodic states compared at the same phase (whole cycles from t=0)
                fields[mode] = [lat.read_fields(k, wss=False, wall_dr=False)[1]
                                for k in range(len(wl.geoms))]
            except lbm.Diverged as e:
                if log:
                    log(f"{mode} start diverged: {e}")
                res = PeriodicResult([-2] * len(wl.geoms), [], 0.0)
                fields[mode] = None
            out[mode] = res
    finally:
        lat.close()
    for k in range(len(wl.geoms)):
        uc = fields["cold"][k] if fields.get("cold") else None
        diffs = [float(np.abs(fields[m][k] - uc).max() / np.abs(uc).max())
                 for m in modes if m != "cold" and fields.get(m) is not None and uc is not None]
        out["state_diff"].append(max(diffs) if diffs else float("nan"))
    return out


# ------------------------------------------------------------- experiment --
MODES = ("cold", "prior", "warm")

# A network trained by `experiment()` with the default settings (256 sweep
# instances, seeds 1000-1255, 8 phases, 2048 sites per instance and phase,
# 30 epochs): python -m paper_2108_08783_amd.warmstart --test-sweep 16
# --test-trees 4 --save-net <file>, parameters stored as float32.
NET_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "warmstart_net.npz")
# the same network shape trained on 32 Murray trees (seeds 1000-1031; absolute
# features, 4.2M samples): for tree-shaped vessels, outside the protocol of
# NET_FILE's tubes and single bifurcations
TREE_NET_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                             "warmstart_net_trees.npz")


def save_net_file(path, net):
    """Parameters, training-feature range and feature set of a network
    (.npz; no object arrays)."""
    np.savez(path, params=net.state(), feature_range=net.feature_range,
             feature_set=np.array(getattr(net, "feature_set", "absolute")))


def load_net(state):
    """Network with the standard shape from `save_net_file`'s contents (a
    mapping with params and feature_range) or a bare parameter vector."""
    from . import mlp
    if hasattr(state, "keys"):
        net = mlp.Net(N_FEAT, 128, 4, N_OUT, params=np.asarray(state["params"], np.float64))
        net.feature_range = np.asarray(state["feature_range"], np.float64)
        net.feature_set = str(state["feature_set"]) if "feature_set" in state else "absolute"
        return net
    return mlp.Net(N_FEAT, 128, 4, N_OUT, params=np.asarray(state, np.float64))


def _evaluate(net, wl, dtype, max_cycles, group, log):
    cmp = compare_starts(net, wl, dtype, max_cycles=max_cycles, modes=MODES)
    for m in MODES:
        group[m] += cmp[m].cycles
        group[m + "_du"] += cmp[m].du
        group[m + "_dp"] += cmp[m].dp
    group["state_diff"] += cmp["state_diff"]
    group["sites"] += [g.n_fluid for g in wl.geoms]
    return cmp


def summarize(results):
    """Aggregate figures of the per-instance results of one or more runs."""
    out = {}
    allc = {m: [] for m in MODES}
    for name in ("sweep", "trees"):
        r = results.get(name)
        if not r or not r["cold"]:
            continue
        for m in MODES:
            allc[m] += r[m]
        ok = [i for i in range(len(r["cold"])) if all(r[m][i] > 0 for m in MODES)]
        out[name] = dict(n=len(r["cold"]), **{
            f"cycles_{m}_mean": float(np.mean([r[m][i] for i in ok])) if ok else None
            for m in MODES})
        out[name]["warm_fewer"] = sum(r["warm"][i] < r["cold"][i] for i in ok)
        out[name]["warm_more"] = sum(r["warm"][i] > r["cold"][i] for i in ok)
    ok = [i for i in range(len(allc["cold"])) if all(allc[m][i] > 0 for m in MODES)]
    out["all_converged"] = len(ok) == len(allc["cold"])
    for m in MODES:
        out[f"cycles_{m}_mean"] = float(np.mean([allc[m][i] for i in ok])) if ok else None
    out["median_ratio"] = (float(np.median([allc["warm"][i] / allc["cold"][i] for i in ok]))
                           if ok else None)
    diffs = [d for name in ("sweep", "trees") if results.get(name)
             for d in results[name]["state_diff"]]
    out["max_state_diff"] = float(max(diffs)) if diffs else None
    return out


def experiment(train_batches=4, train_per_batch=64, train_sites=20e6, test_sweep=16,
               test_sweep_sites=5e6, test_trees=16, tree_first=0, tree_scale=1.0, dtype="f32",
               epochs=30, sites_per_phase=2048, max_cycles=12, seed=0, net_params=None,
               save_net=None, checkpoint=None, log=print, feature_set="absolute",
               train_trees=0):
    """Train on cold-started sweep batches (seeds 1000.., run to
    periodicity, sampled at 8 phases), or with `train_trees` > 0 on batches
    of that many Murray trees (seeds 1000.., disjoint from the held-out
    trees' 2000..), unless `net_params` is given, then
    start held-out sweep instances (seed 3000) and Murray trees (seeds
    2000 + tree_first ..) cold, from the prior and from the network, and
    run each to periodicity.  The trained parameters are written to
    `save_net` (.npz) before the evaluation starts; `checkpoint(dict)` is
    called with the results so far after each evaluated workload.  Returns
    (JSON-ready dict, network)."""
    t_all = time.perf_counter()
    out = dict(config=dict(train_instances=train_batches * (train_trees or train_per_batch),
                           train_sites_per_batch=train_sites, test_sweep=test_sweep,
                           test_sweep_sites=test_sweep_sites, test_trees=test_trees,
                           tree_first=tree_first, tree_scale=tree_scale, dtype=dtype,
                           epochs=epochs, sites_per_phase=sites_per_phase, tol=1e-3,
                           period=int(workloads.PERIOD), feature_set=feature_set,
                           train_trees=train_trees))
    if net_params is None:
        Xs, Ts, train_cycles = [], [], []
        t0 = time.perf_counter()
        for b in range(train_batches):
            if train_trees:
                wl = workloads.trees([1000 + b * train_trees + j for j in range(train_trees)],
                                     scale=tree_scale)
            else:
                wl = workloads.sweep(seed=1000 + b, n=train_per_batch, target_sites=train_sites)
            X, T, res = collect_batch(wl, dtype, sites_per_phase=sites_per_phase,
                                      max_cycles=max_cycles, seed=b, feature_set=feature_set)
            Xs.append(X)
            Ts.append(T)
            train_cycles += res.cycles
            log(f"[warmstart] train batch {b}: {wl.n_sites} sites, cold cycles "
                f"median {np.median(res.cycles):.0f}, {res.seconds:.1f}s")
        X, T = np.concatenate(Xs), np.concatenate(Ts)
        t_data = time.perf_counter() - t0
        net = new_net(seed=seed, feature_set=feature_set)
        t0 = time.perf_counter()
        losses = train(net, X, T, epochs=epochs, log=lambda m: log("[warmstart] " + m)
                       if m.startswith("epoch") and (int(m.split()[1][:-1]) % 5 == 0) else None)
        out["train"] = dict(samples=int(X.shape[0]), cold_cycles_median=float(np.median(train_cycles)),
                            loss_first=losses[0], loss_last=losses[-1],
                            prior_mse=float((T.astype(np.float64) ** 2).mean()),
                            seconds_data=t_data, seconds_train=time.perf_counter() - t0)
        out["loss_first"], out["loss_last"] = losses[0], losses[-1]
        if save_net:
            save_net_file(save_net, net)
        log(f"[warmstart] data {t_data:.0f}s, training {out['train']['seconds_train']:.0f}s")
    else:
        net = load_net(net_params)
        out["config"]["feature_set"] = net.feature_set
    results = {}
    blank = lambda: dict(state_diff=[], sites=[], **{k: [] for m in MODES
                                                      for k in (m, m + "_du", m + "_dp")})
    if test_sweep:
        results["sweep"] = blank()
        sw = workloads.sweep(seed=3000, n=test_sweep, target_sites=test_sweep_sites)
        cmp = _evaluate(net, sw, dtype, max_cycles, results["sweep"], log)
        log("[warmstart] sweep: " + " ".join(f"{m} {cmp[m].cycles}" for m in MODES))
        if checkpoint:
            checkpoint(dict(out, results=results, **summarize(results)))
    if test_trees:
        results["trees"] = blank()
        for i in range(tree_first, tree_first + test_trees):
            t0 = time.perf_counter()
            wl = workloads.tree(seed=2000 + i, scale=tree_scale)
            cmp = _evaluate(net, wl, dtype, max_cycles, results["trees"], log)
            log(f"[warmstart] tree {i}: {wl.n_sites} sites " +
                " ".join(f"{m} {cmp[m].cycles}" for m in MODES) +
                f" diff {cmp['state_diff'][0]:.1e}, {time.perf_counter() - t0:.0f}s")
            if checkpoint:
                checkpoint(dict(out, results=results, **summarize(results)))
    out["results"] = results
    out.update(summarize(results))
    out["seconds_total"] = time.perf_counter() - t_all
    return out, net


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="learned warm start: train and compare")
    ap.add_argument("--train-batches", type=int, default=4)
    ap.add_argument("--train-per-batch", type=int, default=64)
    ap.add_argument("--train-sites", type=float, default=20e6)
    ap.add_argument("--test-sweep", type=int, default=16)
    ap.add_argument("--test-sweep-sites", type=float, default=5e6)
    ap.add_argument("--test-trees", type=int, default=16)
    ap.add_argument("--tree-first", type=int, default=0)
    ap.add_argument("--tree-scale", type=float, default=1.0)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--train-trees", type=int, default=0,
                    help="train on batches of this many Murray trees (seeds 1000..) "
                         "instead of sweep batches")
    ap.add_argument("--sites-per-phase", type=int, default=2048,
                    help="training sites sampled per instance and phase")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--save-net", default=None,
                    help="write the trained parameters and feature range (.npz)")
    ap.add_argument("--load-net", default=None, help="skip training, use these parameters")
    ap.add_argument("--out", default=None, help="write the full result (JSON)")
    ap.add_argument("--merge", nargs="+", default=None,
                    help="only combine the per-instance results of earlier --out files")
    ap.add_argument("--features", choices=FEATURE_SETS, default="absolute",
                    help="feature set of a network trained here (a loaded one keeps its own)")
    ap.add_argument("--out-of-range", choices=("gate", "clamp"), default="gate",
                    help="sites with features outside the training range: no correction "
                         "(gate) or features clamped into the range (clamp)")
    a = ap.parse_args(argv)
    global OUT_OF_RANGE
    OUT_OF_RANGE = a.out_of_range
    if a.merge:
        runs = [json.load(open(f)) for f in a.merge]
        results = {}
        for r in runs:
            for name, g in r["results"].items():
                tgt = results.setdefault(name, {k: [] for k in g})
                for k, v in g.items():
                    tgt[k] += v
        r = dict(runs=a.merge, train=next((x["train"] for x in runs if "train" in x), None),
                 results=results, **summarize(results))
    else:
        p = dict(np.load(a.load_net)) if a.load_net else None
        def save(d):
            if a.out:
                with open(a.out, "w") as f:
                    f.write(json.dumps(d) + "\n")
        r, net = experiment(a.train_batches, a.train_per_batch, a.train_sites, a.test_sweep,
                            a.test_sweep_sites, a.test_trees, a.tree_first, a.tree_scale,
                            a.dtype, a.epochs, sites_per_phase=a.sites_per_phase,
                            net_params=p, save_net=a.save_net,
                            checkpoint=save, log=lambda m: print(m, flush=True),
                            feature_set=a.features, train_trees=a.train_trees)
    if a.out:
        with open(a.out, "w") as f:
            f.write(json.dumps(r) + "\n")
    print(json.dumps({k: v for k, v in r.items() if k != "results"}), flush=True)


if __name__ == "__main__":
    main()
