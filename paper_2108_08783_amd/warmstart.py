"""Learned warm start of the periodic state.

A per-site network predicts density and velocity of the periodic
(cycle-to-cycle converged) flow from local geometry and drive features; the
prediction initialises the populations at equilibrium (Sec. 2.1 eq. feq),
after which the ordinary update runs unchanged.  The zero-velocity start is
the fallback and the judge: both starts must converge to the same periodic
state, and the figure of merit is the number of cardiac cycles needed.

Features (16 per site, host-side, from the generator's segment list):
  0  (r(t) - |x - q|) / r(t): wall distance relative to the local radius
  1  r(t) / 24: local radius
  2  r(t) / r_inlet: radius relative to the inlet (under Murray's law the
     mean velocity of a branch scales with it)
  3  t: position along the owning segment (0 at its start)
  4  path position: distance from the inlet along the tree over the
     (mean) inlet-to-outlet path length through the segment
  5  downstream Poiseuille pressure estimate over u0: the sum of
     8 nu L / (r_inlet r) over the rest of the segment and the mean path to
     the outlets (Murray flow split), scaled by 1/2
  6  downstream path length over r_inlet, scaled by 1/40
  7-11 generation one-hot (0..4, deeper generations share slot 4)
  12 log10(k) + 2: wall stiffness of the segment
  13 u0 / 0.02: inlet amplitude
  14, 15 sin and cos of 2 pi (phase of the predicted state in the cycle)
Outputs (4): (rho - 1) / (10 u0), and the velocity / u0 in the segment's
frame (axial, radial, azimuthal), each as a correction to a physics prior:
the quasi-steady Poiseuille state of the tree with Murray flow split,
  u_axial = 2 u_mean (1 - (|x - q| / r)^2), u_mean = u_in(phase) r / r_inlet,
  p - p_out = u_in(phase) * (downstream Poiseuille pressure estimate),
so that sites unlike the training data fall back toward the prior.
"""
from __future__ import annotations

import dataclasses
import math
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
    static: np.ndarray   # [n, 12] features 0..11
    seg: np.ndarray      # [n] owning segment
    axis: np.ndarray     # [n, 3]
    radial: np.ndarray   # [n, 3]
    azim: np.ndarray     # [n, 3]


def _path_lengths(segs, nu):
    """Per segment: distance from the inlet to its start, its length, the
    mean inlet-to-outlet path length through it, and the downstream
    Poiseuille pressure (per unit inlet velocity) and length from its end."""
    n = len(segs)
    parent = [-1] * n
    for j, s in enumerate(segs):
        for i, q in enumerate(segs):
            if i != j and np.allclose(q.p1, s.p0):
                parent[j] = i
                break
    lengths = [float(np.linalg.norm(s.p1 - s.p0)) for s in segs]
    r_in = segs[0].r0
    res = [8.0 * nu * lengths[i] / (r_in * 0.5 * (segs[i].r0 + segs[i].r1)) for i in range(n)]
    start = [0.0] * n
    for j in range(n):            # parents precede children in the lists
        if parent[j] >= 0:
            start[j] = start[parent[j]] + lengths[parent[j]]
    children = [[j for j in range(n) if parent[j] == i] for i in range(n)]
    rem = [0.0] * n
    pend = [0.0] * n
    for i in range(n - 1, -1, -1):
        if children[i]:
            rem[i] = float(np.mean([lengths[c] + rem[c] for c in children[i]]))
            pend[i] = float(np.mean([res[c] + pend[c] for c in children[i]]))
    total = [start[i] + lengths[i] + rem[i] for i in range(n)]
    return start, lengths, total, res, pend, rem


def site_frames(geo: inputs.Geometry, nu: float = 0.1) -> SiteFrame:
    segs = geo.segments
    assert segs, "geometry needs its segment list"
    zz, yy, xx = np.nonzero(geo.labels == inputs.FLUID)
    pos = np.stack([xx, yy, zz], 1).astype(np.float64)
    sid = geo.segment[zz, yy, xx].astype(np.int64)
    n = len(sid)
    p0 = np.array([s.p0 for s in segs])[sid]
    p1 = np.array([s.p1 for s in segs])[sid]
    r0 = np.array([s.r0 for s in segs])[sid]
    r1 = np.array([s.r1 for s in segs])[sid]
    gen = np.array([s.gen for s in segs])[sid]
    d = p1 - p0
    L = np.linalg.norm(d, axis=1)
    a = d / L[:, None]
    t = np.clip(((pos - p0) * a).sum(1) / L, 0.0, 1.0)
    q = p0 + t[:, None] * d
    rv = pos - q
    dist = np.linalg.norm(rv, axis=1)
    r = r0 + t * (r1 - r0)
    fallback = np.cross(a, np.where(np.abs(a[:, 2:3]) < 0.9, [[0, 0, 1.0]], [[0, 1.0, 0]]))
    fallback /= np.linalg.norm(fallback, axis=1, keepdims=True)
    radial = np.where(dist[:, None] > 1e-9, rv / np.maximum(dist, 1e-12)[:, None], fallback)
    azim = np.cross(a, radial)
    start, lengths, total, res, pend, rem = (np.array(v)[sid] for v in _path_lengths(segs, nu))
    path = (start + t * lengths) / total
    r_in = segs[0].r0
    static = np.zeros((n, 12))
    static[:, 0] = np.clip((r - dist) / r, -0.5, 1.0)
    static[:, 1] = r / 24.0
    static[:, 2] = r / r_in
    static[:, 3] = t
    static[:, 4] = path
    static[:, 5] = 0.5 * (res * (1.0 - t) + pend)
    static[:, 6] = (lengths * (1.0 - t) + rem) / r_in / 40.0
    static[np.arange(n), 7 + np.minimum(gen, 4)] = 1.0
    return SiteFrame(static, sid, a, radial, azim)


def features(frame: SiteFrame, k_seg: Sequence[float], u0: float, phase: float) -> np.ndarray:
    n = frame.static.shape[0]
    X = np.empty((n, N_FEAT), np.float32)
    X[:, :12] = frame.static
    X[:, 12] = np.log10(np.asarray(k_seg, np.float64)[frame.seg]) + 2.0
    X[:, 13] = u0 / 0.02
    X[:, 14] = math.sin(2 * math.pi * phase)
    X[:, 15] = math.cos(2 * math.pi * phase)
    return X


def prior(frame: SiteFrame, phase: float, amp: float = 0.5) -> np.ndarray:
    """Quasi-steady Poiseuille/Murray estimate in output units."""
    st = frame.static
    drive = 1.0 + amp * math.sin(2 * math.pi * phase)
    s = np.clip(1.0 - st[:, 0], 0.0, 1.0)            # |x - q| / r
    P = np.zeros((st.shape[0], N_OUT), np.float32)
    P[:, 0] = 3.0 * (2.0 * st[:, 5]) * drive / 10.0   # 3 dp / (10 u0), dp/u0 = 2 f5
    P[:, 1] = 2.0 * drive * st[:, 2] * (1.0 - s * s)
    return P


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
                  tol=1e-3, max_cycles=20, seed=0, log=None):
    """Runs a batch of instances cold to periodicity, then samples every
    instance at `phases` phases of one further cycle.  Returns (X, T,
    PeriodicResult).  All instances share the drive period."""
    rng = np.random.default_rng(seed)
    period = int(wl.params[0].iolets[0]["period"])
    lat = workloads.lattice(wl, dtype)
    lat.autotune(64)
    res = run_to_periodic(lat, len(wl.geoms), period, tol, max_cycles, log=log)
    subs = []
    for k, g in enumerate(wl.geoms):
        fr = site_frames(g)
        n = fr.static.shape[0]
        idx = np.sort(rng.choice(n, min(sites_per_phase, n), replace=False))
        subs.append((idx, SiteFrame(fr.static[idx], fr.seg[idx], fr.axis[idx], fr.radial[idx],
                                    fr.azim[idx])))
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
            Xs.append(features(sub, p.k, u0, phase))
            Ts.append(targets(sub, rho[idx], u[idx], u0) - prior(sub, phase))
        lat.step(step)
    lat.close()
    return np.concatenate(Xs), np.concatenate(Ts), res


GEN_SLOTS = range(7, 12)
TRUST = 1.0


def new_net(seed=0, width=128, depth=4):
    """Network with the standard shape; the first-layer weights of the
    generation one-hot inputs start at zero, so generations absent from
    the training data contribute nothing at inference."""
    from . import mlp
    p = mlp.init_params(N_FEAT, width, depth, N_OUT, seed=seed)
    W0 = p[:N_FEAT * width].reshape(width, N_FEAT)
    W0[:, list(GEN_SLOTS)] = 0.0
    return mlp.Net(N_FEAT, width, depth, N_OUT, params=p)


def train(net, X: np.ndarray, T: np.ndarray, epochs=30, batch=8192, lr=2e-3, seed=0,
          weights=(1.0, 1.0, 1.0, 1.0), log=None):
    """Adam on the weighted MSE with a cosine learning-rate decay; returns
    the per-epoch mean losses."""
    import torch
    rng = np.random.default_rng(seed)
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


def predict(net, frame: SiteFrame, k_seg, u0, phase, chunk=1 << 20):
    """Network prediction (rho, u) of every site of one instance."""
    import torch
    X = features(frame, k_seg, u0, phase)
    Y = prior(frame, phase)
    for s in range(0, X.shape[0], chunk):
        xb = net.to_bf16(torch.tensor(X[s:s + chunk], device="cuda"))
        # trust region: the correction to the prior is at most one output
        # unit (u0 in velocity, 10 u0 in density)
        Y[s:s + chunk] += np.clip(net.forward(xb).cpu().numpy(), -TRUST, TRUST)
    return assemble(frame, Y, u0)


def compare_starts(net, wl: workloads.Workload, dtype="f32", tol=1e-3, max_cycles=20, log=None,
                   modes=("cold", "prior", "warm")):
    """Starts the same instances from rest ("cold"), from the physics prior
    alone ("prior") and from the network ("warm"), runs each to periodicity
    and returns the PeriodicResult per mode plus, per instance, the largest
    difference of each periodic state from the cold one (max |du| / max |u|
    at the same phase)."""
    period = int(wl.params[0].iolets[0]["period"])
    out = {"state_diff": []}
    fields = {}
    for mode in modes:
        lat = workloads.lattice(wl, dtype)
        lat.autotune(64)
        if mode != "cold":
            for k, (g, p) in enumerate(zip(wl.geoms, wl.params)):
                fr = site_frames(g)
                u0 = p.iolets[0]["a0"]
                if mode == "warm":
                    rho, u = predict(net, fr, p.k, u0, 0.0)
                else:
                    rho, u = assemble(fr, prior(fr, 0.0), u0)
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
        lat.close()
    for k in range(len(wl.geoms)):
        uc = fields["cold"][k] if fields.get("cold") else None
        diffs = [float(np.abs(fields[m][k] - uc).max() / np.abs(uc).max())
                 for m in modes if m != "cold" and fields.get(m) is not None and uc is not None]
        out["state_diff"].append(max(diffs) if diffs else float("nan"))
    return out


# ------------------------------------------------------------- experiment --
def experiment(train_batches=4, train_per_batch=64, train_sites=20e6, test_sweep=16,
               test_sweep_sites=5e6, test_trees=16, tree_scale=1.0, dtype="f32", epochs=30,
               sites_per_phase=2048, max_cycles=12, seed=0, log=print):
    """Train on cold-started sweep batches (seeds 1000.., run to
    periodicity, sampled at 8 phases), then compare cold and warm starts on
    held-out sweep instances (seed 3000) and Murray trees (seeds 2000..).
    Returns a JSON-ready dict."""
    t_all = time.perf_counter()
    Xs, Ts, train_cycles = [], [], []
    t0 = time.perf_counter()
    for b in range(train_batches):
        wl = workloads.sweep(seed=1000 + b, n=train_per_batch, target_sites=train_sites)
        X, T, res = collect_batch(wl, dtype, sites_per_phase=sites_per_phase,
                                  max_cycles=max_cycles, seed=b)
        Xs.append(X)
        Ts.append(T)
        train_cycles += res.cycles
        log(f"[warmstart] train batch {b}: {wl.n_sites} sites, cold cycles "
            f"median {np.median(res.cycles):.0f}, {res.seconds:.1f}s")
    X, T = np.concatenate(Xs), np.concatenate(Ts)
    t_data = time.perf_counter() - t0
    net = new_net(seed=seed)
    t0 = time.perf_counter()
    losses = train(net, X, T, epochs=epochs, log=lambda m: log("[warmstart] " + m)
                   if m.startswith("epoch") and (int(m.split()[1][:-1]) % 5 == 0) else None)
    t_train = time.perf_counter() - t0
    # held-out evaluation
    results = {}
    sw = workloads.sweep(seed=3000, n=test_sweep, target_sites=test_sweep_sites)
    cmp = compare_starts(net, sw, dtype, max_cycles=max_cycles)
    modes = ("cold", "prior", "warm")
    results["sweep"] = dict(state_diff=cmp["state_diff"])
    for m in modes:
        results["sweep"][m] = cmp[m].cycles
        results["sweep"][m + "_du"] = cmp[m].du
        results["sweep"][m + "_dp"] = cmp[m].dp
    log(f"[warmstart] sweep: cold {cmp['cold'].cycles} prior {cmp['prior'].cycles} "
        f"warm {cmp['warm'].cycles}")
    trees = dict(state_diff=[], sites=[])
    for m in modes:
        trees[m] = []
        trees[m + "_du"] = []
        trees[m + "_dp"] = []
    for i in range(test_trees):
        wl = workloads.tree(seed=2000 + i, scale=tree_scale)
        cmp = compare_starts(net, wl, dtype, max_cycles=max_cycles, log=log)
        for m in modes:
            trees[m] += cmp[m].cycles
            trees[m + "_du"] += cmp[m].du
            trees[m + "_dp"] += cmp[m].dp
        trees["state_diff"] += cmp["state_diff"]
        trees["sites"].append(wl.n_sites)
        log(f"[warmstart] tree {i}: {wl.n_sites} sites cold {cmp['cold'].cycles} "
            f"prior {cmp['prior'].cycles} warm {cmp['warm'].cycles} "
            f"diff {cmp['state_diff'][0]:.1e}")
    results["trees"] = trees
    cold = results["sweep"]["cold"] + trees["cold"]
    warm = results["sweep"]["warm"] + trees["warm"]
    pri = results["sweep"]["prior"] + trees["prior"]
    ok = [(c, w) for c, w in zip(cold, warm) if c > 0 and w > 0]
    return dict(
        cycles_prior_mean=float(np.mean([x for x in pri if x > 0])) if pri else None,
        cycles=dict(sweep={m: results["sweep"][m] for m in modes},
                    trees={m: trees[m] for m in modes}),
        config=dict(train_instances=train_batches * train_per_batch, train_sites_per_batch=train_sites,
                    test_sweep=test_sweep, test_trees=test_trees, tree_scale=tree_scale, dtype=dtype,
                    epochs=epochs, samples=int(X.shape[0]), tol=1e-3, period=int(workloads.PERIOD)),
        train_cold_cycles_median=float(np.median(train_cycles)),
        loss_first=losses[0], loss_last=losses[-1],
        cycles_cold_mean=float(np.mean([c for c, _ in ok])) if ok else None,
        cycles_warm_mean=float(np.mean([w for _, w in ok])) if ok else None,
        median_ratio=float(np.median([w / c for c, w in ok])) if ok else None,
        all_converged=len(ok) == len(cold),
        max_state_diff=float(max(results["sweep"]["state_diff"] + trees["state_diff"])),
        seconds=dict(data=t_data, train=t_train, total=time.perf_counter() - t_all),
        results=results)


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
    ap.add_argument("--tree-scale", type=float, default=1.0)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    r = experiment(a.train_batches, a.train_per_batch, a.train_sites, a.test_sweep,
                   a.test_sweep_sites, a.test_trees, a.tree_scale, a.dtype, a.epochs,
                   log=lambda m: print(m, flush=True))
    s = json.dumps(r)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s + "\n")
    print(json.dumps({k: v for k, v in r.items() if k != "results"}), flush=True)


if __name__ == "__main__":
    main()
