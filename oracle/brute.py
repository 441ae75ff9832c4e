"""Brute-force single-step transcription of the method, for pinning the oracle.

TEST INFRASTRUCTURE ONLY.  Pure-Python loops over a tiny box; written
independently of ``lbm_oracle.c``:

  * the velocity set is enumerated from its definition (all integer vectors
    with components in {-1,0,1} and squared length <= 2, Sec. 2.1) and the
    weights are assigned by squared length (1/3, 1/18, 1/36);
  * the equilibrium uses the textbook coefficients 3, 9/2, 3/2 (C_s^2 = 1/3);
  * streaming is done in PUSH form, f_i(x + c_i) <- f*_i(x) (Sec. 2.1 eq.
    LBE_SRT as printed), rather than the oracle's pull form;
  * the elastic wall velocity uses the combined form U_w = s U_f with
    s = (F + Delta r - 1)/Delta r (Sec. 2.3, equal to the interpolation form
    for Delta x = 1);
  * an iolet link takes the equilibrium at the prescribed moment and the
    fluid node's other moment, at a density iolet with a given inward normal
    only the velocity along it (Sec. 3, zeroth-order reading).

Populations are addressed by velocity vector, so the caller's direction order
does not matter.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def velocity_set():
    vecs = [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2]
    w = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    return [(v, w[sum(a * a for a in v)]) for v in vecs]


def _feq(w, c, rho, u):
    cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


def step(labels, f, tau, *, mode, F, P0, k_seg, segment, iolets, iolet_weight, t):
    """One step.  ``f`` maps (x, y, z) of every fluid voxel to a dict
    {velocity tuple: value}.  ``labels`` indexed [z, y, x].  ``iolets`` maps
    id -> dict(kind, a0, amp, period, phase, direction).  Returns new f."""
    vs = velocity_set()
    omega = 1.0 / tau
    nz, ny, nx = labels.shape
    mom = {}
    fstar = {}
    for key, fi in f.items():
        rho = sum(fi.values())
        u = [sum(fi[c] * c[a] for c, _ in vs) / rho for a in range(3)]
        mom[key] = (rho, u)
        fstar[key] = {c: fi[c] - omega * (fi[c] - _feq(w, c, rho, u)) for c, w in vs}
    new = {key: {} for key in f}
    # push every post-collision value to its downstream fluid neighbour
    for (x, y, z), fs in fstar.items():
        for c, _ in vs:
            dst = (x + c[0], y + c[1], z + c[2])
            if dst in new:
                new[dst][c] = fs[c]
    # links whose upstream voxel is not fluid
    for (x, y, z), fi in f.items():
        rho, u = mom[(x, y, z)]
        for c, w in vs:
            if c in new[(x, y, z)]:
                continue
            lab = int(labels[z - c[2], y - c[1], x - c[0]])
            fneq = fi[c] - _feq(w, c, rho, u)
            if lab == 0 and mode == 0:
                cbar = (-c[0], -c[1], -c[2])
                new[(x, y, z)][c] = fstar[(x, y, z)][cbar]
            elif lab == 0:
                k = k_seg[int(segment[z, y, x])]
                dE = max(0.0, (rho / 3.0 - P0) / k)
                dr = 1.0 + dE
                s = (F + dr - 1.0) / dr
                new[(x, y, z)][c] = _feq(w, c, rho, [s * a for a in u]) + (1 - omega) * fneq
            else:
                io = iolets[lab - 2]
                val = io["a0"]
                if io["amp"] != 0.0:
                    val *= 1.0 + io["amp"] * math.sin(2 * math.pi * t / io["period"] + io["phase"])
                d = io.get("direction")
                nn = math.sqrt(sum(a * a for a in d)) if d is not None else 0.0
                if io["kind"] == 0 and nn > 0.0:
                    nv = [a / nn for a in d]
                    un = sum(u[a] * nv[a] for a in range(3))
                    new[(x, y, z)][c] = _feq(w, c, val, [un * a for a in nv])
                elif io["kind"] == 0:
                    new[(x, y, z)][c] = _feq(w, c, val, u)
                else:
                    sp = float(iolet_weight[z, y, x]) * val
                    uin = [sp * d for d in io["direction"]]
                    new[(x, y, z)][c] = _feq(w, c, rho, uin)
    return new


def from_array(coords, f, c_table):
    """Convert an (N, 19) array in an arbitrary direction order ``c_table``
    into the dict form used here."""
    out = {}
    for s, (x, y, z) in enumerate(coords):
        out[(int(x), int(y), int(z))] = {tuple(int(a) for a in c_table[i]): float(f[s, i])
                                         for i in range(19)}
    return out


def to_array(coords, fd, c_table):
    out = np.zeros((len(coords), 19))
    for s, (x, y, z) in enumerate(coords):
        d = fd[(int(x), int(y), int(z))]
        for i in range(19):
            out[s, i] = d[tuple(int(a) for a in c_table[i])]
    return out
