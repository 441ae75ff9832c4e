"""Local slip ratio F of the elastic wall rule (Sec. 2.3 and the closing
discussion of Sec. 4).

The wall rule sets the wall-node velocity from U_R = F U_f, F being the
ratio of the oscillating axial velocity at the extended wall (radius R) to
the one at the fluid node (radius R - Delta r).  Under Womersley's profile
for an elastic tube, w(r) proportional to 1 - M J0(Lambda r / R) / J0(Lambda)
(Sec. 2.2), that ratio is

    F = (1 - M) / (1 - M J0(Lambda (1 - Delta r / R)) / J0(Lambda)),

with Lambda = i^(3/2) alpha and alpha = R sqrt(omega / nu) the Womersley
number.  M, the elasticity factor, is a parameter of the vessel and fluid
that the paper leaves to the user.

Readings taken here:
  - F from the relation is complex (the two velocities differ in phase); the
    wall rule takes a real factor, so the applied F is its modulus, the
    ratio of the two oscillation amplitudes;
  - on the lattice the undeformed wall sits on the wall node (Delta r =
    Delta x + Delta E), so a vessel voxelised with radius r (fluid where the
    distance to the axis is < r) has its last fluid nodes half a spacing
    inside r on average, the extended wall at R = r + 1/2 + Delta E, and
    Delta r / R = (1 + Delta E) / (r + 1/2 + Delta E);
  - a per-segment F uses the segment's mean radius and one design
    extension Delta E per segment.

This module runs on the host once per geometry; the values it returns are
handed to the library through ``Lattice.set_wall_F``.
"""
from __future__ import annotations

import cmath
import math
from typing import Sequence

import numpy as np
from scipy.optimize import brentq
from scipy.special import jv

# the library accepts F in [0, 1)
F_MAX = 1.0 - 1e-6


def womersley_number(radius, period, nu):
    """alpha = R sqrt(omega / nu), omega = 2 pi / period (lattice or SI units
    alike)."""
    return np.asarray(radius, float) * np.sqrt(2.0 * math.pi / period / nu)


def womersley_shape(M, alpha, y):
    """Radial shape of the oscillating axial velocity in an elastic tube,
    1 - M J0(Lambda y) / J0(Lambda) with y = r / R (Sec. 2.2); M = 1 is the
    rigid tube (no slip at y = 1)."""
    lam = cmath.exp(0.75j * math.pi) * float(alpha)
    return 1.0 - M * jv(0, lam * np.asarray(y, float)) / jv(0, lam)


def F_ratio(M, alpha, dr_over_R):
    """The complex ratio w(R) / w(R - Delta r) of Sec. 2.3 (vectorised over
    alpha and dr_over_R; M may be complex)."""
    lam = cmath.exp(0.75j * math.pi) * np.asarray(alpha, float)
    x = np.asarray(dr_over_R, float)
    return (1.0 - M) / (1.0 - M * jv(0, lam * (1.0 - x)) / jv(0, lam))


def F_local(M, alpha, dr_over_R):
    """Applied slip ratio: |F_ratio|, limited to the library's [0, 1)."""
    return np.minimum(np.abs(F_ratio(M, alpha, dr_over_R)), F_MAX)


def calibrate_M(F, alpha, dr_over_R):
    """Real M in [0, 1) for which F_local(M, alpha, dr_over_R) = F, e.g. the
    M implied by the paper's choice F = 0.85 for its verification cylinder
    (alpha = 3, radius 50 lattice spacings, small extension)."""
    if not 0.0 < F < 1.0:
        raise ValueError("F must lie in (0, 1)")
    return brentq(lambda m: float(np.abs(F_ratio(m, alpha, dr_over_R))) - F, 0.0, 1.0 - 1e-12,
                  xtol=1e-14)


def dr_over_R(radius, dE=0.0):
    """Delta r / R for a vessel voxelised with the given radius (lattice
    spacings) and design extension dE (reading above)."""
    r = np.asarray(radius, float)
    return (1.0 + dE) / (r + 0.5 + dE)


def segment_radii(geo) -> np.ndarray:
    """Radius per wall segment id (lattice spacings): the mean (r0 + r1) / 2
    of each generated segment, or the radius of a straight cylinder."""
    if geo.segments:
        r = np.full(geo.n_seg, np.nan)
        for s in geo.segments:
            r[s.sid] = 0.5 * (s.r0 + s.r1)
        if np.isnan(r).any():
            raise ValueError("segment ids without a radius")
        return r
    if geo.info.get("kind") == "cylinder":
        return np.full(geo.n_seg, float(geo.info["R"]))
    raise ValueError("the geometry carries no segment radii")


def segment_F(geo, M, period, nu, dE: float | Sequence[float] = 0.0):
    """One F per wall segment id of a generated geometry.  dE: design
    extension, scalar or one value per segment id.  Returns float64
    [geo.n_seg]."""
    r = segment_radii(geo)
    dE = np.broadcast_to(np.asarray(dE, float), r.shape)
    return F_local(M, womersley_number(r + 0.5 + dE, period, nu), dr_over_R(r, dE))
