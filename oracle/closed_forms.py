"""Closed forms and unit conversions used to pin the oracle.

TEST INFRASTRUCTURE ONLY.  Everything here is textbook fluid mechanics or the
paper's own relations, evaluated independently of the oracle's C code.
"""
from __future__ import annotations

import cmath
import math

import numpy as np


# ----------------------------------------------------------------- units --
def tau_from_physical(nu, dx, dt):
    """Sec. 2.1 eq. Viscosity, nu = C_s^2 (tau - 1/2) in lattice units, with
    nu_lattice = nu dt / dx^2 and C_s^2 = 1/3."""
    return 0.5 + 3.0 * nu * dt / (dx * dx)


def womersley_number(R, omega, rho, mu):
    """Sec. 2.2: alpha = R sqrt(omega rho / mu)."""
    return R * math.sqrt(omega * rho / mu)


def wall_stiffness(Y, h, sigma, R):
    """Sec. 2.4: Delta E = ((1 - sigma^2) R^2 / (Y h)) (p - P0), so the
    stiffness is k = Y h / ((1 - sigma^2) R^2) (pressure per length)."""
    return Y * h / ((1.0 - sigma * sigma) * R * R)


def stiffness_lattice(k_phys, rho, dx, dt):
    """k in lattice units: pressure unit rho dx^2/dt^2, length unit dx."""
    return k_phys * dx / (rho * dx * dx / (dt * dt))


# ------------------------------------------------------- steady channels --
def plane_poiseuille(y, h, G, mu):
    """u(y) = G/(2 mu) (h^2 - y^2) between walls at y = +-h, G = -dp/dz."""
    return G / (2.0 * mu) * (h * h - y * y)


def slip_half_width_sq(Yw, F):
    """Half-width^2 b^2 of the parabola A (b^2 - y^2) whose value at the wall
    node Y_w equals F times its value at the last fluid node Y_w - 1 (the
    elastic rule of Sec. 2.3 with Delta E = 0, i.e. U_w = F U_f)."""
    return (Yw * Yw - F * (Yw - 1.0) ** 2) / (1.0 - F)


def slip_poiseuille_two_walls(y, Yw, F_lo, F_hi, A):
    """Steady plane Poiseuille u(y) = -A y^2 + beta y + gamma between wall
    nodes at y = -Y_w and y = +Y_w whose slip ratios differ (the elastic
    rule of Sec. 2.3 with Delta E = 0 on each wall: u(wall node) = F u(last
    fluid node)).  The two slip conditions are linear in (beta, gamma)."""
    y1 = Yw - 1.0
    # lower wall: u(-Yw) - F_lo u(-y1) = 0; upper wall: u(Yw) - F_hi u(y1) = 0
    M = np.array([[-Yw + F_lo * y1, 1.0 - F_lo],
                  [Yw - F_hi * y1, 1.0 - F_hi]])
    rhs = np.array([A * (Yw * Yw - F_lo * y1 * y1), A * (Yw * Yw - F_hi * y1 * y1)])
    beta, gamma = np.linalg.solve(M, rhs)
    y = np.asarray(y, float)
    return -A * y * y + beta * y + gamma


def duct_poiseuille(x, y, a, b, G, mu, nterms=101):
    """Fully developed flow in the rectangle |x| < a, |y| < b (Fourier series,
    e.g. White, Viscous Fluid Flow, Sec. 3-3)."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    u = np.zeros(np.broadcast(x, y).shape)
    for n in range(1, 2 * nterms, 2):
        k = n * math.pi / (2.0 * a)
        # cosh(k y)/cosh(k b) written with exponentials to avoid overflow
        ratio = np.exp(k * (np.abs(y) - b)) * (1.0 + np.exp(-2 * k * np.abs(y))) / (
            1.0 + math.exp(-2 * k * b))
        u += ((-1) ** ((n - 1) // 2)) / n ** 3 * (1.0 - ratio) * np.cos(k * x)
    return 16.0 * G * a * a / (mu * math.pi ** 3) * u


# ------------------------------------------------------ oscillatory flow --
def bessel_j(n, z, terms=80):
    """J_n(z) for complex z by its power series sum_k (-1)^k (z/2)^(2k+n) /
    (k! (k+n)!)."""
    z = complex(z)
    s = 0j
    term = (z / 2) ** n / math.factorial(n)
    for k in range(terms):
        s += term
        term *= -(z / 2) ** 2 / ((k + 1) * (k + 1 + n))
    return s


def womersley_pipe(r, R, alpha, G_hat, rho, omega):
    """Complex amplitude of the axial velocity in a rigid pipe driven by the
    pressure gradient -dp/dz = Re[G_hat e^{i omega t}] (Sec. 2.2 with M = 1
    and c -> infinity): (G_hat/(i omega rho)) (1 - J0(Lambda r/R)/J0(Lambda)),
    Lambda = i^{3/2} alpha."""
    lam = cmath.exp(1.5j * math.pi / 2) * alpha
    j0l = bessel_j(0, lam)
    r = np.atleast_1d(np.asarray(r, float))
    out = np.array([(G_hat / (1j * omega * rho)) * (1 - bessel_j(0, lam * ri / R) / j0l) for ri in r])
    return out


def womersley_plane(y, h, nu, G_hat, rho, omega):
    """Complex amplitude of the velocity between plates at y = +-h driven by
    -dp/dz = Re[G_hat e^{i omega t}]: (G_hat/(i omega rho))
    (1 - cosh(k y)/cosh(k h)), k = sqrt(i omega / nu)."""
    k = cmath.sqrt(1j * omega / nu)
    y = np.atleast_1d(np.asarray(y, float))
    return np.array([(G_hat / (1j * omega * rho)) * (1 - cmath.cosh(k * yi) / cmath.cosh(k * h))
                     for yi in y])
