"""The verification-cylinder set-up (Sec. 2.4, Table A1) against the
oracle's independent unit conversions and closed forms.  No GPU."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from paper_2108_08783_amd import verification as V


@pytest.mark.parametrize("R", [50, 100, 200])
def test_lattice_parameters_match_table_a1(R):
    c = V.case(R)
    dx, dt = V.RESOLUTIONS[R]
    assert c.tau == pytest.approx(cf.tau_from_physical(V.MU / V.RHO, dx, dt), rel=1e-12)
    assert round(c.tau, 3) == pytest.approx({50: 0.537, 100: 0.573, 200: 0.646}[R], abs=1.5e-3)
    assert c.L == round(0.04 / dx)
    assert c.alpha == pytest.approx(3.0, rel=2e-3)
    k_phys = cf.wall_stiffness(V.YOUNG, V.H_OVER_R * V.R_M, V.POISSON, V.R_M)
    assert c.k == pytest.approx(cf.stiffness_lattice(k_phys, V.RHO, dx, dt), rel=1e-12)
    # the lattice Womersley number of the period in steps equals the physical one
    alpha_lu = R * math.sqrt(2 * math.pi / c.period / c.nu)
    assert alpha_lu == pytest.approx(c.alpha, rel=2e-3)


def test_gradient_amplitude_in_lattice_units():
    c = V.case(50, kp=50.0)
    dx, dt = V.RESOLUTIONS[50]
    # 50 Pa/m times the length unit over the pressure unit rho dx^2 / dt^2
    assert c.G == pytest.approx(50.0 * dx / (V.RHO * dx * dx / (dt * dt)), rel=1e-12)
    assert V.case(50, kp=-150.0).G == pytest.approx(3 * c.G, rel=1e-12)


def test_womersley_profile_matches_the_oracle_closed_form():
    R, nu = 49.9, 0.0123
    omega = 2 * math.pi / 142800
    G = 1e-7 * np.exp(0.3j)
    r = np.linspace(0.0, R, 9)
    alpha = R * math.sqrt(omega / nu)
    a = V.womersley_profile(r, R, omega, nu, G)
    b = cf.womersley_pipe(r, R, alpha, G, 1.0, omega)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_same_dimensionless_problem_at_another_tau():
    a, b = V.case(50), V.case(50, tau=0.573)
    assert b.tau == 0.573 and b.alpha == a.alpha
    assert 50 * math.sqrt(2 * math.pi / b.period / b.nu) == pytest.approx(3.0, rel=1e-3)
    # lattice velocities G R^2 / nu and the stiffness-to-pressure ratio kept
    assert b.G / b.nu == pytest.approx(a.G / a.nu, rel=1e-12)
    assert b.k / b.G == pytest.approx(a.k / a.G, rel=1e-12)
