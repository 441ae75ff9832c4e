"""The local slip ratio F (Sec. 2.3 relation, applied per segment as the
Sec. 4 discussion proposes), pinned without Bessel functions: the profile
1 - M J0(Lambda r/R)/J0(Lambda) is the solution of the oscillating
momentum equation that is regular on the axis and moves with the wall, so a
finite-difference solve of that equation must give the same ratio.  No
GPU."""
import math

import numpy as np
import pytest
from scipy.linalg import solve_banded

from paper_2108_08783_amd import inputs, slip


def _profile_fd(M, alpha, n=4000):
    """phi'' + phi'/y = i alpha^2 (phi - 1) on 0 <= y <= 1 (y = r/R), phi
    regular at y = 0, phi(1) = 1 - M; second-order central differences,
    phi'' + phi'/y -> 2 phi'' on the axis."""
    h = 1.0 / n
    y = np.arange(n + 1) * h
    k = 1j * alpha * alpha
    ab = np.zeros((3, n + 1), complex)      # upper, diagonal, lower
    rhs = np.full(n + 1, -k, complex)
    ab[1, 0] = -4.0 / h ** 2 - k
    ab[0, 1] = 4.0 / h ** 2
    j = np.arange(1, n)
    ab[1, j] = -2.0 / h ** 2 - k
    ab[0, j + 1] = 1.0 / h ** 2 + 1.0 / (2 * h * y[j])
    ab[2, j - 1] = 1.0 / h ** 2 - 1.0 / (2 * h * y[j])
    ab[1, n] = 1.0
    ab[2, n - 1] = 0.0
    rhs[n] = 1.0 - M
    return y, solve_banded((1, 1), ab, rhs)


@pytest.mark.parametrize("M", [0.5, 0.828, 0.97, 0.9 + 0.05j])
@pytest.mark.parametrize("alpha", [1.0, 3.0, 6.0, 10.0])
def test_ratio_matches_a_finite_difference_womersley_profile(M, alpha):
    n = 4000
    y, phi = _profile_fd(M, alpha, n)
    for x in (0.02, 0.1, 0.25):
        j = int(round(n * (1 - x)))
        want = phi[n] / phi[j]
        got = complex(slip.F_ratio(M, alpha, x))
        assert abs(got - want) <= 2e-5 * abs(want)


def test_limits():
    for a in (0.5, 3.0, 8.0):
        for x in (0.01, 0.1):
            assert abs(slip.F_ratio(1.0, a, x)) == 0.0          # rigid: no slip
            assert abs(slip.F_ratio(0.0, a, x) - 1.0) < 1e-15     # plug flow
    # the fluid node on the extended wall, and the quasi-steady limit
    assert abs(slip.F_ratio(0.8, 3.0, 1e-9) - 1.0) < 1e-6
    assert abs(slip.F_ratio(0.8, 1e-4, 0.1) - 1.0) < 1e-6


def test_F_falls_with_womersley_number_and_with_relative_gap():
    a = np.linspace(0.5, 10, 40)
    x = np.linspace(0.005, 0.2, 40)
    F = slip.F_local(0.828, a[:, None], x[None, :])
    assert np.all(np.diff(F, axis=0) < 0) and np.all(np.diff(F, axis=1) < 0)
    assert np.all((F > 0) & (F < 1))


def test_calibration_round_trip_and_the_papers_cylinder():
    x = slip.dr_over_R(50.0)
    M = slip.calibrate_M(0.85, 3.0, x)
    assert 0 < M < 1
    assert float(slip.F_local(M, 3.0, x)) == pytest.approx(0.85, abs=1e-10)
    with pytest.raises(ValueError):
        slip.calibrate_M(1.0, 3.0, x)


def test_dr_over_R_reading():
    # undeformed: one spacing over the extended radius r + 1/2
    assert slip.dr_over_R(9.5) == pytest.approx(0.1)
    assert slip.dr_over_R(9.5, dE=0.5) == pytest.approx(1.5 / 10.5)


def test_segment_F_on_a_tree():
    g = inputs.murray_tree(3, scale=0.25)
    M = slip.calibrate_M(0.85, 3.0, slip.dr_over_R(50.0))
    F = slip.segment_F(g, M, period=4000.0, nu=0.1)
    assert F.shape == (g.n_seg,) and np.all((F > 0) & (F < 1))
    # F per segment follows its radius: thinner vessels have a lower alpha
    # but a larger relative gap; check against a direct evaluation
    for s in g.segments[:5]:
        r = 0.5 * (s.r0 + s.r1)
        a = (r + 0.5) * math.sqrt(2 * math.pi / 4000.0 / 0.1)
        assert F[s.sid] == pytest.approx(abs(complex(slip.F_ratio(M, a, 1 / (r + 0.5)))))


def test_segment_F_on_a_cylinder_uses_its_radius():
    g = inputs.cylinder(12, 8)
    F = slip.segment_F(g, 0.8, period=400.0, nu=0.1, dE=0.2)
    a = (12.7) * math.sqrt(2 * math.pi / 400.0 / 0.1)
    assert F.shape == (1,)
    assert F[0] == pytest.approx(abs(complex(slip.F_ratio(0.8, a, 1.2 / 12.7))))
    with pytest.raises(ValueError):
        slip.segment_F(inputs.duct(4, 4, 4), 0.8, period=400.0, nu=0.1)


def test_womersley_shape():
    from paper_2108_08783_amd import verification
    y = np.linspace(0, 1, 11)
    for M in (0.5, 0.83, 0.9 + 0.05j):
        sh = slip.womersley_shape(M, 3.0, y)
        assert abs(sh[-1] - (1 - M)) < 1e-14                      # wall value
        for x in (0.02, 0.1):                                      # F is its ratio
            want = complex(slip.F_ratio(M, 3.0, x))
            got = complex(slip.womersley_shape(M, 3.0, 1.0) / slip.womersley_shape(M, 3.0, 1 - x))
            assert abs(got - want) < 1e-13
    # M = 1 is the rigid profile up to a complex factor
    R, nu = 20.0, 0.1
    omega = (3.0 / R) ** 2 * nu
    rig = verification.womersley_profile(y * R, R, omega, nu, 1e-6)
    sh = slip.womersley_shape(1.0, 3.0, y)
    ratio = rig[:-1] / sh[:-1]
    assert np.abs(ratio / ratio[0] - 1).max() < 1e-10
