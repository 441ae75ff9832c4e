"""Host-side pieces of the learned warm start: the one-dimensional network
prior against the limits it must reach (slip Poiseuille at low frequency, a
lossless acoustic line for a full-slip wall, mass conservation, the slip
condition itself) and the feature layout.  No GPU."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import jv

from paper_2108_08783_amd import inputs, warmstart

NU = 0.1


@pytest.mark.parametrize("s", [0.0, 0.5, 0.85])
def test_womersley_low_frequency_limit_is_slip_poiseuille(s):
    # omega -> 0: the series impedance i omega / (pi r^2 m) must become the
    # steady resistance 4 nu / (pi r^2 (b^2 - r^2/2)) of the slip parabola
    r = 10.0
    omega = 1e-7
    kw = np.sqrt(-1j * omega / NU)
    _, m = warmstart._womersley(r, s, kw)
    Z = 1j * omega / (math.pi * r * r * m)
    b2 = warmstart._b2(r, s)
    R = 4 * NU / (math.pi * r * r * (b2 - 0.5 * r * r))
    assert abs(Z - R) / R < 1e-4


@pytest.mark.parametrize("r,s", [(6.0, 0.0), (20.0, 0.5), (40.0, 0.85)])
def test_womersley_profile_meets_the_slip_condition_and_its_mean(r, s):
    omega = 2 * math.pi / 4000
    kw = np.sqrt(-1j * omega / NU)
    beta, m = warmstart._womersley(r, s, kw)
    prof = lambda y: 1.0 + beta * jv(0, kw * y)
    Rw = r + 0.5
    # slip rule: the wall node carries s times the velocity one node inside
    assert abs(prof(Rw) - s * prof(Rw - 1.0)) < 1e-12 * max(1.0, abs(prof(Rw - 1.0)))
    # the mean over the disk y < r, by quadrature
    re = integrate.quad(lambda y: (prof(y) * 2 * y).real, 0, r, limit=200)[0] / (r * r)
    im = integrate.quad(lambda y: (prof(y) * 2 * y).imag, 0, r, limit=200)[0] / (r * r)
    assert abs(complex(re, im) - m) < 1e-9 * abs(m)


def test_womersley_profile_satisfies_the_oscillating_momentum_equation():
    # i omega u = -dp/dx + nu lap(u) with -dp/dx = i omega C0 (C0 = 1)
    r, s = 15.0, 0.3
    omega = 2 * math.pi / 4000
    kw = np.sqrt(-1j * omega / NU)
    beta, _ = warmstart._womersley(r, s, kw)
    u = lambda y: 1.0 + beta * jv(0, kw * y)
    for y in (1.0, 5.0, 12.0):
        h = 1e-3
        d2 = (u(y + h) - 2 * u(y) + u(y - h)) / h ** 2
        d1 = (u(y + h) - u(y - h)) / (2 * h)
        lap = d2 + d1 / y
        assert abs(1j * omega * u(y) - (1j * omega + NU * lap)) < 1e-7


def _tube(r=8.0, length=120.0):
    g = inputs.straight_tube_x(r, length)
    return g, warmstart.site_frames(g)


def _section(fr, t0, t1):
    t = fr.static[:, 3]
    return (t > t0) & (t < t1)


def test_prior_mean_flow_conserves_the_inlet_flow():
    g, fr = _tube()
    u0 = 0.02
    P = warmstart.network_prior(g, fr, [1e9], 0.85, 1 / 3, u0, 0.0, nu=NU, amp=0.0)
    r = fr.r
    for lo in (0.2, 0.5, 0.8):
        sel = _section(fr, lo, lo + 0.02)
        # area-weighted mean axial velocity over the disk: the profile is
        # normalised to mean 1 over y < r, so its site mean is close to 1
        d = r[sel] * (1 - fr.static[sel, 0])
        inside = d < r[sel] - 1
        assert abs(P.Y[sel, 1][inside].mean() - 1.0) < 0.08


def _excess_pressure(P, u0):
    # output 0 is (3p - 1)/(10 u0), so p - 1/3 = out * 10 u0 / 3
    return P.Y[:, 0] * 10 * u0 / 3


def test_prior_low_frequency_is_quasi_steady():
    # period -> infinity: at a quarter period (flow 1 + amp times the mean)
    # pressure excess and velocity are the steady ones scaled by 1 + amp
    g, fr = _tube()
    u0, amp = 0.02, 0.5
    k = [1e9]                                   # stiff: constant slip F
    base = warmstart.network_prior(g, fr, k, 0.85, 1 / 3, u0, 0.0, nu=NU, amp=0.0, period=1e9)
    peak = warmstart.network_prior(g, fr, k, 0.85, 1 / 3, u0, 0.25, nu=NU, amp=amp, period=1e9)
    dps, dpp = _excess_pressure(base, u0), _excess_pressure(peak, u0)
    sel = dps > 0.2 * dps.max()
    assert np.allclose(dpp[sel], (1 + amp) * dps[sel], rtol=1e-4)
    assert np.allclose(peak.Y[:, 1], (1 + amp) * base.Y[:, 1], rtol=1e-4, atol=1e-6)


def test_prior_full_slip_line_is_a_lossless_acoustic_line():
    # F = 1 (slip factor 1, plug flow, no viscous drop): an inviscid line
    # with wave speed c = 1/sqrt(3), flow amplitude -i amp A u0 at x = 0 and
    # p = P0 at x = L has the pressure phasor
    #   p(x) - P0 = c amp u0 sin(w (L - x)/c) / cos(w L/c)   (real)
    g, fr = _tube(r=8.0, length=100.0)
    seg = g.segments[0]
    L = float(np.linalg.norm(seg.p1 - seg.p0))
    c = 1 / math.sqrt(3)
    omega = c * (math.pi / 4) / L
    u0, amp = 0.02, 0.5
    kw = dict(nu=NU, amp=amp, period=2 * math.pi / omega, n_sub=64)
    p0 = warmstart.network_prior(g, fr, [1e9], 1.0, 1 / 3, u0, 0.0, **kw)
    p1 = warmstart.network_prior(g, fr, [1e9], 1.0, 1 / 3, u0, 0.25, **kw)
    x = fr.static[:, 3] * L
    want = c * amp * u0 * np.sin(omega * (L - x) / c) / math.cos(omega * L / c)
    assert np.abs(_excess_pressure(p0, u0) - want).max() < 1e-3 * want.max()
    assert np.abs(_excess_pressure(p1, u0)).max() < 1e-3 * want.max()


def test_feature_layout():
    g, fr = _tube()
    P = warmstart.network_prior(g, fr, [0.01], 0.5, 1 / 3, 0.02, 0.1, nu=NU)
    X = warmstart.features(fr, [0.01], 0.02, 0.1, P)
    assert X.shape == (fr.static.shape[0], warmstart.N_FEAT)
    assert np.array_equal(X[:, 5], P.Y[:, 0]) and np.array_equal(X[:, 10], P.Y[:, 1])
    assert np.array_equal(X[:, 11], P.slip)
    # one generation-0 tube of radius 8: absolute radius, radius over the
    # inlet's, the generation one-hot
    assert np.allclose(X[:, 1], 8.0 / 24.0) and np.allclose(X[:, 2], 1.0)
    assert np.all(X[:, 7] == 1.0) and np.all(X[:, 8:10] == 0.0)
    # the scale-free set: radius over the reference, generation 0, slots 7-9 unused
    Xs = warmstart.features(warmstart.site_frames(g, "scale_free"), [0.01], 0.02, 0.1, P)
    assert np.all(Xs[:, 1] == 1.0) and np.all(Xs[:, 2] == 0.0) and np.all(Xs[:, 7:10] == 0.0)
    assert np.array_equal(np.delete(Xs, [1, 2, 7, 8, 9], 1), np.delete(X, [1, 2, 7, 8, 9], 1))
    assert np.allclose(X[:, 14], math.sin(0.2 * math.pi)) and np.allclose(X[:, 15], math.cos(0.2 * math.pi))


def test_local_feature_layout():
    """The local set on one tube of radius 8 (no junctions): radius over the
    reference 1, the local Womersley number r sqrt(omega / nu) / 3,
    distances to the ends in radii (/ 16, capped), junction flags 0, the
    prior's axial velocity in the section's mean-flow velocity, and the
    correction unit of each site that velocity (here u0: one section)."""
    g, _ = _tube()
    fr = warmstart.site_frames(g, "local")
    assert fr.kind == "local"
    P = warmstart.network_prior(g, fr, [0.01], 0.5, 1 / 3, 0.02, 0.1, nu=NU)
    X = warmstart.features(fr, [0.01], 0.02, 0.1, P)
    kappa = math.sqrt(2 * math.pi / 4000.0 / NU)
    assert np.allclose(P.kappa, kappa)
    assert np.all(X[:, 1] == 1.0) and np.allclose(X[:, 2], 8.0 * kappa / 3.0)
    L = float(np.linalg.norm(g.segments[0].p1 - g.segments[0].p0))
    t = fr.static[:, 3].astype(np.float64)
    assert np.allclose(X[:, 4], np.minimum(t * L / 8.0, 16.0) / 16.0, atol=1e-6)
    assert np.allclose(X[:, 6], np.minimum((1 - t) * L / 8.0, 16.0) / 16.0, atol=1e-6)
    assert np.all(X[:, 5] == 0.0) and np.all(X[:, 7:10] == 0.0)
    assert np.allclose(P.scale, 1.0)
    assert np.allclose(X[:, 10], P.Y[:, 1] / P.scale)
    assert np.array_equal(warmstart.out_scale(fr, P), P.scale)
    absolute = warmstart.site_frames(g)
    assert np.all(warmstart.out_scale(absolute, P) == 1.0)


def test_tree_features_are_free_of_the_scale():
    """With the scale-free feature set, on a Murray tree the radius feature
    is r(t) over the parent's end radius and the generation feature is the
    segment's generation; both, and the other geometric features, take the
    same values per segment at quarter and at half scale (the held-out trees
    are larger than the training vessels, so an absolute radius would put
    them outside the range)."""
    stats = []
    for scale in (0.25, 0.5):
        g = inputs.murray_tree(2000, scale=scale)
        fr = warmstart.site_frames(g, "scale_free")
        segs = {sg.sid: sg for sg in g.segments}
        parent, _ = warmstart._topology(g.segments)
        rref = {sg.sid: (g.segments[parent[j]].r1 if parent[j] >= 0 else sg.r0)
                for j, sg in enumerate(g.segments)}
        ref = np.array([rref[int(s)] for s in fr.seg])
        assert np.allclose(fr.static[:, 1], fr.r / ref, rtol=1e-6)
        gen = np.array([segs[int(s)].gen for s in fr.seg])
        assert np.array_equal(fr.static[:, 2], gen.astype(np.float32))
        assert np.all(fr.static[:, 7:10] == 0.0)
        # per-segment mean of the scale-free geometric features
        ids = sorted(segs)
        stats.append(np.array([[fr.static[fr.seg == i][:, j].mean() for j in (1, 2, 3, 4)]
                               for i in ids]))
    assert stats[0].shape == stats[1].shape
    assert np.abs(stats[0] - stats[1]).max() < 0.08


def test_feature_range_gate():
    rng = np.random.default_rng(0)
    X = rng.uniform(0, 1, (1000, warmstart.N_FEAT)).astype(np.float32)
    X[:, 9] = 0.0                                   # a slot never set in training
    r = warmstart.feature_range(X)
    assert warmstart.in_range(X, r).all()
    Y = X[:5].copy()
    Y[0, 3] = 1.2                                   # beyond the 5 % margin
    Y[1, 3] = 1.04                                  # inside it
    Y[2, 9] = 1.0                                   # the unseen slot
    assert warmstart.in_range(Y, r).tolist() == [False, True, False, True, True]
    assert warmstart.in_range(Y, None).all()
