"""Pins of the FP64 network reference: gradients against central finite
differences, the loss gradient against its definition, Adam's first step
against its closed form, and bf16 rounding against exhaustive cases."""
import numpy as np
import pytest

from oracle import mlp as M


@pytest.mark.parametrize("dims", [(5, 7, 2, 3), (16, 12, 4, 4)])
def test_backward_matches_finite_differences(dims):
    rng = np.random.default_rng(0)
    d = M.layer_dims(*dims)
    p = rng.normal(0, 0.5, M.n_params(d))
    X = rng.normal(0, 1, (9, dims[0]))
    dY = rng.normal(0, 1, (9, dims[3]))
    Y, cache = M.forward(p, X, d)
    g = M.backward(p, cache, dY, d)
    h = 1e-6
    idx = rng.choice(len(p), 40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = ((M.forward(p + e, X, d)[0] * dY).sum() - (M.forward(p - e, X, d)[0] * dY).sum()) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_silu_derivative_and_values():
    z = np.linspace(-8, 8, 101)
    assert np.allclose(M.silu(z), z / (1 + np.exp(-z)))
    fd = (M.silu(z + 1e-6) - M.silu(z - 1e-6)) / 2e-6
    assert np.allclose(M.dsilu(z), fd, atol=1e-8)
    assert M.silu(0.0) == 0.0 and M.dsilu(0.0) == 0.5


def test_mse_gradient():
    rng = np.random.default_rng(1)
    Y, T, w = rng.normal(size=(6, 4)), rng.normal(size=(6, 4)), rng.uniform(0.5, 2, 4)
    L, dY = M.mse(Y, T, w)
    assert L == pytest.approx((w * (Y - T) ** 2).mean())
    e = np.zeros_like(Y)
    e[2, 1] = 1e-6
    assert dY[2, 1] == pytest.approx((M.mse(Y + e, T, w)[0] - M.mse(Y - e, T, w)[0]) / 2e-6, rel=1e-6)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = M.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g))


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-30, 65504.0])
    r = M.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0          # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7                # tie rounds up to even
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8)
