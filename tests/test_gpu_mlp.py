"""Warm-start network kernels (bf16 MFMA GEMM, forward, backward, loss,
Adam) against the FP64 NumPy reference on identical bf16-rounded inputs.

Tolerances: the GEMM accumulates in FP32, so it matches FP64 on the same
bf16 operands to ~1e-6 relative.  Forward and backward round activations
and back-propagated gradients to bf16 between layers (2^-9 relative per
rounding), so whole tensors are held to 1e-2 relative (max-norm) and the
FP32-accumulated loss to 1e-3."""
import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _t(x, dtype):
    import torch
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("M_,N_,K_", [(1, 1, 1), (64, 64, 32), (130, 70, 45), (257, 128, 16),
                                      (128, 128, 1000)])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("tb", [0, 1])
def test_gemm_matches_numpy(M_, N_, K_, ta, tb):
    import torch
    from paper_2108_08783_amd import mlp
    rng = np.random.default_rng(M_ * 7 + N_ + K_)
    A = M.bf16_round(rng.normal(size=(K_, M_) if ta else (M_, K_)))
    B = M.bf16_round(rng.normal(size=(N_, K_) if tb else (K_, N_)))
    ref = (A.T if ta else A) @ (B.T if tb else B)
    At, Bt = _t(A, torch.bfloat16), _t(B, torch.bfloat16)
    C = torch.full((M_, N_), 7.0, dtype=torch.float32, device="cuda")
    mlp.mlp_gemm_bf16(M_, N_, K_, At, A.shape[1], ta, Bt, B.shape[1], tb, C, N_)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()) * np.sqrt(K_)
    # accumulate flag adds to C
    mlp.mlp_gemm_bf16(M_, N_, K_, At, A.shape[1], ta, Bt, B.shape[1], tb, C, N_, accumulate=True)
    torch.cuda.synchronize()
    assert np.allclose(C.cpu().numpy(), 2 * got, rtol=1e-6, atol=1e-6)


def _net_and_ref(n=300, dims=(16, 128, 4, 4), seed=3):
    import torch
    from paper_2108_08783_amd import mlp
    rng = np.random.default_rng(seed)
    p = M.bf16_round(mlp.init_params(*dims, seed=seed))
    p[-dims[3]:] = M.bf16_round(rng.normal(0, 0.1, dims[3]))
    net = mlp.Net(*dims, params=p)
    X = M.bf16_round(rng.normal(size=(n, dims[0])))
    Xb = net.to_bf16(_t(X, torch.float32))
    return net, p, X, Xb, M.layer_dims(*dims)


def _rel(a, b):
    r = np.abs(a - b).max() / np.abs(b).max()
    print(f"MLP rel err {r:.3e}", flush=True)
    return r


def test_forward_matches_reference():
    net, p, X, Xb, d = _net_and_ref()
    Y = net.forward(Xb).cpu().numpy()
    Yr, _ = M.forward(p, X, d)
    assert _rel(Y, Yr) <= 1e-2


def test_inference_equals_the_forward_output():
    """The inference pass (no pre-activations stored) gives the forward
    pass's output bit for bit, on 70,001 samples (many tiles and a ragged
    last one), and stays within the forward bound of the reference."""
    import torch
    net, p, X, Xb, d = _net_and_ref(n=70001)
    Yf = net.forward(Xb).clone()
    net.Z.fill_(float("nan"))              # inference must write its whole output
    Yi = net.infer(Xb)
    torch.cuda.synchronize()
    assert torch.equal(Yf, Yi)
    Yr, _ = M.forward(p, X, d)
    assert _rel(Yi.cpu().numpy(), Yr) <= 1e-2


def test_backward_matches_reference():
    import torch
    net, p, X, Xb, d = _net_and_ref(n=257)
    rng = np.random.default_rng(9)
    dY = rng.normal(size=(257, 4))
    net.forward(Xb)
    g = net.backward(Xb, _t(dY, torch.float32)).cpu().numpy()
    Yr, cache = M.forward(p, X, d)
    gr = M.backward(p, cache, dY, d)
    off = 0
    for i, o in d:          # per tensor: W then b
        for size in (i * o, o):
            assert _rel(g[off:off + size], gr[off:off + size]) <= 1e-2, (i, o, size)
            off += size


def test_backward_with_split_sums_matches_reference_and_is_deterministic():
    """40,000 samples: the weight-gradient products and the bias sums over
    the samples are split into partial ranges (4 and 40) that are added in a
    fixed order.  Against the reference, and bit-identical on a second call."""
    import torch
    n = 40000
    net, p, X, Xb, d = _net_and_ref(n=n)
    rng = np.random.default_rng(11)
    dY = rng.normal(size=(n, 4))
    net.forward(Xb)
    g1 = net.backward(Xb, _t(dY, torch.float32)).cpu().numpy().copy()
    g2 = net.backward(Xb, _t(dY, torch.float32)).cpu().numpy()
    assert np.array_equal(g1, g2)
    Yr, cache = M.forward(p, X, d)
    gr = M.backward(p, cache, dY, d)
    off = 0
    for i, o in d:          # per tensor: W then b
        for size in (i * o, o):
            assert _rel(g1[off:off + size], gr[off:off + size]) <= 1e-2, (i, o, size)
            off += size


def test_loss_and_adam_match_reference():
    import torch
    from paper_2108_08783_amd import mlp
    net, p, X, Xb, d = _net_and_ref(n=200)
    rng = np.random.default_rng(4)
    T = rng.normal(size=(200, 4))
    w = np.array([4.0, 1.0, 1.0, 0.5])
    loss = net.train_step(Xb, _t(T, torch.float32), _t(w, torch.float32), lr=1e-3)
    Yr, cache = M.forward(p, X, d)
    Lr, dYr = M.mse(Yr, T, w)
    print(f"MLP loss rel err {abs(loss.item() - Lr) / Lr:.3e}", flush=True)
    assert loss.item() == pytest.approx(Lr, rel=1e-3)
    gr = M.backward(p, cache, dYr, d)
    pr, _, _ = M.adam(p, gr, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    step_gpu = net.state() - p
    step_ref = pr - p
    big = np.abs(gr) > 1e-3 * np.abs(gr).max()       # sign-stable entries
    assert np.allclose(step_gpu[big], step_ref[big], rtol=2e-2, atol=1e-6)


def test_training_reduces_loss():
    import torch
    from paper_2108_08783_amd import mlp
    rng = np.random.default_rng(5)
    n = 4096
    X = rng.uniform(-1, 1, (n, 16))
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], X[:, 2] ** 2, np.tanh(X[:, 3] + X[:, 4]),
                  0.5 * X[:, 5]], 1)
    net = mlp.Net(seed=1)
    Xb = net.to_bf16(_t(X, torch.float32))
    Tt = _t(T, torch.float32)
    first = net.train_step(Xb, Tt, lr=2e-3).item()
    for _ in range(400):
        last = net.train_step(Xb, Tt, lr=2e-3)
    assert last.item() < first / 10


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 70001])
def test_fused_inference_matches_forward_and_reference(n):
    """mlp_infer_fused (every layer in one launch, weights in LDS, operands
    passed between layers by lane swaps) against the layer-by-layer forward
    pass on the same bf16 weights and inputs (FP32 rounding order and SiLU
    reciprocal differ, so a hidden activation may round to the neighbouring
    bf16 value: held to 5e-3 of the output range) and against the FP64
    reference (1e-2), for ragged sample counts."""
    import torch
    net, p, X, Xb, d = _net_and_ref(n=n)
    Yf = net.forward(Xb).clone()
    Y = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
    net.infer_fused(Xb, Y)
    torch.cuda.synchronize()
    Yn = Y.cpu().numpy()
    assert np.isfinite(Yn).all()
    diff = np.abs(Yn - Yf.cpu().numpy()).max() / np.abs(Yf.cpu().numpy()).max()
    print(f"MLP fused vs forward {diff:.3e}", flush=True)
    assert diff <= 5e-3
    Yr, _ = M.forward(p, X, d)
    assert _rel(Yn, Yr) <= 1e-2


@pytest.mark.parametrize("dims", [(7, 128, 2, 3), (32, 128, 5, 16), (16, 128, 1, 1)])
def test_fused_inference_other_shapes(dims):
    """Input widths that are not a multiple of 8 (element-wise staging),
    1 to 5 hidden layers and 1 to 16 outputs, against the FP64 reference."""
    import torch
    net, p, X, Xb, d = _net_and_ref(n=777, dims=dims, seed=5)
    Y = net.infer_fused(Xb)
    torch.cuda.synchronize()
    Yr, _ = M.forward(p, X, d)
    assert _rel(Y.cpu().numpy(), Yr) <= 1e-2


def test_fused_inference_rejects_unsupported_shapes():
    import torch
    from paper_2108_08783_amd import mlp
    net = mlp.Net(n_in=16, width=64, depth=2, n_out=4, seed=1)
    Xb = net.to_bf16(torch.zeros(10, 16, device="cuda"))
    with pytest.raises(RuntimeError):
        net.infer_fused(Xb)
    net = mlp.Net(seed=1)
    Y = net.infer_fused(torch.zeros((0, 16), dtype=torch.bfloat16, device="cuda"))
    assert Y.shape == (0, 4)
