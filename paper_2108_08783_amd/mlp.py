"""ctypes binding of the warm-start network kernels (C ABI in
``include/lbm_mlp.h``), with torch tensors as device memory.

The functions keep the C names and only marshal pointers; ``Net`` owns the
parameter, moment and activation tensors of one network and runs forward,
backward and Adam steps through the library's kernels on torch's current
stream.
"""
from __future__ import annotations

import ctypes
import math
import sys

import numpy as np

from . import lbm

MLP_EXPORTS = ["mlp_param_count", "mlp_act_floats", "mlp_act_bf16", "mlp_gemm_bf16",
               "mlp_forward", "mlp_infer", "mlp_backward", "mlp_mse", "mlp_mse_partials", "mlp_adam",
               "mlp_to_bf16", "mlp_last_error", "mlp_infer_fused"]


class Shape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("width", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("n_out", ctypes.c_int32)]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    lib = lbm.load()
    P, I, L, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
    sig = {
        "mlp_param_count": ([P], L), "mlp_act_floats": ([P, L], L), "mlp_act_bf16": ([P, L], L),
        "mlp_gemm_bf16": ([I, I, I, P, I, I, P, I, I, P, I, I, P], I),
        "mlp_forward": ([P, P, P, L, P, P, P, P], I),
        "mlp_infer": ([P, P, P, L, P, P, P, P], I),
        "mlp_infer_fused": ([P, P, P, L, P, P, P], I),
        "mlp_backward": ([P, P, L, P, P, P, P, P, P, P, P], I),
        "mlp_mse": ([L, I, P, P, P, P, P, P, P], I), "mlp_mse_partials": ([L, I], L),
        "mlp_adam": ([L, P, P, P, P, P, F, F, F, F, L, P], I),
        "mlp_to_bf16": ([L, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    lib.mlp_last_error.argtypes = []
    lib.mlp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"{load().mlp_last_error().decode()} (status {rc})")


def mlp_param_count(shape):
    return int(load().mlp_param_count(ctypes.byref(shape)))


def mlp_gemm_bf16(M, N, K, A, lda, transA, B, ldb, transB, C, ldc, accumulate=False):
    _check(load().mlp_gemm_bf16(M, N, K, _ptr(A), lda, int(transA), _ptr(B), ldb, int(transB),
                                _ptr(C), ldc, int(accumulate), _stream()))


def mlp_to_bf16(x, y):
    _check(load().mlp_to_bf16(x.numel(), _ptr(x), _ptr(y), _stream()))


def mlp_forward(shape, params, wb, n, X, Z, A):
    _check(load().mlp_forward(ctypes.byref(shape), _ptr(params), _ptr(wb), n, _ptr(X), _ptr(Z),
                              _ptr(A), _stream()))


def mlp_infer(shape, params, wb, n, X, Z, A):
    _check(load().mlp_infer(ctypes.byref(shape), _ptr(params), _ptr(wb), n, _ptr(X), _ptr(Z),
                              _ptr(A), _stream()))


def mlp_infer_fused(shape, params, wb, n, X, Y):
    _check(load().mlp_infer_fused(ctypes.byref(shape), _ptr(params), _ptr(wb), n, _ptr(X), _ptr(Y),
                                  _stream()))


def mlp_backward(shape, wb, n, X, Z, A, dY, grad, work_f, work_b):
    _check(load().mlp_backward(ctypes.byref(shape), _ptr(wb), n, _ptr(X), _ptr(Z), _ptr(A),
                               _ptr(dY), _ptr(grad), _ptr(work_f), _ptr(work_b), _stream()))


def mlp_mse(n, c, Y, T, w, dY, loss, partial):
    _check(load().mlp_mse(n, c, _ptr(Y), _ptr(T), _ptr(w), _ptr(dY), _ptr(loss), _ptr(partial),
                          _stream()))


def mlp_adam(params, wb, grad, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().mlp_adam(params.numel(), _ptr(params), _ptr(wb), _ptr(grad), _ptr(m), _ptr(v),
                           float(lr), float(beta1), float(beta2), float(eps), int(t), _stream()))


def init_params(n_in, width, depth, n_out, seed=0):
    """He-uniform weights, zero biases, in the library's layout (FP64)."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(depth + 1):
        i = n_in if l == 0 else width
        o = n_out if l == depth else width
        bound = math.sqrt(6.0 / i) if l < depth else math.sqrt(1.0 / i)
        out += [rng.uniform(-bound, bound, (o, i)).ravel(), np.zeros(o)]
    return np.concatenate(out)


class Net:
    """One network on the GPU: FP32 master parameters, bf16 copy, Adam
    moments; activations are (re)allocated per batch size."""

    def __init__(self, n_in=16, width=128, depth=4, n_out=4, seed=0, params=None):
        import torch
        self.shape = Shape(n_in, width, depth, n_out)
        self.n_param = mlp_param_count(self.shape)
        p = init_params(n_in, width, depth, n_out, seed) if params is None else np.asarray(params)
        assert p.size == self.n_param
        dev = torch.device("cuda")
        self.params = torch.tensor(p, dtype=torch.float32, device=dev)
        self.wb = torch.empty(self.n_param, dtype=torch.bfloat16, device=dev)
        mlp_to_bf16(self.params, self.wb)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.t = 0
        self._n = -1

    def _buffers(self, n):
        import torch
        if n == self._n:
            return
        s = self.shape
        lib = load()
        dev = self.params.device
        self.Z = torch.empty(int(lib.mlp_act_floats(ctypes.byref(s), n)), dtype=torch.float32,
                             device=dev)
        self.A = torch.empty(max(1, int(lib.mlp_act_bf16(ctypes.byref(s), n))), dtype=torch.bfloat16,
                             device=dev)
        wmax = max(s.width, s.n_out)
        self.work_f = torch.empty(2 * n * wmax, dtype=torch.float32, device=dev)
        self.work_b = torch.empty(n * wmax, dtype=torch.bfloat16, device=dev)
        self.dY = torch.empty(n * s.n_out, dtype=torch.float32, device=dev)
        self.partial = torch.empty(int(lib.mlp_mse_partials(n, s.n_out)), dtype=torch.float32,
                                   device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self._n = n

    def to_bf16(self, x):
        import torch
        x = x.contiguous().to(torch.float32)
        y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
        mlp_to_bf16(x, y)
        return y

    def forward(self, Xb):
        """Xb: bf16 tensor [n, n_in].  Returns the FP32 output view [n, n_out]."""
        n = Xb.shape[0]
        self._buffers(n)
        mlp_forward(self.shape, self.params, self.wb, n, Xb, self.Z, self.A)
        off = n * self.shape.depth * self.shape.width
        return self.Z[off:off + n * self.shape.n_out].view(n, self.shape.n_out)

    def infer(self, Xb):
        """Output only (no pre-activations kept for a backward pass); equal to
        forward's.  Returns the FP32 view [n, n_out]."""
        n = Xb.shape[0]
        self._buffers(n)
        mlp_infer(self.shape, self.params, self.wb, n, Xb, self.Z, self.A)
        off = n * self.shape.depth * self.shape.width
        return self.Z[off:off + n * self.shape.n_out].view(n, self.shape.n_out)

    def infer_fused(self, Xb, out=None):
        """Output of every layer in one fused launch (weights in LDS,
        activations in registers): FP32 tensor [n, n_out], equal to forward's
        to FP32 rounding.  Needs width 128, n_in <= 32, n_out <= 16."""
        import torch
        n = Xb.shape[0]
        Y = out if out is not None else torch.empty((n, self.shape.n_out), dtype=torch.float32,
                                                    device=self.params.device)
        mlp_infer_fused(self.shape, self.params, self.wb, n, Xb, Y)
        return Y

    def backward(self, Xb, dY):
        n = Xb.shape[0]
        mlp_backward(self.shape, self.wb, n, Xb, self.Z, self.A, dY, self.grad, self.work_f,
                     self.work_b)
        return self.grad

    def train_step(self, Xb, T, w=None, lr=1e-3):
        """One Adam step on the weighted MSE; returns the loss tensor [1]."""
        n = Xb.shape[0]
        Y = self.forward(Xb)
        mlp_mse(n, self.shape.n_out, Y, T, w, self.dY, self.loss, self.partial)
        self.backward(Xb, self.dY)
        self.t += 1
        mlp_adam(self.params, self.wb, self.grad, self.m, self.v, lr, self.t)
        return self.loss

    def state(self):
        return self.params.detach().cpu().numpy().astype(np.float64)



def flops_per_site(n_in=16, width=128, depth=4, n_out=4):
    """Multiply-add flops of one forward pass per sample (2 per weight)."""
    dims = [n_in] + [width] * depth + [n_out]
    return 2 * sum(a * b for a, b in zip(dims[:-1], dims[1:]))


def bench(n=7_484_227, reps=10, seed=0):
    """Forward pass, inference pass, fused inference and training step of the default network
    on n samples of random features, timed with HIP events on torch's
    current stream; returns a dict of milliseconds and rates."""
    import torch
    net = Net(seed=seed)
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = net.to_bf16(torch.randn(n, net.shape.n_in, device="cuda", generator=g))
    T = torch.randn(n, net.shape.n_out, device="cuda", generator=g)
    out = dict(samples=n, flop_per_sample=flops_per_site())
    Yf = torch.empty((n, net.shape.n_out), dtype=torch.float32, device="cuda")
    for name, fn in (("forward", lambda: net.forward(X)), ("infer", lambda: net.infer(X)),
                     ("infer_fused", lambda: net.infer_fused(X, Yf)),
                     ("train_step", lambda: net.train_step(X, T, lr=1e-4))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flop = out["flop_per_sample"] * n * (3 if name == "train_step" else 1)
        tflops = flop / (ms * 1e-3) / 1e12
        out[name] = dict(ms=round(ms, 3), tflops=round(tflops, 2),
                         frac_of_bf16_dense_peak=round(tflops / 2500.0, 4))
        print(f"[mlp] {name}: {ms:.3f} ms for {n} samples, {flop / (ms * 1e-3) / 1e12:.1f} TFLOP/s",
              file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="time the warm-start network on one GPU")
    ap.add_argument("--samples", type=int, default=7_484_227)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args()
    print(json.dumps(bench(a.samples, a.reps)), flush=True)
