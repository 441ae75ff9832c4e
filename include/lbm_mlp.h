/*
 * lbm_mlp.h -- C ABI of the warm-start network kernels (gfx950).
 *
 * A small multilayer perceptron maps per-site features of a vessel (wall
 * distance, local radius, position along the segment and the tree,
 * generation, wall stiffness, inlet amplitude, cycle phase) to the density
 * and velocity of the periodic state.  Its output only initialises the
 * lattice Boltzmann populations through lbm_init_fields_device (Sec. 2.1 eq.
 * feq); the update and its boundary rules are unchanged, and a warm-started
 * run must reach the same periodic state as one started from rest.
 *
 * Network: depth hidden layers of `width` units with SiLU, then a linear
 * output layer of n_out units.  GEMM operands are bf16, accumulation and
 * biases FP32.  Parameter vector (FP32 master and bf16 copy share the
 * layout): for each layer l, W_l (out_l x in_l, row-major) then b_l (out_l).
 *
 * Conventions: all pointers are DEVICE pointers allocated by the caller
 * (the Python side uses torch tensors); the library allocates nothing.
 * Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 * default stream).  Functions return 0 on success, -1 for invalid
 * arguments and -3 for a HIP launch failure; mlp_last_error() describes the
 * last failure of the calling thread.  bf16 conversions round to nearest
 * even.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_in, width, depth, n_out;
} mlp_shape;

/* Number of parameters (FP32 master or bf16 copy), or -1. */
int64_t mlp_param_count(const mlp_shape* s);

/* Sizes of the activation buffers for n samples: FP32 pre-activations Z
 * (n * (depth * width + n_out) floats; the network output Y is the last
 * n * n_out block, row-major) and bf16 post-activations A (n * depth *
 * width). */
int64_t mlp_act_floats(const mlp_shape* s, int64_t n);
int64_t mlp_act_bf16(const mlp_shape* s, int64_t n);

/* C[M x N] (or C +=, if accumulate) = op(A) op(B) with op(A)(m,k) =
 * transA ? A[k*lda+m] : A[m*lda+k] and op(B)(k,n) = transB ? B[n*ldb+k] :
 * B[k*ldb+n]; bf16 operands, FP32 C (row-major, ldc).  At most 2^31 - 1
 * output tiles of 64 x 64 (else -1). */
int mlp_gemm_bf16(int M, int N, int K, const uint16_t* A, int lda, int transA, const uint16_t* B,
                  int ldb, int transB, float* C, int ldc, int accumulate, void* stream);

/* Forward pass of n samples X (n x n_in bf16, row-major): fills Z and A
 * (see mlp_act_*).  params: FP32 master (biases are read from it), wb:
 * bf16 copy (GEMM weights).  n < 2^31 and at most 2^31 - 1 tiles of 64 x 64
 * per layer product (else -1). */
int mlp_forward(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
                const uint16_t* X, float* Z, uint16_t* A, void* stream);

/* Inference: as mlp_forward, but only the output Y (the last n * n_out
 * block of Z) and the bf16 activations A are written; the hidden
 * pre-activations are not kept, so no backward pass can follow.  Y is
 * identical to mlp_forward's. */
int mlp_infer(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
              const uint16_t* X, float* Z, uint16_t* A, void* stream);

/* Inference of n samples in one launch: Y (n x n_out FP32, row-major,
 * 16-byte aligned) from X, with every layer fused (weights resident in LDS,
 * activations in registers), so only X and Y touch memory.  Needs width =
 * 128, n_in <= 32, n_out <= 16 and depth <= 5 (else -1; mlp_infer covers
 * other shapes).  Hidden biases enter as the accumulators' initial values
 * and SiLU uses the hardware reciprocal, so Y agrees with mlp_forward's to
 * FP32 rounding (and bf16 rounding of a hidden activation where that
 * differs), not bit for bit. */
int mlp_infer_fused(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
                    const uint16_t* X, float* Y, void* stream);

/* Backward pass for the loss gradient dY (n x n_out FP32) of the forward
 * pass that produced Z and A: writes the gradient of every parameter into
 * grad (FP32, parameter layout).  Workspaces: work_f of
 * 2 * n * max(width, n_out) floats and work_b of n * max(width, n_out)
 * bf16.  The weight and bias gradients are sums over the samples: they are
 * split into sample ranges whose partial sums (held in work_f) are added in
 * a fixed order, so a repeated call gives bit-identical gradients.  Same
 * limits on n as mlp_forward. */
int mlp_backward(const mlp_shape* s, const uint16_t* wb, int64_t n, const uint16_t* X,
                 const float* Z, const uint16_t* A, const float* dY, float* grad, float* work_f,
                 uint16_t* work_b, void* stream);

/* Weighted mean squared error L = sum_ij w_j (Y_ij - T_ij)^2 / (n c) into
 * *loss (device float) and its gradient into dY (may be NULL); w (c
 * floats) may be NULL for unit weights; partial holds
 * mlp_mse_partials(n, c) floats. */
int mlp_mse(int64_t n, int c, const float* Y, const float* T, const float* w, float* dY,
            float* loss, float* partial, void* stream);
int64_t mlp_mse_partials(int64_t n, int c);

/* One Adam step (Kingma & Ba, bias-corrected, step t >= 1) on the FP32
 * master params with first/second moments m, v; refreshes the bf16 copy. */
int mlp_adam(int64_t nparam, float* params, uint16_t* wb, const float* grad, float* m, float* v,
             float lr, float beta1, float beta2, float eps, int64_t t, void* stream);

/* y = bf16(x) for n floats. */
int mlp_to_bf16(int64_t n, const float* x, uint16_t* y, void* stream);

const char* mlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_MLP_H */
