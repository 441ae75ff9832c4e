// Warm-start network kernels for gfx950: bf16 MFMA GEMM with FP32
// accumulation, bias/SiLU epilogues, their backward, MSE loss and Adam.
//
// The network maps per-site geometry and drive features to the density and
// velocity of the periodic state; it only supplies an initial field for the
// lattice Boltzmann update (the update itself is unchanged).
//
// Parameter layout (FP32 master and bf16 copy alike): for each layer l,
// W_l (out_l x in_l, row-major) followed by b_l (out_l).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "../../include/lbm_mlp.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf(float v) {  // round to nearest even
    uint32_t b = __float_as_uint(v);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// C[M x N] (+)= op(A)[M x K] op(B)[K x N]; op(A)(m,k) = transA ? A[k*lda+m]
// : A[m*lda+k]; op(B)(k,n) = transB ? B[n*ldb+k] : B[k*ldb+n].  bf16
// operands, FP32 accumulation and output.  Tile 64 x 64 per 256-thread
// block, K staged through LDS in steps of 32, each wave computing a 32 x 32
// quarter as 2 x 2 MFMA 16x16x32 tiles.
constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;

__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t* __restrict__ A,
                                              int lda, int transA, const uint16_t* __restrict__ B,
                                              int ldb, int transB, float* __restrict__ C, int ldc,
                                              int accumulate) {
    __shared__ __attribute__((aligned(16))) uint16_t As[TM][LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[TN][LDK];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
        // stage A (64 x 32) and B (32 x 64, stored n-major), zero outside
#pragma unroll
        for (int r = 0; r < (TM * TK) / 256; ++r) {
            const int e = t + 256 * r;
            int m, k;
            if (transA) { k = e / TM; m = e % TM; } else { m = e / TK; k = e % TK; }
            const int gm = m0 + m, gk = k0 + k;
            uint16_t v = 0;
            if (gm < M && gk < K) v = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[m][k] = v;
        }
#pragma unroll
        for (int r = 0; r < (TN * TK) / 256; ++r) {
            const int e = t + 256 * r;
            int n, k;
            if (transB) { n = e / TK; k = e % TK; } else { k = e / TN; n = e % TN; }
            const int gn = n0 + n, gk = k0 + k;
            uint16_t v = 0;
            if (gn < N && gk < K) v = transB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
            Bs[n][k] = v;
        }
        __syncthreads();
        const int row = lane & 15, kg = (lane >> 4) * 8;
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = *(const bf16x8*)&As[wm + 16 * a + row][kg];
#pragma unroll
        for (int b = 0; b < 2; ++b) bfr[b] = *(const bf16x8*)&Bs[wn + 16 * b + row][kg];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // lane holds rows 4*(lane/16) + r of column lane % 16 of each 16x16 tile
    const int col = lane & 15, rg = (lane >> 4) * 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * a + rg + r, gn = n0 + wn + 16 * b + col;
                if (gm < M && gn < N) {
                    float* p = C + (int64_t)gm * ldc + gn;
                    *p = accumulate ? *p + acc[a][b][r] : acc[a][b][r];
                }
            }
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Z[n x c] += b; act: A = bf16(silu(Z)) (Z kept as the pre-activation),
// else Y = Z (output layer).
__global__ void k_bias_act(int64_t n, int c, float* __restrict__ Z, const float* __restrict__ bias,
                           uint16_t* __restrict__ Aout, int act) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * c) return;
    const float z = Z[e] + bias[e % c];
    Z[e] = z;
    if (act) Aout[e] = f2bf(silu(z));
}

// dZ = dA * silu'(Zpre) (bf16 for the next GEMM, FP32 copy for the bias
// gradient); dA is FP32.
__global__ void k_act_bwd(int64_t n, int c, const float* __restrict__ dA,
                          const float* __restrict__ Zpre, float* __restrict__ dZf,
                          uint16_t* __restrict__ dZb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * c) return;
    const float g = dA[e] * dsilu(Zpre[e]);
    dZf[e] = g;
    dZb[e] = f2bf(g);
}

__global__ void k_f32_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] = f2bf(x[e]);
}

// db[j] (+)= sum_i dZ[i][j]: one block per column group, strided rows.
__global__ __launch_bounds__(256) void k_colsum(int64_t n, int c, const float* __restrict__ dZ,
                                                float* __restrict__ db) {
    __shared__ float red[256];
    const int j = blockIdx.x;
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += dZ[i * c + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[j] = red[0];
}

// Mean squared error over n x c entries with per-column weights:
// L = sum_ij w_j (Y - T)^2 / (n c); dY = 2 w_j (Y - T) / (n c).  The loss is
// accumulated per block and summed by the host-side launcher's second pass.
__global__ __launch_bounds__(256) void k_mse(int64_t n, int c, const float* __restrict__ Y,
                                             const float* __restrict__ T,
                                             const float* __restrict__ w, float* __restrict__ dY,
                                             float* __restrict__ partial) {
    __shared__ float red[256];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (e < n * c) {
        const float inv = 1.0f / (float)(n * c);
        const float wj = w ? w[e % c] : 1.0f;
        const float d = Y[e] - T[e];
        l = wj * d * d * inv;
        if (dY) dY[e] = 2.0f * wj * d * inv;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(int n, const float* __restrict__ x, float* __restrict__ out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Adam (Kingma & Ba) on the FP32 master weights, refreshing the bf16 copy.
__global__ void k_adam(int64_t n, float* __restrict__ p, uint16_t* __restrict__ pb,
                       const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    p[e] = pe;
    pb[e] = f2bf(pe);
}

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


struct Dims {
    int L;            // layers
    int in[8], out[8];
    int64_t woff[8], boff[8];
};

Dims dims(const mlp_shape* s) {
    Dims d{};
    d.L = s->depth + 1;
    int64_t off = 0;
    for (int l = 0; l < d.L; ++l) {
        d.in[l] = l == 0 ? s->n_in : s->width;
        d.out[l] = l == d.L - 1 ? s->n_out : s->width;
        d.woff[l] = off;
        off += (int64_t)d.in[l] * d.out[l];
        d.boff[l] = off;
        off += d.out[l];
    }
    return d;
}

bool valid(const mlp_shape* s) {
    return s && s->n_in > 0 && s->width > 0 && s->n_out > 0 && s->depth >= 1 && s->depth <= 6;
}

thread_local char g_err[256] = "";

int err(const char* m) {
    std::strncpy(g_err, m, sizeof(g_err) - 1);
    return -1;
}

int check(hipError_t e) {
    if (e == hipSuccess) return 0;
    std::strncpy(g_err, hipGetErrorString(e), sizeof(g_err) - 1);
    return -3;
}

}  // namespace

extern "C" {

const char* mlp_last_error(void) { return g_err; }

int64_t mlp_param_count(const mlp_shape* s) {
    if (!valid(s)) return -1;
    const Dims d = dims(s);
    return d.boff[d.L - 1] + d.out[d.L - 1];
}

int64_t mlp_act_floats(const mlp_shape* s, int64_t n) {
    if (!valid(s) || n < 0) return -1;
    return n * ((int64_t)s->depth * s->width + s->n_out);
}

int64_t mlp_act_bf16(const mlp_shape* s, int64_t n) {
    if (!valid(s) || n < 0) return -1;
    return n * (int64_t)s->depth * s->width;
}

int mlp_gemm_bf16(int M, int N, int K, const uint16_t* A, int lda, int transA, const uint16_t* B,
                  int ldb, int transB, float* C, int ldc, int accumulate, void* stream) {
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return err("mlp_gemm_bf16: bad arguments");
    if (M == 0 || N == 0) return 0;
    dim3 grid(nb(M, TM), nb(N, TN));
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, (hipStream_t)stream, M, N, K, A, lda, transA, B,
                       ldb, transB, C, ldc, accumulate);
    return check(hipGetLastError());
}

int mlp_forward(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
                const uint16_t* X, float* Z, uint16_t* A, void* stream) {
    if (!valid(s) || !params || !wb || !X || !Z || !A || n < 0)
        return err("mlp_forward: bad arguments");
    if (n == 0) return 0;
    if (n > INT32_MAX) return err("mlp_forward: at most 2^31-1 samples per call");
    const Dims d = dims(s);
    hipStream_t st = (hipStream_t)stream;
    const uint16_t* x = X;
    for (int l = 0; l < d.L; ++l) {
        const bool last = l == d.L - 1;
        float* Zl = Z + (int64_t)l * n * s->width;
        int rc = mlp_gemm_bf16((int)n, d.out[l], d.in[l], x, d.in[l], 0, wb + d.woff[l], d.in[l], 1,
                               Zl, d.out[l], 0, stream);
        if (rc) return rc;
        uint16_t* Al = last ? nullptr : A + (int64_t)l * n * s->width;
        hipLaunchKernelGGL(k_bias_act, dim3(nb(n * d.out[l], 256)), dim3(256), 0, st, n, d.out[l], Zl,
                           params + d.boff[l], Al, last ? 0 : 1);
        rc = check(hipGetLastError());
        if (rc) return rc;
        x = Al;
    }
    return 0;
}

int mlp_backward(const mlp_shape* s, const uint16_t* wb, int64_t n, const uint16_t* X,
                 const float* Z, const uint16_t* A, const float* dY, float* grad, float* work_f,
                 uint16_t* work_b, void* stream) {
    if (!valid(s) || !wb || !X || !Z || !A || !dY || !grad || !work_f || !work_b || n <= 0)
        return err("mlp_backward: bad arguments");
    if (n > INT32_MAX) return err("mlp_backward: at most 2^31-1 samples per call");
    const Dims d = dims(s);
    hipStream_t st = (hipStream_t)stream;
    const int L = d.L;
    const int64_t wmax = s->width > s->n_out ? s->width : s->n_out;
    float* dA = work_f;                 // n x width
    float* dZf = work_f + n * wmax;     // n x max(width, n_out)
    int rc = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int out = d.out[l], in = d.in[l];
        if (l == L - 1) {
            rc = check(hipMemcpyAsync(dZf, dY, sizeof(float) * n * out, hipMemcpyDeviceToDevice, st));
            if (rc) return rc;
            hipLaunchKernelGGL(k_f32_to_bf16, dim3(nb(n * out, 256)), dim3(256), 0, st, n * out, dZf,
                               work_b);
        } else {
            hipLaunchKernelGGL(k_act_bwd, dim3(nb(n * out, 256)), dim3(256), 0, st, n, out, dA,
                               Z + (int64_t)l * n * s->width, dZf, work_b);
        }
        rc = check(hipGetLastError());
        if (rc) return rc;
        const uint16_t* prev = l == 0 ? X : A + (int64_t)(l - 1) * n * s->width;
        // dW_l = dZ_l^T prev  (out x in), db_l = column sums of dZ_l
        rc = mlp_gemm_bf16(out, in, (int)n, work_b, out, 1, prev, in, 0, grad + d.woff[l], in, 0, stream);
        if (rc) return rc;
        hipLaunchKernelGGL(k_colsum, dim3(out), dim3(256), 0, st, n, out, dZf, grad + d.boff[l]);
        rc = check(hipGetLastError());
        if (rc) return rc;
        // dA_{l-1} = dZ_l W_l  (n x in)
        if (l > 0) {
            rc = mlp_gemm_bf16((int)n, in, out, work_b, out, 0, wb + d.woff[l], in, 0, dA, in, 0, stream);
            if (rc) return rc;
        }
    }
    return 0;
}

int mlp_mse(int64_t n, int c, const float* Y, const float* T, const float* w, float* dY,
            float* loss, float* partial, void* stream) {
    if (n <= 0 || c <= 0 || !Y || !T || !loss || !partial) return err("mlp_mse: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const unsigned blocks = nb(n * c, 256);
    hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, st, n, c, Y, T, w, dY, partial);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, (int)blocks, partial, loss);
    return check(hipGetLastError());
}

int64_t mlp_mse_partials(int64_t n, int c) { return (n * c + 255) / 256; }

int mlp_adam(int64_t nparam, float* params, uint16_t* wb, const float* grad, float* m, float* v,
             float lr, float beta1, float beta2, float eps, int64_t t, void* stream) {
    if (nparam <= 0 || !params || !wb || !grad || !m || !v || t < 1) return err("mlp_adam: bad arguments");
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(nb(nparam, 256)), dim3(256), 0, (hipStream_t)stream, nparam, params,
                       wb, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return check(hipGetLastError());
}

int mlp_to_bf16(int64_t n, const float* x, uint16_t* y, void* stream) {
    if (n < 0 || !x || !y) return err("mlp_to_bf16: bad arguments");
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(nb(n, 256)), dim3(256), 0, (hipStream_t)stream, n, x, y);
    return check(hipGetLastError());
}

}  // extern "C"
