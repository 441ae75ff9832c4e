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

#include <algorithm>
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

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// C[M x N] (+)= op(A)[M x K] op(B)[K x N]; op(A)(m,k) = transA ? A[k*lda+m]
// : A[m*lda+k]; op(B)(k,n) = transB ? B[n*ldb+k] : B[k*ldb+n].  bf16
// operands, FP32 accumulation and output.  Tile 64 x 64 per 256-thread
// block, K staged through LDS in steps of 32, each wave computing a 32 x 32
// quarter as 2 x 2 MFMA 16x16x32 tiles.  Split K: block z covers
// k in [z kchunk, (z + 1) kchunk) and writes slab z of C (M ldc floats
// each); with one slab this is the plain product.
constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8, LDC = TN + 4;
static_assert(2 * 64 * LDK * 2 <= TM * LDC * 4, "operand tiles fit in the output tile");

// Staging of the 64 x 32 tile T[r][k] = src(r0 + r, k0 + k), with
// src(r, k) = kmajor ? S[k ld + r] : S[r ld + k] and zeros outside r < R,
// k < ke: each thread loads 8 elements into registers (load_frag) and later
// writes them into LDS (store_frag), so the next tile's loads are in flight
// while the current one is multiplied.  With vec (16-byte aligned rows,
// checked by the caller) the 8 elements are consecutive in memory: 8 values
// of k of one r, or (kmajor) 8 values of r of one k; otherwise element q of
// thread t is tile element t + 256 q.
union Frag {
    uint4 v;
    uint16_t h[8];
};

// LDS tiles hold row r's group of 8 k values g at group g ^ (r / 8 mod 4):
// a thread that writes 8 rows of one k (k-major operands) then spreads over
// 4 bank groups instead of one, and a group of 8 k stays 16-byte aligned
// for the MFMA operand reads.
__device__ __forceinline__ int swz(int r) { return ((r >> 3) & 3) << 3; }

template <bool kmajor>
__device__ __forceinline__ void frag_pos(bool vec, int t, int q, int& r, int& k) {
    if (vec && !kmajor) {
        r = t >> 2;
        k = (t & 3) * 8 + q;
    } else if (vec) {
        r = (t & 7) * 8 + q;
        k = t >> 3;
    } else {
        const int e = t + 256 * q;
        r = kmajor ? e % 64 : e / TK;
        k = kmajor ? e / 64 : e % TK;
    }
}

template <bool kmajor>
__device__ __forceinline__ Frag load_frag(const uint16_t* __restrict__ S, int ld, int r0, int R,
                                          int k0, int ke, bool vec, int t) {
    Frag f;
    if (vec) {
        int r, k;
        frag_pos<kmajor>(true, t, 0, r, k);
        const int gr = r0 + r, gk = k0 + k;
        const bool whole = kmajor ? (gk < ke && gr + 8 <= R) : (gr < R && gk + 8 <= ke);
        if (whole) {
            f.v = kmajor ? *(const uint4*)(S + (int64_t)gk * ld + gr)
                         : *(const uint4*)(S + (int64_t)gr * ld + gk);
            return f;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int r, k;
        frag_pos<kmajor>(vec, t, q, r, k);
        const int gr = r0 + r, gk = k0 + k;
        f.h[q] = (gr < R && gk < ke) ? (kmajor ? S[(int64_t)gk * ld + gr] : S[(int64_t)gr * ld + gk])
                                     : (uint16_t)0;
    }
    return f;
}

template <bool kmajor>
__device__ __forceinline__ void store_frag(uint16_t (&T)[64][LDK], const Frag& f, bool vec, int t) {
    if (vec && !kmajor) {
        const int r = t >> 2;
        *(uint4*)&T[r][((t & 3) * 8) ^ swz(r)] = f.v;
        return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        int r, k;
        frag_pos<kmajor>(vec, t, q, r, k);
        T[r][k ^ swz(r)] = f.h[q];
    }
}

// Workgroups are handed to the 8 XCDs in turn, each XCD with its own L2:
// block b of nblk takes id j per + min(j, rem) + k (j = b mod 8, k = b / 8),
// so each XCD works through a contiguous range of ids (a bijection).
__device__ __forceinline__ int xcd_order(int b, int nblk) {
    const int per = nblk >> 3, rem = nblk & 7;
    const int j = b & 7, k = b >> 3;
    return j * per + (j < rem ? j : rem) + k;
}

// Epilogue (bias != null): C = acc + bias[n] and, when Aout != null,
// Aout = bf16(silu(C)) at the same index (the fused bias and activation of a
// forward layer).  C == null (no accumulate, one slab): only Aout is
// written, for inference without the pre-activations.  One instantiation per operand layout, so each carries only
// the staging it uses.
template <int transA, int transB, bool va, bool vb>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const uint16_t* __restrict__ A,
                                              int lda, const uint16_t* __restrict__ B, int ldb,
                                              float* __restrict__ C, int ldc,
                                              int accumulate, int kchunk,
                                              const float* __restrict__ bias,
                                              uint16_t* __restrict__ Aout) {
    // operand tiles during the K loop, then the output tile (row stride LDC
    // floats) for the epilogue's row-wise stores
    __shared__ __attribute__((aligned(16))) float smem[TM * LDC];
    uint16_t (&As)[TM][LDK] = *reinterpret_cast<uint16_t (*)[TM][LDK]>(smem);
    uint16_t (&Bs)[TN][LDK] = *reinterpret_cast<uint16_t (*)[TN][LDK]>(
        reinterpret_cast<uint16_t*>(smem) + TM * LDK);
    float (&Cs)[TM][LDC] = *reinterpret_cast<float (*)[TM][LDC]>(smem);
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    // (slab, tile) ids in XCD order, tiles in order of n within m: the tiles
    // that share a row strip of op(A), and the tiles of one slab, run on one
    // XCD close together, so a strip is read from HBM once
    const int ntn = (N + TN - 1) / TN, nx = (int)gridDim.x;
    const int id = xcd_order((int)blockIdx.x + nx * (int)blockIdx.z, nx * (int)gridDim.z);
    const int tile = id % nx, zb = id / nx;
    const int m0 = (tile / ntn) * TM, n0 = (tile % ntn) * TN;
    const int64_t kz = (int64_t)zb * kchunk;
    const int kb = (int)kz, ke = (int)(kz + kchunk < K ? kz + kchunk : K);
    if (C) C += (int64_t)zb * M * ldc;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // A (64 x 32) and B (32 x 64, stored n-major) tiles, zero outside; the
    // next pair is loaded while the current one is multiplied
    constexpr bool ka = transA != 0, kbm = transB == 0;
    Frag fa = load_frag<ka>(A, lda, m0, M, kb, ke, va, t);
    Frag fb = load_frag<kbm>(B, ldb, n0, N, kb, ke, vb, t);
    for (int k0 = kb; k0 < ke; k0 += TK) {
        store_frag<ka>(As, fa, va, t);
        store_frag<kbm>(Bs, fb, vb, t);
        __syncthreads();
        if (k0 + TK < ke) {
            fa = load_frag<ka>(A, lda, m0, M, k0 + TK, ke, va, t);
            fb = load_frag<kbm>(B, ldb, n0, N, k0 + TK, ke, vb, t);
        }
        const int row = lane & 15, kg = (lane >> 4) * 8;
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int m = wm + 16 * a + row;
            af[a] = *(const bf16x8*)&As[m][kg ^ swz(m)];
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int n = wn + 16 * b + row;
            bfr[b] = *(const bf16x8*)&Bs[n][kg ^ swz(n)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // lane holds rows 4*(lane/16) + r of column lane % 16 of each 16x16
    // tile; the tile goes through LDS (the K loop ended with a barrier, so
    // the operand tiles are dead) and leaves row by row: in each of 4 passes
    // 16 consecutive threads write one whole row of the tile with 16-byte
    // stores (4 columns each), so every store fills whole lines
    const int col = lane & 15, rg = (lane >> 4) * 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) Cs[wm + 16 * a + rg + r][wn + 16 * b + col] = acc[a][b][r];
    __syncthreads();
    const bool vc = (!C || ((((uintptr_t)C & 15) == 0) && ((ldc & 3) == 0))) &&
                    (!Aout || ((((uintptr_t)Aout & 7) == 0) && ((ldc & 3) == 0)));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = (t >> 4) + 16 * j, c = (t & 15) * 4;
        const int gm = m0 + row, gn = n0 + c;
        if (gm >= M) break;
        const float4 q = *(const float4*)&Cs[row][c];
        float v[4] = {q.x, q.y, q.z, q.w};
        const int64_t e = (int64_t)gm * ldc + gn;
        if (vc && gn + 4 <= N) {
            if (accumulate) {
                const float4 o = *(const float4*)(C + e);
                v[0] = o.x + v[0];
                v[1] = o.y + v[1];
                v[2] = o.z + v[2];
                v[3] = o.w + v[3];
            }
            if (bias) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] += bias[gn + u];
            }
            if (C) *(float4*)(C + e) = make_float4(v[0], v[1], v[2], v[3]);
            if (Aout) {
                const uint32_t lo = (uint32_t)f2bf(silu(v[0])) | ((uint32_t)f2bf(silu(v[1])) << 16);
                const uint32_t hi = (uint32_t)f2bf(silu(v[2])) | ((uint32_t)f2bf(silu(v[3])) << 16);
                *(uint2*)(Aout + e) = make_uint2(lo, hi);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (gn + u >= N) break;
                float x = accumulate ? C[e + u] + v[u] : v[u];
                if (bias) x += bias[gn + u];
                if (C) C[e + u] = x;
                if (Aout) Aout[e + u] = f2bf(silu(x));
            }
        }
    }
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

// The same dZ as bf16 only, with its column sums over rows
// [b rows, (b + 1) rows) into part[b c + j] (block b), added in the order of
// k_colsum_part, so the bias gradient needs no FP32 copy of dZ.
__global__ __launch_bounds__(256) void k_act_bwd_colsum(int64_t n, int c, int64_t rows,
                                                        const float* __restrict__ dA,
                                                        const float* __restrict__ Zpre,
                                                        uint16_t* __restrict__ dZb,
                                                        float* __restrict__ part) {
    __shared__ float red[256];
    const int t = threadIdx.x, per = 256 / c;
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(n, r0 + rows);
    float s = 0.f;
    if (t < per * c) {
        const int j = t % c;
        for (int64_t i = r0 + t / c; i < r1; i += per) {
            const int64_t e = i * c + j;
            const float g = dA[e] * dsilu(Zpre[e]);
            dZb[e] = f2bf(g);
            s += g;
        }
    }
    red[t] = s;
    __syncthreads();
    if (t < c) {
        float a = 0.f;
        for (int q = 0; q < per; ++q) a += red[q * c + t];
        part[(int64_t)blockIdx.x * c + t] = a;
    }
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

// Column sums of rows [b rows, (b + 1) rows) of dZ [n x c] into part[b c + j]
// (block b).  Thread t sums column t % c over every (256 / c)-th row of the
// range; the partial sums of a column are then added in thread order.
__global__ __launch_bounds__(256) void k_colsum_part(int64_t n, int c, int64_t rows,
                                                     const float* __restrict__ dZ,
                                                     float* __restrict__ part) {
    __shared__ float red[256];
    const int t = threadIdx.x, per = 256 / c;
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(n, r0 + rows);
    float s = 0.f;
    if (t < per * c) {
        const int j = t % c;
        for (int64_t i = r0 + t / c; i < r1; i += per) s += dZ[i * c + j];
    }
    red[t] = s;
    __syncthreads();
    if (t < c) {
        float a = 0.f;
        for (int q = 0; q < per; ++q) a += red[q * c + t];
        part[(int64_t)blockIdx.x * c + t] = a;
    }
}

// out[e] = sum over z < S of part[z count + e], in order of z.
__global__ void k_reduce_slabs(int S, int64_t count, const float* __restrict__ part,
                               float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float a = 0.f;
    for (int z = 0; z < S; ++z) a += part[(int64_t)z * count + e];
    out[e] = a;
}

// out[j] = sum over z < S of part[z count + j] for few columns: block j,
// thread t adds z = t, t + 256, ..., and the 256 partial sums meet in a fixed
// tree (the order does not depend on scheduling).
__global__ __launch_bounds__(256) void k_reduce_cols(int S, int count,
                                                     const float* __restrict__ part,
                                                     float* __restrict__ out) {
    __shared__ float red[256];
    const int j = blockIdx.x, t = threadIdx.x;
    float a = 0.f;
    for (int z = t; z < S; z += 256) a += part[(int64_t)z * count + j];
    red[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[j] = red[0];
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

// ---------------------------------------------------------------------------
// Fused inference: every layer of one network in one kernel.  The bf16
// weights (about 108 KB for 16 -> 128 x 4 -> 4) stay in LDS for the whole
// launch and the activations never leave registers, so HBM sees only the
// features in and the outputs out (32 + 16 bytes per sample).
//
// Each layer is computed transposed, out^T (out x S) = W (out x in) in^T
// (in x S), with MFMA 16x16x32 bf16: A = a 16 x 32 block of W (read from
// LDS, stored there in operand order so that lane l's 16 bytes are at
// l * 16 of a 1 KB block), B = a 32 x 16 block of in^T (16 samples), D = a
// 16 x 16 block of out^T.  Lane l holds D rows 4 (l / 16) + 0..3 (four
// output features) of column l % 16 (one sample), and the next layer's B
// operand wants rows 8 (l / 16) + 0..7 of the same column: after the
// epilogue (bias, SiLU, bf16 pairs) two output tiles become one K tile of
// the next layer through two lane swaps across 32- and 16-lane halves
// (v_permlane32_swap, v_permlane16_swap), with no LDS round trip.
namespace fused {
constexpr int W = 128;            // hidden width
constexpr int NT = W / 16;        // output tiles of a hidden layer
constexpr int NK = W / 32;        // K tiles of a hidden layer
constexpr int J = 4;              // 16-sample tiles per wave and step
constexpr int THREADS = 512;
constexpr int MAX_DEPTH = 5;

template <int DEPTH>
struct Lds {
    // operand blocks: layer 0 (NT x 1), hidden layers (NT x NK each), head (1 x NK)
    uint4 w[(NT + (DEPTH - 1) * NT * NK + NK) * 64];
    float bias[DEPTH * W + 16];
};

__device__ __forceinline__ int block_of(int layer, int o, int k) {
    return layer == 0 ? o : NT + (layer - 1) * NT * NK + o * NK + k;
}

// silu(z) = z / (1 + e^-z) with the hardware reciprocal (1 ulp)
__device__ __forceinline__ float silu_fast(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned pack_bf16(float x, float y) {  // round to nearest even
    const f32x2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// Two output tiles (h = 0, 1) of one 16-sample tile, after bias and SiLU,
// as the next layer's B operand: components {a, b} of the first and the
// second source row group.
__device__ __forceinline__ bf16x8 to_operand(const f32x4& d0, const f32x4& d1) {
    const unsigned a0 = pack_bf16(silu_fast(d0[0]), silu_fast(d0[1]));
    const unsigned b0 = pack_bf16(silu_fast(d0[2]), silu_fast(d0[3]));
    const unsigned a1 = pack_bf16(silu_fast(d1[0]), silu_fast(d1[1]));
    const unsigned b1 = pack_bf16(silu_fast(d1[2]), silu_fast(d1[3]));
    const auto ra = __builtin_amdgcn_permlane32_swap(a0, a1, false, false);
    const auto qa = __builtin_amdgcn_permlane16_swap(ra[0], ra[1], false, false);
    const auto rb = __builtin_amdgcn_permlane32_swap(b0, b1, false, false);
    const auto qb = __builtin_amdgcn_permlane16_swap(rb[0], rb[1], false, false);
    const u32x4 v = {(unsigned)qa[0], (unsigned)qb[0], (unsigned)qa[1], (unsigned)qb[1]};
    return __builtin_bit_cast(bf16x8, v);
}

template <int DEPTH>
__global__ __launch_bounds__(THREADS) void k_mlp_fused(int64_t n, int n_in, int n_out,
                                                       const uint16_t* __restrict__ wb,
                                                       const float* __restrict__ params,
                                                       const uint16_t* __restrict__ X,
                                                       float* __restrict__ Y, int vec_x) {
    __shared__ Lds<DEPTH> L;
    const int t = threadIdx.x;
    // ---- weights and biases into LDS, in operand order, zero padded
    constexpr int NBLK = NT + (DEPTH - 1) * NT * NK + NK;
    for (int c = t; c < NBLK * 64; c += THREADS) {
        const int blk = c >> 6, lane = c & 63;
        int layer, o, k;
        if (blk < NT) {
            layer = 0; o = blk; k = 0;
        } else if (blk < NT + (DEPTH - 1) * NT * NK) {
            const int b = blk - NT;
            layer = 1 + b / (NT * NK); o = (b % (NT * NK)) / NK; k = b % NK;
        } else {
            layer = DEPTH; o = 0; k = blk - NT - (DEPTH - 1) * NT * NK;
        }
        const int in = layer == 0 ? n_in : W, out = layer == DEPTH ? n_out : W;
        int64_t off = 0;   // W_layer offset in the parameter layout
        for (int q = 0; q < layer; ++q) {
            const int iq = q == 0 ? n_in : W;
            off += (int64_t)iq * W + W;
        }
        const int r = 16 * o + (lane & 15), k0 = 32 * k + 8 * (lane >> 4);
        union { uint4 v; uint16_t h[8]; } u;
        u.v = make_uint4(0u, 0u, 0u, 0u);
        if (r < out) {
            const uint16_t* src = wb + off + (int64_t)r * in + k0;
            if (k0 + 8 <= in && ((uintptr_t)src & 15) == 0) {
                u.v = *(const uint4*)src;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (k0 + q < in) u.h[q] = src[q];
            }
        }
        L.w[c] = u.v;
    }
    for (int c = t; c < DEPTH * W + 16; c += THREADS) {
        const int layer = c < DEPTH * W ? c / W : DEPTH, j = c < DEPTH * W ? c % W : c - DEPTH * W;
        const int out = layer == DEPTH ? n_out : W;
        int64_t off = 0;   // b_layer offset: W_0 b_0 ... W_layer
        for (int q = 0; q < layer; ++q) off += (int64_t)(q == 0 ? n_in : W) * W + W;
        off += (int64_t)(layer == 0 ? n_in : W) * out;
        L.bias[c] = j < out ? params[off + j] : 0.0f;
    }
    __syncthreads();

    const int wave = t >> 6, lane = t & 63, g = lane >> 4, li = lane & 15;
    const int64_t nwaves = (int64_t)gridDim.x * (THREADS / 64);
    for (int64_t grp = (int64_t)blockIdx.x * (THREADS / 64) + wave; grp * (16 * J) < n;
         grp += nwaves) {
        const int64_t s0 = grp * (16 * J);
        bf16x8 B[NK][J];
        // ---- layer 0: features k = 8 g + 0..7 of sample s0 + 16 j + li (K padded to 32)
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t sm = s0 + 16 * j + li;
            union { uint4 v; uint16_t h[8]; } u;
            u.v = make_uint4(0u, 0u, 0u, 0u);
            if (sm < n && 8 * g < n_in) {
                const uint16_t* src = X + sm * n_in + 8 * g;
                if (vec_x && 8 * g + 8 <= n_in) {
                    u.v = *(const uint4*)src;
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (8 * g + q < n_in) u.h[q] = src[q];
                }
            }
            B[0][j] = __builtin_bit_cast(bf16x8, u.v);
        }
        bf16x8 Bn[NK][J];
#pragma unroll
        for (int p = 0; p < NK; ++p) {
            f32x4 acc[2][J];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 b4 = *(const float4*)&L.bias[16 * (2 * p + h) + 4 * g];
                const bf16x8 A = __builtin_bit_cast(bf16x8, L.w[block_of(0, 2 * p + h, 0) * 64 + lane]);
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    acc[h][j] = f32x4{b4.x, b4.y, b4.z, b4.w};
                    acc[h][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[0][j], acc[h][j], 0, 0, 0);
                }
            }
#pragma unroll
            for (int j = 0; j < J; ++j) Bn[p][j] = to_operand(acc[0][j], acc[1][j]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // ---- hidden layers
#pragma unroll
        for (int l = 1; l < DEPTH; ++l) {
#pragma unroll
            for (int p = 0; p < NK; ++p)
#pragma unroll
                for (int j = 0; j < J; ++j) B[p][j] = Bn[p][j];
#pragma unroll
            for (int p = 0; p < NK; ++p) {
                f32x4 acc[2][J];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float4 b4 = *(const float4*)&L.bias[l * W + 16 * (2 * p + h) + 4 * g];
#pragma unroll
                    for (int j = 0; j < J; ++j) acc[h][j] = f32x4{b4.x, b4.y, b4.z, b4.w};
                }
#pragma unroll
                for (int k = 0; k < NK; ++k)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const bf16x8 A =
                            __builtin_bit_cast(bf16x8, L.w[block_of(l, 2 * p + h, k) * 64 + lane]);
#pragma unroll
                        for (int j = 0; j < J; ++j)
                            acc[h][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B[k][j], acc[h][j], 0, 0, 0);
                    }
#pragma unroll
                for (int j = 0; j < J; ++j) Bn[p][j] = to_operand(acc[0][j], acc[1][j]);
                // keep the scheduler from hoisting the next pair's operand
                // reads over this one (they would all be live at once)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // ---- output layer (n_out <= 16 outputs in one tile, no activation)
        f32x4 y[J];
        {
            const float4 b4 = *(const float4*)&L.bias[DEPTH * W + 4 * g];
#pragma unroll
            for (int j = 0; j < J; ++j) y[j] = f32x4{b4.x, b4.y, b4.z, b4.w};
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const bf16x8 A = __builtin_bit_cast(bf16x8, L.w[(NT + (DEPTH - 1) * NT * NK + k) * 64 + lane]);
#pragma unroll
                for (int j = 0; j < J; ++j)
                    y[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bn[k][j], y[j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int64_t sm = s0 + 16 * j + li;
            if (sm >= n) continue;
            if (n_out == 4) {
                if (g == 0) *(float4*)(Y + sm * 4) = make_float4(y[j][0], y[j][1], y[j][2], y[j][3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * g + q < n_out) Y[sm * n_out + 4 * g + q] = y[j][q];
            }
        }
    }
}
}  // namespace fused

inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// blocks of k_gemm for an M x N product (one per 64 x 64 tile)
inline unsigned tiles(int M, int N) { return nb(M, TM) * nb(N, TN); }


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

// every product of a pass over n samples has at most 2^31 - 1 tiles
bool tiles_fit(const mlp_shape* s, int64_t n) {
    const int w = std::max(s->width, std::max(s->n_in, s->n_out));
    return (int64_t)nb(n, TM) * nb(w, TN) <= INT32_MAX;
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

// 16-byte operand staging needs 16-byte aligned rows
bool vec_ok(const void* p, int ld) { return (((uintptr_t)p & 15) == 0) && ((ld & 7) == 0); }

template <int TA, int TB>
void launch_gemm(dim3 grid, hipStream_t st, int M, int N, int K, const uint16_t* A, int lda,
                 const uint16_t* B, int ldb, float* C, int ldc, int accumulate, int kchunk,
                 const float* bias, uint16_t* Aout) {
    const bool va = vec_ok(A, lda), vb = vec_ok(B, ldb);
    if (va && vb)
        hipLaunchKernelGGL((k_gemm<TA, TB, true, true>), grid, dim3(256), 0, st, M, N, K, A, lda,
                           B, ldb, C, ldc, accumulate, kchunk, bias, Aout);
    else if (va)
        hipLaunchKernelGGL((k_gemm<TA, TB, true, false>), grid, dim3(256), 0, st, M, N, K, A, lda,
                           B, ldb, C, ldc, accumulate, kchunk, bias, Aout);
    else if (vb)
        hipLaunchKernelGGL((k_gemm<TA, TB, false, true>), grid, dim3(256), 0, st, M, N, K, A, lda,
                           B, ldb, C, ldc, accumulate, kchunk, bias, Aout);
    else
        hipLaunchKernelGGL((k_gemm<TA, TB, false, false>), grid, dim3(256), 0, st, M, N, K, A, lda,
                           B, ldb, C, ldc, accumulate, kchunk, bias, Aout);
}

// Weight gradient C [M x N] = A^T B over K samples (A: K x M, B: K x N, bf16
// row-major).  Its output is only M x N, so the K range is split over up to
// 512 blocks of z, whose slabs (in work, work_floats floats) are then added
// in slab order: the result does not depend on scheduling.  Few samples take
// the plain product.
int gemm_tn_split(int M, int N, int64_t K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                  float* C, float* work, int64_t work_floats, hipStream_t st) {
    const int64_t slab = (int64_t)M * N;
    int64_t S = std::min<int64_t>(512, K / 8192);
    S = std::min<int64_t>(S, work_floats / slab);
    if (S <= 1) {
        launch_gemm<1, 0>(dim3(tiles(M, N)), st, M, N, (int)K, A, lda, B, ldb, C, N, 0, (int)K,
                          nullptr, nullptr);
        return check(hipGetLastError());
    }
    const int64_t kc = ((K + S - 1) / S + TK - 1) / TK * TK;
    S = (K + kc - 1) / kc;
    launch_gemm<1, 0>(dim3(tiles(M, N), 1, (unsigned)S), st, M, N, (int)K, A, lda, B, ldb, work, N,
                      0, (int)kc, nullptr, nullptr);
    hipLaunchKernelGGL(k_reduce_slabs, dim3(nb(slab, 256)), dim3(256), 0, st, (int)S, slab, work, C);
    return check(hipGetLastError());
}

// Up to 4096 row ranges of n rows for column sums of c columns whose
// partial sums fit in work_floats: B ranges of `rows` rows each.
void row_ranges(int64_t n, int c, int64_t work_floats, int64_t& B, int64_t& rows) {
    B = std::min<int64_t>(4096, (n + 1023) / 1024);
    B = std::max<int64_t>(1, std::min<int64_t>(B, work_floats / c));
    rows = (n + B - 1) / B;
    B = (n + rows - 1) / rows;
}

// Column sums of dZ [n x c] into db over up to 4096 row ranges, whose
// partial sums (in work) are added in range order.
int colsum_split(int64_t n, int c, const float* dZ, float* db, float* work, int64_t work_floats,
                 hipStream_t st) {
    if (c > 256) {
        hipLaunchKernelGGL(k_colsum, dim3(c), dim3(256), 0, st, n, c, dZ, db);
        return check(hipGetLastError());
    }
    int64_t B, rows;
    row_ranges(n, c, work_floats, B, rows);
    hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)B), dim3(256), 0, st, n, c, rows, dZ, work);
    hipLaunchKernelGGL(k_reduce_cols, dim3(c), dim3(256), 0, st, (int)B, c, work, db);
    return check(hipGetLastError());
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
    if ((int64_t)nb(M, TM) * nb(N, TN) > INT32_MAX) return err("mlp_gemm_bf16: too many tiles");
    dim3 grid(tiles(M, N));
    hipStream_t st = (hipStream_t)stream;
    if (transA && transB)
        launch_gemm<1, 1>(grid, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate, K, nullptr, nullptr);
    else if (transA)
        launch_gemm<1, 0>(grid, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate, K, nullptr, nullptr);
    else if (transB)
        launch_gemm<0, 1>(grid, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate, K, nullptr, nullptr);
    else
        launch_gemm<0, 0>(grid, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate, K, nullptr, nullptr);
    return check(hipGetLastError());
}

int mlp_forward(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
                const uint16_t* X, float* Z, uint16_t* A, void* stream) {
    if (!valid(s) || !params || !wb || !X || !Z || !A || n < 0)
        return err("mlp_forward: bad arguments");
    if (n == 0) return 0;
    if (n > INT32_MAX || !tiles_fit(s, n)) return err("mlp_forward: too many samples per call");
    const Dims d = dims(s);
    hipStream_t st = (hipStream_t)stream;
    const uint16_t* x = X;
    for (int l = 0; l < d.L; ++l) {
        const bool last = l == d.L - 1;
        float* Zl = Z + (int64_t)l * n * s->width;
        uint16_t* Al = last ? nullptr : A + (int64_t)l * n * s->width;
        // Z_l = x W_l^T + b_l and A_l = bf16(silu(Z_l)) in the GEMM's epilogue
        launch_gemm<0, 1>(dim3(tiles((int)n, d.out[l])), st, (int)n, d.out[l], d.in[l], x, d.in[l],
                          wb + d.woff[l], d.in[l], Zl, d.out[l], 0, d.in[l], params + d.boff[l], Al);
        const int rc = check(hipGetLastError());
        if (rc) return rc;
        x = Al;
    }
    return 0;
}

int mlp_infer(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
              const uint16_t* X, float* Z, uint16_t* A, void* stream) {
    if (!valid(s) || !params || !wb || !X || !Z || !A || n < 0)
        return err("mlp_infer: bad arguments");
    if (n == 0) return 0;
    if (n > INT32_MAX || !tiles_fit(s, n)) return err("mlp_infer: too many samples per call");
    const Dims d = dims(s);
    hipStream_t st = (hipStream_t)stream;
    const uint16_t* x = X;
    for (int l = 0; l < d.L; ++l) {
        const bool last = l == d.L - 1;
        // hidden layers: A_l = bf16(silu(x W_l^T + b_l)) only; output layer:
        // Y = x W^T + b into its block of Z
        float* Yl = last ? Z + (int64_t)l * n * s->width : nullptr;
        uint16_t* Al = last ? nullptr : A + (int64_t)l * n * s->width;
        launch_gemm<0, 1>(dim3(tiles((int)n, d.out[l])), st, (int)n, d.out[l], d.in[l], x, d.in[l],
                          wb + d.woff[l], d.in[l], Yl, d.out[l], 0, d.in[l], params + d.boff[l], Al);
        const int rc = check(hipGetLastError());
        if (rc) return rc;
        x = Al;
    }
    return 0;
}

int mlp_infer_fused(const mlp_shape* s, const float* params, const uint16_t* wb, int64_t n,
                    const uint16_t* X, float* Y, void* stream) {
    if (!valid(s) || n < 0) return err("mlp_infer_fused: bad arguments");
    if (s->width != fused::W || s->n_in > 32 || s->n_out > 16 || s->depth > fused::MAX_DEPTH)
        return err("mlp_infer_fused: needs width 128, n_in <= 32, n_out <= 16, depth <= 5");
    if (n == 0) return 0;
    if (!params || !wb || !X || !Y) return err("mlp_infer_fused: bad arguments");
    if ((uintptr_t)Y & 15) return err("mlp_infer_fused: Y must be 16-byte aligned");
    static int n_cu = 0;
    if (!n_cu) {
        int dev = 0;
        int rc = check(hipGetDevice(&dev));
        if (rc) return rc;
        rc = check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        if (rc) return rc;
    }
    // one block per compute unit (the weights fill most of its LDS), each
    // wave walking over groups of 64 samples
    const int64_t groups = (n + 16 * fused::J - 1) / (16 * fused::J);
    const int64_t per_block = fused::THREADS / 64;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(n_cu, (groups + per_block - 1) / per_block));
    const int vec_x = ((uintptr_t)X & 15) == 0 && (s->n_in & 7) == 0;
    hipStream_t st = (hipStream_t)stream;
    switch (s->depth) {
        case 1: hipLaunchKernelGGL(fused::k_mlp_fused<1>, dim3(blocks), dim3(fused::THREADS), 0, st, n, s->n_in, s->n_out, wb, params, X, Y, vec_x); break;
        case 2: hipLaunchKernelGGL(fused::k_mlp_fused<2>, dim3(blocks), dim3(fused::THREADS), 0, st, n, s->n_in, s->n_out, wb, params, X, Y, vec_x); break;
        case 3: hipLaunchKernelGGL(fused::k_mlp_fused<3>, dim3(blocks), dim3(fused::THREADS), 0, st, n, s->n_in, s->n_out, wb, params, X, Y, vec_x); break;
        case 4: hipLaunchKernelGGL(fused::k_mlp_fused<4>, dim3(blocks), dim3(fused::THREADS), 0, st, n, s->n_in, s->n_out, wb, params, X, Y, vec_x); break;
        default: hipLaunchKernelGGL(fused::k_mlp_fused<5>, dim3(blocks), dim3(fused::THREADS), 0, st, n, s->n_in, s->n_out, wb, params, X, Y, vec_x); break;
    }
    return check(hipGetLastError());
}

int mlp_backward(const mlp_shape* s, const uint16_t* wb, int64_t n, const uint16_t* X,
                 const float* Z, const uint16_t* A, const float* dY, float* grad, float* work_f,
                 uint16_t* work_b, void* stream) {
    if (!valid(s) || !wb || !X || !Z || !A || !dY || !grad || !work_f || !work_b || n <= 0)
        return err("mlp_backward: bad arguments");
    if (n > INT32_MAX || !tiles_fit(s, n)) return err("mlp_backward: too many samples per call");
    const Dims d = dims(s);
    hipStream_t st = (hipStream_t)stream;
    const int L = d.L;
    const int64_t wmax = s->width > s->n_out ? s->width : s->n_out;
    float* dA = work_f;                 // n x width
    float* dZf = work_f + n * wmax;     // n x max(width, n_out)
    int rc = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int out = d.out[l], in = d.in[l];
        // dZ_l as bf16 into work_b and db_l = column sums of dZ_l (partial
        // sums in the dZf half of work_f)
        if (l == L - 1) {
            hipLaunchKernelGGL(k_f32_to_bf16, dim3(nb(n * out, 256)), dim3(256), 0, st, n * out, dY,
                               work_b);
            rc = check(hipGetLastError());
            if (rc) return rc;
            rc = colsum_split(n, out, dY, grad + d.boff[l], dZf, n * wmax, st);
            if (rc) return rc;
        } else if (out <= 256) {
            int64_t B, rows;
            row_ranges(n, out, n * wmax, B, rows);
            hipLaunchKernelGGL(k_act_bwd_colsum, dim3((unsigned)B), dim3(256), 0, st, n, out, rows,
                               dA, Z + (int64_t)l * n * s->width, work_b, dZf);
            hipLaunchKernelGGL(k_reduce_cols, dim3(out), dim3(256), 0, st, (int)B, out, dZf,
                               grad + d.boff[l]);
            rc = check(hipGetLastError());
            if (rc) return rc;
        } else {
            hipLaunchKernelGGL(k_act_bwd, dim3(nb(n * out, 256)), dim3(256), 0, st, n, out, dA,
                               Z + (int64_t)l * n * s->width, dZf, work_b);
            rc = check(hipGetLastError());
            if (rc) return rc;
            hipLaunchKernelGGL(k_colsum, dim3(out), dim3(256), 0, st, n, out, dZf, grad + d.boff[l]);
            rc = check(hipGetLastError());
            if (rc) return rc;
        }
        const uint16_t* prev = l == 0 ? X : A + (int64_t)(l - 1) * n * s->width;
        // dW_l = dZ_l^T prev  (out x in).  dA_l is consumed (dZ_l is in
        // work_b), so its n x wmax floats hold the partial products until
        // dA_{l-1} is formed below.
        rc = gemm_tn_split(out, in, n, work_b, out, prev, in, grad + d.woff[l], dA, n * wmax, st);
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
