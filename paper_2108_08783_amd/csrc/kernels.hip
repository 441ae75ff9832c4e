// HIP kernels for gfx950: the fused pull-scheme collide-and-stream update
// with its compacted boundary pass, initialisation, read-out, wall shear
// stress, checkpoint and periodicity kernels.
//
// State convention.  Buffer S(t) holds, for every site y and direction i,
// the post-collision deviation h*_i(y, t-1) = f*_i - w_i in plane i at y
// (structure of arrays, plane stride np).  A site x pulls f_i(x, t) from
// S(t) at y = x - c_i when that voxel is fluid, and from its own opposite
// slot (plane opp(i), site x) when it is not: for a bounce-back wall that slot
// holds f*_opp(i)(x) (Sec. 2.4), for an elastic wall or an iolet link the
// boundary pass of the previous step wrote the link's value there (Sec. 2.3,
// Sec. 3).  Every slot is read by exactly one site per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "../../include/lbm.h"
#include "d3q19.hpp"
#include "kernels.hpp"

namespace lbm {
namespace {

// ---------------------------------------------------------------- codecs --
// Populations are stored as deviations h = f - w (Sec. 2.1 weights).  FP16
// deviations are scaled by 2^10 (exact) so that small values stay normal;
// BF16 keeps FP32's exponent range and needs no scale.  Conversions to
// 16 bits round to nearest even.
template <int DT>
struct Codec;
//
// The update kernel works on scale * h (sdec / senc): scaling by a power of
// two commutes with every rounding, so carrying the FP16 scale through the
// moments, the relaxation and the link rules gives the same bits as
// unscaling on load and rescaling on store, without the two multiplies per
// population.
template <>
struct Codec<LBM_F64> {
    using raw = double;
    using acc = double;
    static constexpr acc scale = 1.0;
    __device__ static acc dec(raw v) { return v; }
    __device__ static raw enc(acc v) { return v; }
    __device__ static acc sdec(raw v) { return v; }
    __device__ static raw senc(acc v) { return v; }
};
template <>
struct Codec<LBM_F32> {
    using raw = float;
    using acc = float;
    static constexpr acc scale = 1.0f;
    __device__ static acc dec(raw v) { return v; }
    __device__ static raw enc(acc v) { return v; }
    __device__ static acc sdec(raw v) { return v; }
    __device__ static raw senc(acc v) { return v; }
};
template <>
struct Codec<LBM_F16DEV> {
    using raw = uint16_t;
    using acc = float;
    static constexpr acc scale = 1024.0f;
    __device__ static acc dec(raw v) {
        return (float)__builtin_bit_cast(_Float16, v) * (1.0f / 1024.0f);
    }
    __device__ static raw enc(acc v) { return __builtin_bit_cast(uint16_t, (_Float16)(v * 1024.0f)); }
    __device__ static acc sdec(raw v) { return (float)__builtin_bit_cast(_Float16, v); }
    __device__ static raw senc(acc v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
template <>
struct Codec<LBM_BF16DEV> {
    using raw = uint16_t;
    using acc = float;
    static constexpr acc scale = 1.0f;
    __device__ static acc sdec(raw v) { return dec(v); }
    __device__ static raw senc(acc v) { return enc(v); }
    __device__ static acc dec(raw v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static raw enc(acc v) {
        uint32_t b = __float_as_uint(v);
        b += 0x7FFFu + ((b >> 16) & 1u);
        return (raw)(b >> 16);
    }
};

template <typename acc>
struct W {
    static constexpr acc w0 = (acc)(1.0 / 3.0);
    static constexpr acc w1 = (acc)(1.0 / 18.0);
    static constexpr acc w2 = (acc)(1.0 / 36.0);
};

__device__ __forceinline__ constexpr int dopp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------- gather --
template <typename I>
__device__ __forceinline__ void load_offsets(const I* __restrict__ nbr, int64_t np, int x,
                                             I (&d)[18]) {
#pragma unroll
    for (int i = 0; i < 18; ++i) d[i] = nbr[(int64_t)i * np + x];
}

// f_i(x, t) - w_i for all i from buffer A (both sentinels redirect to the
// site's own opposite slot).
template <int DT, typename I>
__device__ __forceinline__ void gather(const typename Codec<DT>::raw* __restrict__ A, int64_t np,
                                       int x, const I (&d)[18],
                                       typename Codec<DT>::acc (&h)[Q]) {
    h[0] = Codec<DT>::dec(A[x]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const I di = d[i - 1];
        const bool redirect = di <= Sentinel<I>::GHOST;
        const int64_t idx = redirect ? (int64_t)dopp(i) * np + x : (int64_t)i * np + x + di;
        h[i] = Codec<DT>::dec(A[idx]);
    }
}

// Byte offset of element e of a population buffer.  When every buffer is
// smaller than 2^31 bytes (SMALL) the offset is formed in 32 bits, so the
// load or store takes a uniform base address and a 32-bit per-lane offset.
template <int DT, bool SMALL>
struct Off {
    using raw = typename Codec<DT>::raw;
    using type = typename std::conditional<SMALL, uint32_t, uint64_t>::type;
    __device__ static type of(int64_t e) { return (type)e * (type)sizeof(raw); }
    __device__ static const raw* ptr(const raw* base, type off) {
        return (const raw*)((const char*)base + off);
    }
    __device__ static raw* ptr(raw* base, type off) { return (raw*)((char*)base + off); }
};

template <typename raw, bool NTL>
__device__ __forceinline__ raw ld(const raw* p) {
    if constexpr (NTL)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// NTL: non-temporal loads (every population is read exactly once per step).
template <int DT, bool SMALL, bool NTL>
__device__ __forceinline__ void gather32(const typename Codec<DT>::raw* __restrict__ A, int64_t np,
                                         int x, const int32_t (&d)[18],
                                         typename Codec<DT>::acc (&h)[Q]) {
    using O = Off<DT, SMALL>;
    using T = typename O::type;
    using raw = typename O::raw;
    const T npt = (T)np, xt = (T)x;
    h[0] = Codec<DT>::sdec(ld<raw, NTL>(O::ptr(A, xt * (T)sizeof(raw))));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int32_t di = d[i - 1];
        const bool redirect = di <= Sentinel<int32_t>::GHOST;
        const T e = redirect ? (T)dopp(i) * npt + xt : (T)i * npt + (T)(x + di);
        h[i] = Codec<DT>::sdec(ld<raw, NTL>(O::ptr(A, e * (T)sizeof(raw))));
    }
}

// Slot of the 8-entry stretch table holding the row (y - cy, z - cz) of
// direction i (rows in the order (1,0),(-1,0),(0,1),(0,-1),(1,1),(-1,-1),
// (1,-1),(-1,1) of (dy,dz)); -1 for the same row.
__device__ __forceinline__ constexpr int row_slot(int i) {
    return (CY[i] == 0 && CZ[i] == 0) ? -1
         : (CY[i] == -1 && CZ[i] == 0) ? 0
         : (CY[i] == 1 && CZ[i] == 0) ? 1
         : (CY[i] == 0 && CZ[i] == -1) ? 2
         : (CY[i] == 0 && CZ[i] == 1) ? 3
         : (CY[i] == -1 && CZ[i] == -1) ? 4
         : (CY[i] == 1 && CZ[i] == 1) ? 5
         : (CY[i] == -1 && CZ[i] == 1) ? 6 : 7;
}

// Neighbour offsets of site x (32-bit, table sentinels) and its boundary
// record id (-1 for interior sites; only looked up by sites with
// boundary-pass links in table addressing).
template <int ADDR, bool ALIGNED>
__device__ __forceinline__ void site_offsets(const StepArgs& a, int x, int32_t (&d)[18], int& rec) {
    if constexpr (ADDR == ADDR_COMP) {
        // ALIGNED: the 64 lanes of the wavefront hold the 64 sites of one
        // record, so the record is loaded with scalar loads.  The stretch
        // (every lane) and the link mask (irregular lanes) depend only on
        // the record and are loaded together, so the gathers wait for two
        // memory round trips.
        const int w = ALIGNED ? __builtin_amdgcn_readfirstlane(x >> 6) : (x >> 6);
        const int l = x & 63;
        const WfRec r = a.wf[w];
        const uint64_t bit = 1ull << l, below = bit - 1ull;
        int st = r.cur + __popcll(r.smask & (bit | below));
        st = st < 0 ? 0 : st;
        const int4* S = (const int4*)(a.stretch + 8 * (int64_t)st);
        const int4 s0 = S[0], s1 = S[1];
        uint32_t nf = 0;
        rec = -1;
        if (r.imask & bit) {
            rec = r.firr + __popcll(r.imask & below);
            nf = a.nfm[rec];
        }
        const int32_t D[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        const int32_t sent = (nf >> 31) ? Sentinel<int32_t>::GHOST : Sentinel<int32_t>::BB;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int rs = row_slot(i);
            d[i - 1] = ((nf >> (i - 1)) & 1u) ? sent : (rs < 0 ? 0 : D[rs]) - CX[i];
        }
        if (r.emask & bit) {
            // a row of several fluid runs: the site's own 18 offsets
            const int e = r.fexc + __popcll(r.emask & below);
#pragma unroll
            for (int i = 0; i < 18; ++i) d[i] = a.exc[(int64_t)i * a.n_exc_pad + e];
        }
    } else {
        using I = typename std::conditional<ADDR == ADDR_T16, int16_t, int32_t>::type;
        const I* nbr = (const I*)a.nbr;
        bool ghost = false;
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const I v = nbr[(int64_t)i * a.np + x];
            d[i] = v == Sentinel<I>::BB ? Sentinel<int32_t>::BB
                 : v == Sentinel<I>::GHOST ? Sentinel<int32_t>::GHOST : (int32_t)v;
            ghost |= v == Sentinel<I>::GHOST;
        }
        rec = ghost ? a.bidx[x] : -1;
    }
}

// Pulled slots of site x as 32-bit byte offsets (every buffer below 2^31
// bytes).  Plane i is read through its own base pointer
//   P_i = A + (i np - c_ix - np - 1) s        (s = bytes per slot),
// which may lie below A; the offsets are then never negative:
//   fluid upstream site x - c_i = x + d:      (x + d + c_ix + np + 1) s,
//   own opposite slot (plane opp(i), site x): (x + (opp(i) - i + 1) np + c_ix + 1) s.
// With compressed addressing every direction of one lattice row (dy, dz)
// shares one row offset, d + c_ix being the row's stretch entry, and a link
// to a non-fluid voxel picks the opposite-slot offset with a bit-select on
// the site's link mask: no branch and no per-direction index arithmetic.
template <int DT>
__device__ __forceinline__ uint32_t redirect_off(int i, uint32_t xr, uint32_t np) {
    constexpr uint32_t S = sizeof(typename Codec<DT>::raw);
    return xr + ((dopp(i) > i ? 2u * np : 0u) + (uint32_t)CX[i]) * S;
}

template <int DT, int ADDR, bool ALIGNED>
__device__ __forceinline__ void pull_slots(const StepArgs& a, int x, uint32_t (&o)[18],
                                           bool& ghost, int& rec) {
    constexpr uint32_t S = sizeof(typename Codec<DT>::raw);
    const uint32_t np = (uint32_t)a.np;
    const uint32_t own = ((uint32_t)x + np + 1u) * S;   // fluid source in the site's own row
    const uint32_t xr = ((uint32_t)x + 1u) * S;
    if constexpr (ADDR == ADDR_COMP) {
        // ALIGNED: the 64 lanes of the wavefront hold the 64 sites of one
        // record, which is therefore loaded with scalar loads.
        const int w = ALIGNED ? __builtin_amdgcn_readfirstlane(x >> 6) : (x >> 6);
        const int l = x & 63;
        const WfRec r = a.wf[w];
        const uint64_t bit = 1ull << l, below = bit - 1ull;
        int st = r.cur + __popcll(r.smask & (bit | below));
        st = st < 0 ? 0 : st;
        // lane-indexed tables are read as a uniform base plus a 32-bit offset
        const int4* SP = (const int4*)((const char*)a.stretch + (uint64_t)((uint32_t)st * 32u));
        const int4 s0 = SP[0], s1 = SP[1];
        uint32_t nf = 0;
        rec = -1;
        if (r.imask & bit) {
            rec = r.firr + __popcll(r.imask & below);
            nf = *(const uint32_t*)((const char*)a.nfm + (uint64_t)((uint32_t)rec * 4u));
        }
        const int32_t D[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        uint32_t row[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) row[k] = own + (uint32_t)D[k] * S;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int rs = row_slot(i);
            const uint32_t n = rs < 0 ? own : row[rs];
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)nf, i - 1, 1);
            o[i - 1] = (m & redirect_off<DT>(i, xr, np)) | (~m & n);
        }
        ghost = (int32_t)nf < 0;
        if (r.emask & bit) {
            // a row of several fluid runs: the site's own 18 offsets (its
            // non-fluid links are in its link mask as for any irregular site)
            const int e = r.fexc + __popcll(r.emask & below);
            const uint64_t eo = (uint32_t)e * 4u;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int32_t v = *(const int32_t*)((const char*)(a.exc + (int64_t)(i - 1) * a.n_exc_pad) + eo);
                o[i - 1] = v <= Sentinel<int32_t>::GHOST
                               ? redirect_off<DT>(i, xr, np)
                               : ((uint32_t)(x + v + CX[i]) + np + 1u) * S;
            }
        }
    } else {
        using I = typename std::conditional<ADDR == ADDR_T16, int16_t, int32_t>::type;
        const I* nbr = (const I*)a.nbr;
        ghost = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const I v = nbr[(int64_t)(i - 1) * a.np + x];
            const bool sent = v == Sentinel<I>::BB || v == Sentinel<I>::GHOST;
            o[i - 1] = sent ? redirect_off<DT>(i, xr, np)
                            : ((uint32_t)(x + (int32_t)v + CX[i]) + np + 1u) * S;
            ghost |= v == Sentinel<I>::GHOST;
        }
        rec = ghost ? a.bidx[x] : -1;
    }
}

// Raw buffer loads (gfx9 buffer descriptor: stride 0, byte range checked,
// an out-of-range load returns 0).  The per-lane byte offset goes in a
// vector register, the per-plane offset in a scalar one, so a plane costs
// no vector instruction and no scalar base pair.  AUX 2: non-temporal.
constexpr int BUF_DWORD3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             BUF_DWORD3);
}

template <typename raw, int AUX>
__device__ __forceinline__ raw buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(raw) == 2)
        return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX));
    else if constexpr (sizeof(raw) == 4)
        return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
    else
        return __builtin_bit_cast(raw, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
}

// scale * h_i(x, t) for all i, with the offsets of pull_slots.  16-bit
// storage reads through one buffer descriptor that starts (np + 2) slots
// below A, so plane i's scalar offset (i np - c_ix + 1) s is positive and the
// descriptor range ends with A; wider storage reads through a 64-bit base
// per plane (measured: the buffer form is 3 % faster for 16-bit storage and
// 2 % slower for FP32, whose register count then drops it to 6 waves).
template <int DT, bool NTL>
__device__ __forceinline__ void gather_slots(const typename Codec<DT>::raw* __restrict__ A,
                                             int64_t np, int x, const uint32_t (&o)[18],
                                             typename Codec<DT>::acc (&h)[Q]) {
    using raw = typename Codec<DT>::raw;
    constexpr uint32_t S = sizeof(raw);
    if constexpr (S == 2) {
        constexpr int AUX = NTL ? 2 : 0;
        const uint32_t n = (uint32_t)np;
        const __amdgpu_buffer_rsrc_t r =
            buffer_rsrc((const char*)A - (int64_t)(np + 2) * S, (20u * n + 2u) * S);
        h[0] = Codec<DT>::sdec(buf_ld<raw, AUX>(r, (uint32_t)x * S, (n + 2u) * S));
#pragma unroll
        for (int i = 1; i < Q; ++i)
            h[i] = Codec<DT>::sdec(
                buf_ld<raw, AUX>(r, o[i - 1], ((uint32_t)i * n - (uint32_t)CX[i] + 1u) * S));
    } else {
        const char* base = (const char*)A;
        h[0] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(base + (uint64_t)((uint32_t)x * S))));
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const char* P = base + ((int64_t)i * np - CX[i] - np - 1) * (int64_t)S;
            h[i] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(P + (uint64_t)o[i - 1])));
        }
    }
}

// ------------------------------------------------------------- physics ----
// Sec. 2.1 eqs. Density and Momentum in deviation form: sum_i w_i = 1 and
// sum_i w_i c_i = 0, so rho = 1 + sum h_i and rho u = sum h_i c_i.
template <typename acc>
struct Mom {
    acc drho, rho, ux, uy, uz;
};

// isc: 1 / scale when h holds scale * h (the moments are returned unscaled).
template <typename acc>
__device__ __forceinline__ Mom<acc> moments(const acc (&h)[Q], acc isc = (acc)1) {
    Mom<acc> m;
    acc s = h[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) s += h[i];
    const acc jx = (h[1] - h[2]) + (h[7] - h[8]) + (h[9] - h[10]) + (h[11] - h[12]) + (h[13] - h[14]);
    const acc jy = (h[3] - h[4]) + (h[7] - h[8]) - (h[9] - h[10]) + (h[15] - h[16]) + (h[17] - h[18]);
    const acc jz = (h[5] - h[6]) + (h[11] - h[12]) - (h[13] - h[14]) + (h[15] - h[16]) - (h[17] - h[18]);
    m.drho = s * isc;
    m.rho = (acc)1 + m.drho;
    const acc inv = ((acc)1 / m.rho) * isc;
    m.ux = jx * inv;
    m.uy = jy * inv;
    m.uz = jz * inv;
    return m;
}

// Sec. 2.1 eq. feq (standard 1/2 factors) minus w_i:
// w_i (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)).  Pairs (2k+1, 2k+2) are
// opposite directions with c.u = +-cu_k.
// sc: scale of the result (a power of two, folded into the weights).
template <typename acc>
__device__ __forceinline__ void heq(acc drho, acc rho, acc ux, acc uy, acc uz, acc (&e)[Q],
                                    acc sc = (acc)1) {
    const acc r0 = drho - rho * (acc)1.5 * (ux * ux + uy * uy + uz * uz);
    const acc r3 = (acc)3 * rho, r45 = (acc)4.5 * rho;
    e[0] = (W<acc>::w0 * sc) * r0;
    const acc cu[9] = {ux, uy, uz, ux + uy, ux - uy, ux + uz, ux - uz, uy + uz, uy - uz};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const acc w = (k < 3 ? W<acc>::w1 : W<acc>::w2) * sc;
        const acc p = r3 * cu[k];
        const acc q = r45 * cu[k] * cu[k] + r0;
        e[2 * k + 1] = w * (q + p);
        e[2 * k + 2] = w * (q - p);
    }
}

template <typename acc>
__device__ __forceinline__ acc heq_one(int i, acc drho, acc rho, acc ux, acc uy, acc uz) {
    const acc cu = (acc)CX[i] * ux + (acc)CY[i] * uy + (acc)CZ[i] * uz;
    const acc w = i == 0 ? W<acc>::w0 : (i <= 6 ? W<acc>::w1 : W<acc>::w2);
    return w * (drho + rho * ((acc)3 * cu + (acc)4.5 * cu * cu - (acc)1.5 * (ux * ux + uy * uy + uz * uz)));
}

template <typename raw>
__device__ __forceinline__ void put(raw* p, raw v, bool nt) {
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename acc>
__device__ __forceinline__ acc sin_acc(acc v);
template <>
__device__ __forceinline__ double sin_acc<double>(double v) { return sin(v); }
template <>
__device__ __forceinline__ float sin_acc<float>(float v) { return sinf(v); }

// Drive value of an iolet at step t (Sec. 3).  The phase is reduced in
// double so that long runs keep full precision.
template <typename acc>
__device__ __forceinline__ acc drive_dev(const IoletParams& q, int64_t t, acc& minus1) {
    acc s = 0;
    if (q.amp != 0.0) {
        const double ph = (double)t * q.inv_period;
        const double fr = ph - floor(ph);
        s = sin_acc<acc>((acc)(6.283185307179586 * fr + q.phase));
    }
    const acc a0 = (acc)q.a0;
    minus1 = (acc)(q.a0 - 1.0) + a0 * (acc)q.amp * s;
    return a0 * ((acc)1 + (acc)q.amp * s);
}

// ----------------------------------------------------------- update -------
// Block -> site-range mapping that keeps consecutive site ranges on one XCD
// (workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2), so that cache lines shared by neighbouring wavefronts meet in one L2.
__device__ __forceinline__ int remap_xcd(int b, int nblk) {
    const int per = nblk >> 3, rem = nblk & 7;
    const int j = b & 7, k = b >> 3;
    return j * per + (j < rem ? j : rem) + k;
}

// The same in chunks of g consecutive blocks (g a power of two): the k-th
// block that XCD j receives runs block ((k / g) * 8 + j) * g + k % g, so
// each XCD works through its own run of g neighbouring blocks at a time and
// the eight runs advance together through the site range (the work of a
// geometry whose cost varies along the site order stays balanced between
// the XCDs).  Blocks beyond the last whole round of 8 g keep their index.
__device__ __forceinline__ int remap_xcd_chunk(int b, int nblk, int g) {
    const int full = nblk / (8 * g) * (8 * g);
    if (b >= full) return b;
    const int j = b & 7, k = b >> 3;
    return ((k / g) * 8 + j) * g + (k & (g - 1));
}

__device__ __forceinline__ int remap_block(int b, int nblk, int mode) {
    return mode == 0 ? b : mode == 1 ? remap_xcd(b, nblk) : remap_xcd_chunk(b, nblk, mode);
}

// Links whose upstream voxel is an elastic wall or an iolet (boundary record
// j of a site with moments m and post-collision deviations out): the value
// of each such link i replaces out[opp(i)], the slot the site pulls for link
// i at the next step.
//   elastic wall (Sec. 2.3): the wall node carries the fluid node's
//     non-equilibrium part,
//       f_i(x, t+1) = feq_i(rho, U') + (1 - 1/tau) (f_i - feq_i(rho, u))
//                  = feq_i(rho, U') + f*_i - feq_i(rho, u),
//     U' = s u, s = (F + Delta r - 1) / Delta r, Delta r = 1 + Delta E,
//     Delta E = max(0, (p - P0) / k), p = rho / 3;
//   iolets (Sec. 3): the iolet node is at equilibrium,
//       f_i(x, t+1) = feq_i(rho', U'),
//     density iolet rho' = rho_io(t), U' = (u.n) n with n the iolet's unit
//     inward normal if one is set, else U' = u; velocity iolet rho' = rho,
//     U' = weight(x) u_io(t) dir.
// The parts of a boundary record the link rules read.
template <typename acc>
struct BRec {
    uint32_t bw = 0, bi = 0;   // wall mask | instance, iolet mask | slot
    acc c1 = 0, c0 = 0, F = 0; // elastic-wall coefficients (WallCoef)
};

template <typename acc>
__device__ __forceinline__ BRec<acc> load_brec(const StepArgs& a, int j) {
    BRec<acc> r;
    r.bw = a.bwall[j];
    r.bi = a.bio[j];
    if constexpr (std::is_same<acc, float>::value) {
        const WallCoefF q = a.bqf[j];
        r.c1 = q.c1;
        r.c0 = q.c0;
        r.F = q.F;
    } else {
        const WallCoef q = a.bq[j];
        r.c1 = (acc)q.c1;
        r.c0 = (acc)q.c0;
        r.F = (acc)q.F;
    }
    return r;
}


template <typename acc>
__device__ __forceinline__ void apply_links(const StepArgs& a, int j, const Mom<acc>& m,
                                            acc (&out)[Q], const BRec<acc>& r, acc sc) {
    const uint32_t bw = r.bw, bi = r.bi;
    const uint32_t wmask = bw & 0x7FFFEu, imask = bi & 0x7FFFEu;
    const uint32_t inst = bw >> 19;
    acc s = 0;
    if (wmask) {
        acc dE = m.drho * r.c1 + r.c0;
        dE = dE > (acc)0 ? dE : (acc)0;
        s = (r.F + dE) / ((acc)1 + dE);
    }
    acc idr = m.drho, ir = m.rho, ix = m.ux, iy = m.uy, iz = m.uz;
    if (imask) {
        const IoletParams& q = a.iop[bi >> 19];
        const int64_t t = a.clock[a.clock_in] - a.ip[inst].t0;
        acc vm1;
        const acc v = drive_dev<acc>(q, t, vm1);
        if (q.kind == LBM_IOLET_DENSITY) {
            idr = vm1;
            ir = v;
            if (q.pad) {  // the fluid node's velocity along the inward normal only
                const acc d0 = (acc)q.dir[0], d1 = (acc)q.dir[1], d2 = (acc)q.dir[2];
                const acc un = m.ux * d0 + m.uy * d1 + m.uz * d2;
                ix = un * d0;
                iy = un * d1;
                iz = un * d2;
            }
        } else {
            const acc sp = (acc)a.bw[j] * v;
            ix = sp * (acc)q.dir[0];
            iy = sp * (acc)q.dir[1];
            iz = sp * (acc)q.dir[2];
        }
    }
    // Elastic wall links: rho' = rho, U' = s u, so
    //   feq_i(rho, s u) - feq_i(rho, u)
    //     = w_i rho (s - 1) (3 c.u + (s + 1) (9/2 (c.u)^2 - 3/2 u.u)),
    // and opposite directions differ only in the sign of c.u.  The value of
    // link i goes to slot opp(i); both slots of a pair are written from the
    // unmodified post-collision values.
    // out holds sc * h (sc a power of two), so the link terms are scaled too
    const acc A = m.rho * (s - (acc)1) * sc, Bs = s + (acc)1;
    const acc u2 = (acc)1.5 * (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
    const acc cu[9] = {m.ux, m.uy, m.uz, m.ux + m.uy, m.ux - m.uy, m.ux + m.uz, m.ux - m.uz,
                       m.uy + m.uz, m.uy - m.uz};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = 2 * k + 1, o = i + 1;
        const bool wi = (wmask >> i) & 1u, wo = (wmask >> o) & 1u;
        const bool ii = (imask >> i) & 1u, io = (imask >> o) & 1u;
        const acc oi = out[i], oo = out[o];
        const acc w = k < 3 ? W<acc>::w1 : W<acc>::w2;
        const acc t = Bs * ((acc)4.5 * cu[k] * cu[k] - u2), p = (acc)3 * cu[k];
        if (wi) out[o] = oi + w * A * (t + p);
        if (wo) out[i] = oo + w * A * (t - p);
        if (ii | io) {  // iolet links (rare): equilibrium at (rho', U')
            if (ii) out[o] = heq_one<acc>(i, idr, ir, ix, iy, iz) * sc;
            if (io) out[i] = heq_one<acc>(o, idr, ir, ix, iy, iz) * sc;
        }
    }
}

// Collision and store of one site whose pre-collision deviations h are
// gathered, in the codec's scaled domain (moments, BGK, link rules, 19
// coalesced stores).
template <int DT, bool SMALL>
__device__ __forceinline__ void collide_store(const StepArgs& a, int x, bool ghost, int rec,
                                              typename Codec<DT>::acc (&h)[Q],
                                              BRec<typename Codec<DT>::acc> br) {
    using raw = typename Codec<DT>::raw;
    using acc = typename Codec<DT>::acc;
    constexpr acc sc = Codec<DT>::scale;
    raw* __restrict__ B = (raw*)a.B;
    const Mom<acc> m = moments(h, (acc)1 / sc);
    {
        acc e[Q];
        heq(m.drho, m.rho, m.ux, m.uy, m.uz, e, sc);
        const acc om = (acc)a.omega;
#pragma unroll
        for (int i = 0; i < Q; ++i) h[i] = h[i] + om * (e[i] - h[i]);
    }
    acc (&out)[Q] = h;
    if (ghost) apply_links<acc>(a, rec, m, out, br, sc);
    const bool nt = (a.nontemporal & 1) != 0;
    if constexpr (SMALL && sizeof(raw) > 2) {
        // one lane offset, a uniform base per plane
        const uint64_t xs = (uint32_t)x * (uint32_t)sizeof(raw);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            char* Bi = (char*)B + (int64_t)i * a.np * (int64_t)sizeof(raw);
            put((raw*)(Bi + xs), Codec<DT>::senc(out[i]), nt);
        }
    } else {
        using O = Off<DT, SMALL>;
        using T = typename O::type;
        const T npt = (T)a.np, xt = (T)x;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            put(O::ptr(B, ((T)i * npt + xt) * (T)sizeof(raw)), Codec<DT>::senc(out[i]), nt);
    }
}

// One site: pull, BGK collision (Sec. 2.1 eq. LBE_SRT) and store.  A site
// with boundary-pass links either returns (compacted mode, when called from
// the update blocks: the boundary blocks update it) or applies the link
// rules of its boundary record in place (fused mode, and the boundary
// blocks of the compacted mode).
template <int DT, int ADDR, bool ALIGNED, bool SMALL, bool NTL>
__device__ __forceinline__ void update_site(const StepArgs& a, int x, bool from_boundary_blocks) {
    using acc = typename Codec<DT>::acc;
    using raw = typename Codec<DT>::raw;
    int rec;
    bool ghost;
    acc h[Q];
    BRec<acc> br;
    if constexpr (SMALL) {
        uint32_t o[18];
        pull_slots<DT, ADDR, ALIGNED>(a, x, o, ghost, rec);
        if (ghost && !from_boundary_blocks && !a.fused) return;
        // the boundary record is loaded ahead of the gathers, so its latency
        // overlaps theirs (its single-precision coefficients need no
        // conversion, so nothing waits for it before the gathers issue)
        if (ghost) br = load_brec<acc>(a, rec);
        gather_slots<DT, NTL>((const raw*)a.A, a.np, x, o, h);
    } else {
        int32_t d[18];
        site_offsets<ADDR, ALIGNED>(a, x, d, rec);
        ghost = false;
#pragma unroll
        for (int i = 0; i < 18; ++i) ghost |= (d[i] == Sentinel<int32_t>::GHOST);
        if (ghost && !from_boundary_blocks && !a.fused) return;
        if (ghost) br = load_brec<acc>(a, rec);
        gather32<DT, SMALL, NTL>((const raw*)a.A, a.np, x, d, h);
    }
    collide_store<DT, SMALL>(a, x, ghost, rec, h, br);
}

// 16-bit storage is latency-bound: 8 waves per SIMD beats 6.  Only the
// 32-bit offset variants fit the 64 registers of 8 waves; the 64-bit
// variants (population buffers beyond 2 GiB) would spill, and they and
// 32/64-bit storage keep the compiler's choice.
template <int DT, bool SMALL>
constexpr int step_waves() {
    return (SMALL && (DT == LBM_F16DEV || DT == LBM_BF16DEV)) ? 8 : 1;
}

template <int DT, int ADDR, bool SMALL, bool NTL>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(step_waves<DT, SMALL>())))
void k_step(StepArgs a) {
    const int b = blockIdx.x;
    if (b < a.n_int_blocks) {
        const int lb = remap_block(b, a.n_int_blocks, a.xcd_remap);
        const int x = lb * (int)blockDim.x + (int)threadIdx.x;
        if (x < a.n) update_site<DT, ADDR, true, SMALL, NTL>(a, x, false);
    } else {
        const int j = (b - a.n_int_blocks) * (int)blockDim.x + (int)threadIdx.x;
        if (j < a.nb) update_site<DT, ADDR, false, SMALL, NTL>(a, a.rsite[a.bj[j]], true);
    }
    if (b == 0 && threadIdx.x == 0) a.clock[a.clock_in ^ 1] = a.clock[a.clock_in] + 1;
}

// --------------------------------------------------------- site pairs ---
// Two sites per lane (32-bit storage): each wavefront updates a tile of 128
// consecutive sites, lane l the sites x and x + 64.  Each direction's 64
// consecutive entries start at an arbitrary offset, so one wavefront's load
// touches one 128-byte line more than its 256 bytes need; the two loads of
// a direction are issued back to back here, and the line they share is
// fetched once.  The arithmetic is k_step's.

// Pulled slots of site x as in pull_slots (compressed addressing, the
// 64 sites of x's record in one half-tile), as byte offsets (SMALL: every
// buffer below 2 GiB) or as element offsets (scaled to bytes in 64 bits at
// the load).  A lane past the last site (act false) gets the own-slot
// offsets of a site inside the buffer and no boundary record; its results
// are not stored.
template <int DT, bool SMALL>
__device__ __forceinline__ void pair_slots(const StepArgs& a, int x, bool act, uint32_t (&o)[18],
                                           bool& ghost, int& rec) {
    constexpr uint32_t S = SMALL ? sizeof(typename Codec<DT>::raw) : 1u;
    const uint32_t np = (uint32_t)a.np;
    const int xs = act ? x : min(x, (int)np - 1);
    const uint32_t own = ((uint32_t)xs + np + 1u) * S;
    const uint32_t xr = ((uint32_t)xs + 1u) * S;
    // the own opposite slot, in the same unit as every other offset here
    // (redirect_off counts bytes; with element offsets it would not match)
    const auto red = [&](int i) {
        return xr + ((dopp(i) > i ? 2u * np : 0u) + (uint32_t)CX[i]) * S;
    };
    const int w = __builtin_amdgcn_readfirstlane(x >> 6);
    const int l = x & 63;
    const WfRec r = a.wf[w];
    const uint64_t bit = 1ull << l, below = bit - 1ull;
    int st = r.cur + __popcll(r.smask & (bit | below));
    st = st < 0 ? 0 : st;
    const int4* SP = (const int4*)((const char*)a.stretch + (uint64_t)((uint32_t)st * 32u));
    const int4 s0 = SP[0], s1 = SP[1];
    uint32_t nf = 0;
    rec = -1;
    if ((r.imask & bit) && act) {
        rec = r.firr + __popcll(r.imask & below);
        nf = *(const uint32_t*)((const char*)a.nfm + (uint64_t)((uint32_t)rec * 4u));
    }
    if (!act) nf = 0x3FFFFu;   // every link reads the own opposite slot
    const int32_t D[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
    uint32_t row[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) row[k] = own + (uint32_t)D[k] * S;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int rs = row_slot(i);
        const uint32_t n = rs < 0 ? own : row[rs];
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)nf, i - 1, 1);
        o[i - 1] = (m & red(i)) | (~m & n);
    }
    ghost = (int32_t)nf < 0;
    if ((r.emask & bit) && act) {
        const int e = r.fexc + __popcll(r.emask & below);
        const uint64_t eo = (uint32_t)e * 4u;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int32_t v = *(const int32_t*)((const char*)(a.exc + (int64_t)(i - 1) * a.n_exc_pad) + eo);
            o[i - 1] = v <= Sentinel<int32_t>::GHOST
                           ? red(i)
                           : ((uint32_t)(x + v + CX[i]) + np + 1u) * S;
        }
    }
}

template <int DT, bool SMALL, bool NTL>
__global__ __launch_bounds__(1024) void k_step_pair(StepArgs a) {
    using raw = typename Codec<DT>::raw;
    using acc = typename Codec<DT>::acc;
    constexpr uint32_t S = sizeof(raw);
    static_assert(S == 4, "site pairs are built for 32-bit storage");
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0) a.clock[a.clock_in ^ 1] = a.clock[a.clock_in] + 1;
    const int lb = remap_block(b, a.n_int_blocks, a.xcd_remap);
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int t0 = lb * 2 * (int)blockDim.x + wv * 128;   // first site of the wavefront's tile
    const int x0 = t0 + lane, x1 = x0 + 64;
    // a tile without any site is left out (uniform across the wavefront);
    // tiles start at multiples of 128 and the planes hold a multiple of 256
    // entries, so both halves of a started tile lie inside the planes
    if (t0 >= a.n) return;
    const bool v0 = x0 < a.n, v1 = x1 < a.n;
    uint32_t o0[18], o1[18];
    bool g0, g1;
    int r0, r1;
    pair_slots<DT, SMALL>(a, x0, v0, o0, g0, r0);
    pair_slots<DT, SMALL>(a, x1, v1, o1, g1, r1);
    BRec<acc> br0, br1;
    if (g0) br0 = load_brec<acc>(a, r0);
    if (g1) br1 = load_brec<acc>(a, r1);
    acc h0[Q], h1[Q];
    const char* base = (const char*)a.A;
    const int64_t np = a.np;
    const uint32_t xs0 = v0 ? (uint32_t)x0 : 0u, xs1 = v1 ? (uint32_t)x1 : 0u;
    // byte offset of an offset from pair_slots
    constexpr uint64_t U = SMALL ? 1u : S;
    const uint64_t e0 = SMALL ? (uint64_t)(xs0 * S) : (uint64_t)xs0 * S;
    const uint64_t e1 = SMALL ? (uint64_t)(xs1 * S) : (uint64_t)xs1 * S;
    h0[0] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(base + e0)));
    h1[0] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(base + e1)));
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const char* P = base + ((int64_t)i * np - CX[i] - np - 1) * (int64_t)S;
        h0[i] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(P + (uint64_t)o0[i - 1] * U)));
        h1[i] = Codec<DT>::sdec(ld<raw, NTL>((const raw*)(P + (uint64_t)o1[i - 1] * U)));
    }
    if (v0) collide_store<DT, SMALL>(a, x0, g0, r0, h0, br0);
    if (v1) collide_store<DT, SMALL>(a, x1, g1, r1, h1, br1);
}

// ------------------------------------------------------------ read-out ---
template <int DT, typename I>
__global__ __launch_bounds__(256) void k_fields(FieldArgs a) {
    using acc = typename Codec<DT>::acc;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int x = a.first + k;
    I d[18];
    load_offsets<I>((const I*)a.nbr, a.np, x, d);
    acc h[Q];
    gather<DT, I>((const typename Codec<DT>::raw*)a.A, a.np, x, d, h);
    const Mom<acc> m = moments(h);
    double v[3] = {(double)m.ux, (double)m.uy, (double)m.uz};
    int o = k;
    if (a.i2c) {
        o = a.i2c[k];
        const double t = v[0];
        v[0] = v[a.axis];
        v[a.axis] = t;
    }
    const double r = 1.0 + (double)m.drho;
    if (a.bad && !(isfinite(r) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2])))
        atomicOr(a.bad, 1u);
    if (a.rho) a.rho[o] = r;
    if (a.u) {
        a.u[3 * (int64_t)o] = v[0];
        a.u[3 * (int64_t)o + 1] = v[1];
        a.u[3 * (int64_t)o + 2] = v[2];
    }
}

// Wall shear stress (sigma = -(1 - 1/(2 tau)) sum fneq c c, traction
// t = sigma n, WSS = |t - (t.n) n|) and Delta r at the instance's wall sites.
template <int DT, typename I>
__global__ __launch_bounds__(256) void k_wall(WallArgs a) {
    using acc = typename Codec<DT>::acc;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.nw) return;
    const int x = a.wsite[k];
    I d[18];
    load_offsets<I>((const I*)a.nbr, a.np, x, d);
    acc h[Q];
    gather<DT, I>((const typename Codec<DT>::raw*)a.A, a.np, x, d, h);
    const Mom<acc> m = moments(h);
    acc e[Q];
    heq(m.drho, m.rho, m.ux, m.uy, m.uz, e);
    double S[6] = {0, 0, 0, 0, 0, 0};  // xx yy zz xy xz yz
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double fn = (double)(h[i] - e[i]);
        S[0] += fn * CX[i] * CX[i];
        S[1] += fn * CY[i] * CY[i];
        S[2] += fn * CZ[i] * CZ[i];
        S[3] += fn * CX[i] * CY[i];
        S[4] += fn * CX[i] * CZ[i];
        S[5] += fn * CY[i] * CZ[i];
    }
    const double nx = a.wnormal[3 * k], ny = a.wnormal[3 * k + 1], nz = a.wnormal[3 * k + 2];
    const double c = -a.stress_fac;
    const double tx = c * (S[0] * nx + S[3] * ny + S[4] * nz);
    const double ty = c * (S[3] * nx + S[1] * ny + S[5] * nz);
    const double tz = c * (S[4] * nx + S[5] * ny + S[2] * nz);
    const double tn = tx * nx + ty * ny + tz * nz;
    const double sx = tx - tn * nx, sy = ty - tn * ny, sz = tz - tn * nz;
    const int o = a.i2c ? a.i2c[x - a.first] : x - a.first;
    if (a.wss) a.wss[o] = sqrt(sx * sx + sy * sy + sz * sz);
    if (a.dr) {
        float v = 0.0f;
        if (a.elastic) {
            double dE = ((double)m.drho / 3.0 + a.dp0) * a.kinv[a.wk[k]];
            v = (float)(1.0 + (dE > 0 ? dE : 0.0));
        }
        a.dr[o] = v;
    }
}

// f = feq(rho0, u0) (or given populations) scattered into the slots the
// next pull reads.
template <int DT, typename I>
__global__ __launch_bounds__(256) void k_init(InitArgs a) {
    using raw = typename Codec<DT>::raw;
    using acc = typename Codec<DT>::acc;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int x = a.first + k;
    I d[18];
    load_offsets<I>((const I*)a.nbr, a.np, x, d);
    acc e[Q];
    if (a.f) {
#pragma unroll
        for (int i = 0; i < Q; ++i) e[i] = (acc)(a.f[(int64_t)Q * k + i] - weight(i));
    } else {
        double r = 1.0, ux = 0, uy = 0, uz = 0;
        if (a.rho_u) {
            r = a.rho_u[4 * k];
            ux = a.rho_u[4 * k + 1];
            uy = a.rho_u[4 * k + 2];
            uz = a.rho_u[4 * k + 3];
        } else {
            if (a.rho) r = a.rho[k];
            if (a.u) {
                ux = a.u[3 * k];
                uy = a.u[3 * k + 1];
                uz = a.u[3 * k + 2];
            }
        }
        heq<acc>((acc)(r - 1.0), (acc)r, (acc)ux, (acc)uy, (acc)uz, e);
    }
    raw* A = (raw*)a.A;
    A[x] = Codec<DT>::enc(e[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const I di = d[i - 1];
        const bool redirect = di <= Sentinel<I>::GHOST;
        const int64_t idx = redirect ? (int64_t)dopp(i) * a.np + x : (int64_t)i * a.np + x + di;
        A[idx] = Codec<DT>::enc(e[i]);
    }
}

template <int DT, typename I>
__global__ __launch_bounds__(256) void k_read_pop(PopArgs a) {
    using acc = typename Codec<DT>::acc;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int x = a.first + k;
    I d[18];
    load_offsets<I>((const I*)a.nbr, a.np, x, d);
    acc h[Q];
    gather<DT, I>((const typename Codec<DT>::raw*)a.A, a.np, x, d, h);
#pragma unroll
    for (int i = 0; i < Q; ++i) a.f[(int64_t)Q * k + i] = weight(i) + (double)h[i];
}

// Cycle-to-cycle change of u and p against the stored snapshot; block
// maxima are combined with unsigned atomics on the (non-negative) float bits
// (+inf, the largest of them, marks a non-finite site).
template <int DT, typename I>
__global__ __launch_bounds__(256) void k_delta(DeltaArgs a) {
    using acc = typename Codec<DT>::acc;
    __shared__ float red[4][256];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (k < a.n) {
        const int x = a.first + k;
        I d[18];
        load_offsets<I>((const I*)a.nbr, a.np, x, d);
        acc h[Q];
        gather<DT, I>((const typename Codec<DT>::raw*)a.A, a.np, x, d, h);
        const Mom<acc> m = moments(h);
        const float ux = (float)m.ux, uy = (float)m.uy, uz = (float)m.uz;
        const float dp = (float)(m.drho * (acc)(1.0 / 3.0));  // p - 1/3
        float* sn = a.snap + 4 * (int64_t)k;
        if (a.has_snap) {
            v[0] = fmaxf(fabsf(ux - sn[0]), fmaxf(fabsf(uy - sn[1]), fabsf(uz - sn[2])));
            v[2] = fabsf(dp - sn[3]);
        }
        v[1] = fmaxf(fabsf(ux), fmaxf(fabsf(uy), fabsf(uz)));
        v[3] = fabsf((float)((double)dp + a.dp0));
        // fmaxf drops NaN operands: a non-finite value at any site becomes
        // +inf in all four maxima, which the host reports as divergence
        const bool bad = !(fabsf(ux) <= 3.4e38f && fabsf(uy) <= 3.4e38f && fabsf(uz) <= 3.4e38f &&
                           fabsf(dp) <= 3.4e38f);
        if (bad) {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = __builtin_inff();
        }
        sn[0] = ux;
        sn[1] = uy;
        sn[2] = uz;
        sn[3] = dp;
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][t] = v[c];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][t] = fmaxf(red[c][t], red[c][t + w]);
        }
        __syncthreads();
    }
    if (t < 4) atomicMax(a.maxes + t, __float_as_uint(red[t][0]));
}

// Streaming copy (diagnostic bandwidth reference), grid-stride over 16-byte
// vectors.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                              int64_t n, int nt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (nt)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
    else
        dst[e] = src[e];
}

__global__ void k_zero_u32(unsigned int* p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0u;
}

__global__ void k_permute_rho_u(const float* __restrict__ in, float* __restrict__ out,
                                const int32_t* __restrict__ c2i, int n, int axis) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t j = c2i[k];
    const float* v = in + 4 * (int64_t)k;
    float* w = out + 4 * j;
    w[0] = v[0];
#pragma unroll
    for (int m = 0; m < 3; ++m) w[1 + m] = v[1 + (m == 0 ? axis : (m == axis ? 0 : m))];
}

inline int cdiv(int64_t a, int b) { return (int)((a + b - 1) / b); }

template <template <int, typename> class F, typename... Args>
hipError_t dispatch(int dtype, int ibits, Args&&... args) {
    if (ibits == 16) {
        switch (dtype) {
            case LBM_F64: return F<LBM_F64, int16_t>::run(args...);
            case LBM_F32: return F<LBM_F32, int16_t>::run(args...);
            case LBM_F16DEV: return F<LBM_F16DEV, int16_t>::run(args...);
            case LBM_BF16DEV: return F<LBM_BF16DEV, int16_t>::run(args...);
        }
    } else {
        switch (dtype) {
            case LBM_F64: return F<LBM_F64, int32_t>::run(args...);
            case LBM_F32: return F<LBM_F32, int32_t>::run(args...);
            case LBM_F16DEV: return F<LBM_F16DEV, int32_t>::run(args...);
            case LBM_BF16DEV: return F<LBM_BF16DEV, int32_t>::run(args...);
        }
    }
    return hipErrorInvalidValue;
}

template <int DT, int ADDR>
hipError_t step_launch(const StepArgs& a, int block, hipStream_t s) {
    if (a.spt == 2) {
        // the runtime checked: 32-bit storage, compressed addressing, fused
        // boundary mode, n_int_blocks = ceil(n / 2 block)
        if constexpr (ADDR == ADDR_COMP && DT == LBM_F32) {
            const bool small = (int64_t)Q * a.np * 4 < (1ll << 31);
            const bool ntl = (a.nontemporal & 2) != 0;
            const dim3 grid(a.n_int_blocks);
            if (small && ntl)
                hipLaunchKernelGGL((k_step_pair<DT, true, true>), grid, dim3(block), 0, s, a);
            else if (small)
                hipLaunchKernelGGL((k_step_pair<DT, true, false>), grid, dim3(block), 0, s, a);
            else if (ntl)
                hipLaunchKernelGGL((k_step_pair<DT, false, true>), grid, dim3(block), 0, s, a);
            else
                hipLaunchKernelGGL((k_step_pair<DT, false, false>), grid, dim3(block), 0, s, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    const int nb_blocks = a.fused ? 0 : cdiv(a.nb, block);
    // 32-bit byte offsets when a population buffer is below 2^31 bytes
    const bool small = (int64_t)Q * a.np * (int64_t)sizeof(typename Codec<DT>::raw) < (1ll << 31);
    const dim3 grid(a.n_int_blocks + nb_blocks);
    const bool ntl = (a.nontemporal & 2) != 0;
    if (small && ntl)
        hipLaunchKernelGGL((k_step<DT, ADDR, true, true>), grid, dim3(block), 0, s, a);
    else if (small)
        hipLaunchKernelGGL((k_step<DT, ADDR, true, false>), grid, dim3(block), 0, s, a);
    else if (ntl)
        hipLaunchKernelGGL((k_step<DT, ADDR, false, true>), grid, dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL((k_step<DT, ADDR, false, false>), grid, dim3(block), 0, s, a);
    return hipGetLastError();
}

template <int DT>
hipError_t step_addr(int addressing, const StepArgs& a, int block, hipStream_t s) {
    switch (addressing) {
        case ADDR_T16: return step_launch<DT, ADDR_T16>(a, block, s);
        case ADDR_T32: return step_launch<DT, ADDR_T32>(a, block, s);
        case ADDR_COMP: return step_launch<DT, ADDR_COMP>(a, block, s);
    }
    return hipErrorInvalidValue;
}

template <int DT, typename I>
struct FieldsL {
    static hipError_t run(const FieldArgs& a, hipStream_t s) {
        if (a.n == 0) return hipSuccess;
        hipLaunchKernelGGL((k_fields<DT, I>), dim3(cdiv(a.n, 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};
template <int DT, typename I>
struct WallL {
    static hipError_t run(const WallArgs& a, hipStream_t s) {
        if (a.nw == 0) return hipSuccess;
        hipLaunchKernelGGL((k_wall<DT, I>), dim3(cdiv(a.nw, 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};
template <int DT, typename I>
struct InitL {
    static hipError_t run(const InitArgs& a, hipStream_t s) {
        if (a.n == 0) return hipSuccess;
        hipLaunchKernelGGL((k_init<DT, I>), dim3(cdiv(a.n, 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};
template <int DT, typename I>
struct PopL {
    static hipError_t run(const PopArgs& a, hipStream_t s) {
        if (a.n == 0) return hipSuccess;
        hipLaunchKernelGGL((k_read_pop<DT, I>), dim3(cdiv(a.n, 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};
template <int DT, typename I>
struct DeltaL {
    static hipError_t run(const DeltaArgs& a, hipStream_t s) {
        if (a.n == 0) return hipSuccess;
        hipLaunchKernelGGL((k_delta<DT, I>), dim3(cdiv(a.n, 256)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_step(int dtype, int addressing, const StepArgs& a, int block, hipStream_t s) {
    switch (dtype) {
        case LBM_F64: return step_addr<LBM_F64>(addressing, a, block, s);
        case LBM_F32: return step_addr<LBM_F32>(addressing, a, block, s);
        case LBM_F16DEV: return step_addr<LBM_F16DEV>(addressing, a, block, s);
        case LBM_BF16DEV: return step_addr<LBM_BF16DEV>(addressing, a, block, s);
    }
    return hipErrorInvalidValue;
}
hipError_t launch_fields(int dtype, int ibits, const FieldArgs& a, hipStream_t s) {
    return dispatch<FieldsL>(dtype, ibits, a, s);
}
hipError_t launch_wall(int dtype, int ibits, const WallArgs& a, hipStream_t s) {
    return dispatch<WallL>(dtype, ibits, a, s);
}
hipError_t launch_init(int dtype, int ibits, const InitArgs& a, hipStream_t s) {
    return dispatch<InitL>(dtype, ibits, a, s);
}
hipError_t launch_read_pop(int dtype, int ibits, const PopArgs& a, hipStream_t s) {
    return dispatch<PopL>(dtype, ibits, a, s);
}
hipError_t launch_delta(int dtype, int ibits, const DeltaArgs& a, hipStream_t s) {
    return dispatch<DeltaL>(dtype, ibits, a, s);
}
hipError_t launch_copy(void* dst, const void* src, size_t bytes, int nt, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t blocks = (n + 255) / 256;   // one 16-byte vector per thread
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (u32x4*)dst, (const u32x4*)src, n, nt);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if ((n + 255) / 256 > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u32, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_permute_rho_u(const float* in, float* out, const int32_t* c2i, int n, int axis,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_rho_u, dim3(cdiv(n, 256)), dim3(256), 0, s, in, out, c2i, n, axis);
    return hipGetLastError();
}

}  // namespace lbm
