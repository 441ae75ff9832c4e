// D3Q19 velocity set and weights (Sec. 2.1): rest; the six axis
// directions (+x,-x,+y,-y,+z,-z); the twelve face diagonals in the (x,y),
// (x,z), (y,z) families, each ordered (+,+), (-,-), (+,-), (-,+).  Opposite
// directions are adjacent pairs (1,2), (3,4), ..., (17,18).
#pragma once

#include <cstdint>

namespace lbm {

constexpr int Q = 19;

#if defined(__HIPCC__)
#define LBM_HD __host__ __device__
#else
#define LBM_HD
#endif

constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

LBM_HD constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

LBM_HD constexpr double weight(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Neighbour-table sentinels: the link's upstream voxel is not fluid.
//   BB    : bounce-back, the site reads its own opposite slot;
//   GHOST : the site is updated by the boundary pass, which writes the
//           link's value into that same opposite slot.
template <typename I>
struct Sentinel;
template <>
struct Sentinel<int32_t> {
    static constexpr int32_t BB = INT32_MIN;
    static constexpr int32_t GHOST = INT32_MIN + 1;
    static constexpr int64_t MAXABS = INT32_MAX;
};
template <>
struct Sentinel<int16_t> {
    static constexpr int16_t BB = INT16_MIN;
    static constexpr int16_t GHOST = INT16_MIN + 1;
    static constexpr int64_t MAXABS = INT16_MAX;
};

// Per-wavefront record of the compressed addressing (layout shared by the
// host builder and the update kernel; fields described in builder.hpp).
struct alignas(16) WfRec {
    int32_t cur, firr, fexc, pad;
    uint64_t smask, imask, emask, pad2;
};
static_assert(sizeof(WfRec) == 48, "wavefront record layout");

}  // namespace lbm
