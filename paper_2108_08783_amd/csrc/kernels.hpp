// Kernel interface shared by the runtime (lbm_api.cpp) and the HIP kernels
// (kernels.hip).  Plain structs only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "d3q19.hpp"

namespace lbm {

// Per-instance wall parameters (Sec. 2.3, 2.4).
struct InstParams {
    double F;       // U_R / U_f
    double dp0;     // 1/3 - P0: Delta E = max(0, (drho/3 + dp0) / k)
    int64_t t0;     // step count at the instance's last initialisation
    int32_t elastic;
    int32_t pad;
};

// Per-iolet drive (Sec. 3): value(t) = a0 (1 + amp sin(2 pi t/period + phase)).
struct IoletParams {
    double a0, amp, inv_period, phase;
    double dir[3];  // velocity: unit direction; density: inward normal (if project)
    int32_t kind;   // 0 density, 1 velocity
    int32_t pad;    // density: 1 keeps only the velocity along dir
};

// Elastic-wall coefficients of one boundary record (Sec. 2.3, 2.4): with
// drho = rho - 1, Delta E = max(0, drho c1 + c0) and s = (F + Delta E) /
// (1 + Delta E); c1 = 1/(3k), c0 = (1/3 - P0)/k of the site's segment.
struct WallCoef {
    double c1, c0, F, pad;
};

// The same in single precision, read by float accumulation: no conversion
// after the load, so a load issued ahead of the gathers need not complete
// before they are issued (and half the bytes).
struct WallCoefF {
    float c1, c0, F, pad;
};

struct StepArgs {
    const void* A;          // populations read (deviation f - w, SoA, plane stride np)
    void* B;                // populations written
    const void* nbr;        // 18 planes of neighbour offsets (width I)
    int64_t np;             // plane stride in elements
    int32_t n;              // fluid sites
    int32_t n_int_blocks;   // blocks of the interior part
    int32_t nb;             // boundary sites
    int32_t xcd_remap;      // 0 off, 1 one site range per XCD, g >= 2: runs of g blocks
    int32_t nontemporal;
    int32_t clock_in;       // clock slot read this step; the other is written
    int32_t fused;          // 1: boundary links applied inside the update blocks
    int32_t spt;            // sites per lane: 1, or 2 (tiles of 128 sites, 32-bit storage)
    double omega;           // 1 / tau
    const int32_t* bj;      // record ids of sites with boundary-pass links (compacted mode)
    const int32_t* rsite;   // record id -> site
    const int32_t* bidx;    // per site: record id, -1 for interior sites (table addressing)
    const uint32_t* bwall;  // elastic wall link mask | inst << 19
    const uint32_t* bio;    // iolet link mask | iolet slot << 19
    const WallCoef* bq;     // elastic-wall coefficients per record
    const WallCoefF* bqf;   // the same in single precision
    const float* bw;        // iolet profile weight
    const InstParams* ip;
    const IoletParams* iop;
    int64_t* clock;         // [2] steps executed before the current one
    // compressed addressing (see Compressed in builder.hpp)
    const WfRec* wf;         // one record per 64 sites
    const int32_t* stretch;  // 8 per stretch
    const uint32_t* nfm;     // per irregular site: non-fluid link mask
    const int32_t* exc;      // 18 planes x n_exc_pad: offsets of exceptional sites
    int64_t n_exc_pad;
};

// Addressing of the update kernel: per-site offset table of 16 or 32 bits,
// or compressed (stretches, link masks, exceptional-site table).
enum { ADDR_T16 = 16, ADDR_T32 = 32, ADDR_COMP = 0 };

struct FieldArgs {
    const void* A;
    const void* nbr;
    int64_t np;
    int32_t first;          // first site of the instance
    int32_t n;              // sites of the instance
    double omega;
    double* rho;            // n
    double* u;              // 3n
    // optional: outputs at canonical positions i2c[k] with velocity
    // components 0 and `axis` exchanged (NULL: internal order and frame)
    const int32_t* i2c = nullptr;
    int32_t axis = 0;
    unsigned int* bad = nullptr;   // optional: set to 1 if a site is not finite
};

struct WallArgs {
    const void* A;
    const void* nbr;
    int64_t np;
    int32_t first;          // first site of the instance
    int32_t nw;             // wall sites of the instance
    const int32_t* wsite;   // wall-site list of the instance
    const double* wnormal;  // 3 per wall site
    const int32_t* wk;      // stiffness index per wall site
    double omega;
    double stress_fac;      // 1 - 1/(2 tau)
    double dp0;
    int32_t elastic;
    const double* kinv;
    double* wss;            // n (indexed by site - first)
    float* dr;              // n
    const int32_t* i2c = nullptr;  // optional: write at i2c[site - first]
};

struct InitArgs {
    void* A;
    const void* nbr;
    int64_t np;
    int32_t first, n;
    const double* rho;      // n, or NULL
    const double* u;        // 3n, or NULL
    const float* rho_u;     // 4n (device float input), or NULL
    const double* f;        // 19n populations (checkpoint write), or NULL
};

struct PopArgs {
    const void* A;
    const void* nbr;
    int64_t np;
    int32_t first, n;
    double* f;              // 19n
};

struct DeltaArgs {
    const void* A;
    const void* nbr;
    int64_t np;
    int32_t first, n;
    double dp0;             // 1/3 - P0
    float* snap;            // 4n: ux, uy, uz, p - 1/3 of the previous call
    int32_t has_snap;
    unsigned int* maxes;    // 4: max|du|, max|u|, max|dp|, max|p - P0| (float bits)
};

// Launchers (kernels.hip).  dtype: enum lbm_dtype; ibits: 16 or 32.
hipError_t launch_step(int dtype, int addressing, const StepArgs& a, int block, hipStream_t s);
hipError_t launch_fields(int dtype, int ibits, const FieldArgs& a, hipStream_t s);
hipError_t launch_wall(int dtype, int ibits, const WallArgs& a, hipStream_t s);
hipError_t launch_init(int dtype, int ibits, const InitArgs& a, hipStream_t s);
hipError_t launch_read_pop(int dtype, int ibits, const PopArgs& a, hipStream_t s);
hipError_t launch_delta(int dtype, int ibits, const DeltaArgs& a, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, int64_t n, hipStream_t s);
// out[4 c2i[k] + m] = in[4 k + m'] for k < n: site k of a canonical-order
// (rho, ux, uy, uz) array goes to internal site c2i[k], with velocity
// components x and `axis` (1 or 2) exchanged.
hipError_t launch_permute_rho_u(const float* in, float* out, const int32_t* c2i, int n, int axis,
                                hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, int nt, hipStream_t s);

}  // namespace lbm
