// Native runtime and C ABI of the library (declared in include/lbm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "builder.hpp"
#include "d3q19.hpp"
#include "kernels.hpp"

using namespace lbm;

namespace {

thread_local std::string g_last_error = "";

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct InstState {
    int mode = LBM_WALL_BOUNCEBACK;
    double F = 0.0, P0 = 1.0 / 3.0;
    std::vector<double> k;      // per segment
    std::vector<double> Fseg;   // slip ratio per segment
    int64_t t0 = 0;
    std::vector<IoletParams> iolets;
    std::vector<uint8_t> iolet_set;
    DevBuf snap;                // periodicity snapshot
    bool has_snap = false;
};

struct TuneKey {
    int64_t n, nb;
    int dtype;
    bool operator<(const TuneKey& o) const {
        return std::tie(n, nb, dtype) < std::tie(o.n, o.nb, o.dtype);
    }
};
struct TuneVal {
    int block, ibits, xcd, nt, fused, spt;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune_cache;

constexpr int GRAPH_STEPS = 128;  // even

// Staging memory of lbm_read_fields_noalloc: one array per device that the
// library runs on, held until the process ends.  Host code uses only the
// device address obtained for it with hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Looks up the device address of `scratch` on the current device, once per
// device.  Returns nullptr (with the HIP error in *err) on failure.
void* scratch_ptr(int dev, hipError_t* err) {
    *err = hipSuccess;
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

struct lbm_ctx {
    mutable std::string err;  // last error (also set by the const queries)
    Plan plan;
    int dtype = LBM_F32;
    double tau = 1.0;
    size_t esize = 4;
    int64_t np = 0;
    std::vector<InstState> ist;
    std::vector<int> seg_off, iolet_off;
    // site order: per instance the axis exchanged with x (0 none) and, for
    // exchanged instances, canonical local site -> internal local site
    std::vector<int> axis;
    std::vector<std::vector<int32_t>> c2i;
    int n_iolet_slots = 0, n_k = 0;
    // device memory
    std::vector<DevBuf> owned;
    void* buf[2] = {nullptr, nullptr};
    void* nbr32 = nullptr;
    void* nbr16 = nullptr;
    bool have16 = false;
    // boundary records, one per irregular site (any non-fluid link)
    int32_t* bj = nullptr;     // record ids with boundary-pass links
    int32_t* rsite = nullptr;  // record id -> site
    int32_t* bidx = nullptr;   // per site: record id, -1 if interior
    uint32_t* bwall = nullptr;
    uint32_t* bio = nullptr;
    int32_t* bk = nullptr;
    WallCoef* bq = nullptr;
    WallCoefF* bqf = nullptr;
    std::vector<int32_t> rec_k, rec_inst;  // per record: stiffness index, instance
    float* bw = nullptr;
    int64_t nb = 0, n_irr = 0;
    // compressed addressing
    WfRec* wf = nullptr;
    int32_t* stretch = nullptr;
    uint32_t* nfm = nullptr;
    int32_t* exc = nullptr;
    int64_t n_exc = 0, n_exc_pad = 0, n_stretch = 0;
    Compressed comp;        // host copy of the compressed addressing
    int32_t* wsite = nullptr;
    double* wnormal = nullptr;
    int32_t* wk = nullptr;
    InstParams* ip = nullptr;
    IoletParams* iop = nullptr;
    double* kinv = nullptr;
    int64_t* clock = nullptr;
    unsigned int* maxes = nullptr;
    DevBuf scratch;
    // per instance whose fast axis is exchanged: internal local site ->
    // canonical local site, on the device (read-out without host staging)
    std::vector<int32_t*> i2c_dev;
    int device = 0;            // the device the context was created on
    void* noalloc = nullptr;   // device address of that device's staging array
    // state
    int64_t step = 0;
    bool tables_dirty = true, params_dirty = true;
    // launch configuration
    int block = 256, ibits = 32, use_graph = 1, xcd = 1, nt = 0, fused = 1, spt = 1;
    hipStream_t stream = nullptr;      // every operation of the context is enqueued here
    bool own_stream = true;            // false: the caller's stream (not destroyed)
    hipStream_t cap_stream = nullptr;  // private stream the step graphs are captured on
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by buffer parity at start
    int64_t device_bytes = 0;
    // caller's device allocator (NULL: hipMalloc / hipFree)
    lbm_alloc_fn alloc_fn = nullptr;
    lbm_free_fn free_fn = nullptr;
    void* alloc_user = nullptr;
};

namespace {

int fail(const lbm_ctx* c, int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_last_error = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int dalloc(lbm_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (c->alloc_fn) {
        *p = c->alloc_fn(bytes, c->alloc_user);
        if (!*p) return fail(c, LBM_ENOMEM, "caller allocator returned NULL for %zu bytes", bytes);
        if ((uintptr_t)*p % 256) {
            c->free_fn(*p, c->alloc_user);
            *p = nullptr;
            return fail(c, LBM_EINVAL, "caller allocator returned a block not aligned to 256 bytes");
        }
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, LBM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    c->owned.push_back({*p, bytes});
    c->device_bytes += (int64_t)bytes;
    return LBM_OK;
}

// Returns a block to whoever allocated it.  Blocks may still be in use by
// work enqueued on the context's stream, so the stream is drained first.
void release(lbm_ctx* c, void* p) {
    if (c->free_fn)
        c->free_fn(p, c->alloc_user);
    else
        (void)hipFree(p);
}

void dfree(lbm_ctx* c, void* p) {
    if (!p) return;
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i].p == p) {
            c->device_bytes -= (int64_t)c->owned[i].bytes;
            c->owned.erase(c->owned.begin() + i);
            break;
        }
    if (c->stream || !c->own_stream) (void)hipStreamSynchronize(c->stream);
    release(c, p);
}

// Device buffer released on every exit path of the scope that owns it.
struct ScopedDev {
    lbm_ctx* c;
    void* p = nullptr;
    explicit ScopedDev(lbm_ctx* ctx) : c(ctx) {}
    ScopedDev(const ScopedDev&) = delete;
    ScopedDev& operator=(const ScopedDev&) = delete;
    ~ScopedDev() { dfree(c, p); }
};

int ensure_scratch(lbm_ctx* c, size_t bytes) {
    if (c->scratch.bytes >= bytes) return LBM_OK;
    dfree(c, c->scratch.p);
    c->scratch = DevBuf();
    int rc = dalloc(c, &c->scratch.p, bytes);
    if (rc) return rc;
    c->scratch.bytes = bytes;
    return LBM_OK;
}

void drop_graphs(lbm_ctx* c) {
    for (auto& g : c->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

std::vector<int> modes(const lbm_ctx* c) {
    std::vector<int> m(c->ist.size());
    for (size_t i = 0; i < m.size(); ++i) m[i] = c->ist[i].mode;
    return m;
}

int upload(lbm_ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return LBM_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Rebuilds the device neighbour tables and boundary list after a change of
// wall mode (bounce-back links redirect inside the update; elastic links go
// through the boundary pass).
int sync_tables(lbm_ctx* c) {
    if (!c->tables_dirty) return LBM_OK;
    const std::vector<int> m = modes(c);
    if (c->have16) {
        std::vector<int16_t> t16;
        build_device_nbr<int16_t>(c->plan, m, c->np, t16);
        int rc = upload(c, c->nbr16, t16.data(), t16.size() * 2);
        if (rc) return rc;
    }
    std::vector<int32_t> t32;
    build_device_nbr<int32_t>(c->plan, m, c->np, t32);
    BoundaryList bl;
    build_boundary(c->plan, m, c->seg_off, c->iolet_off, bl);
    if ((int64_t)bl.site.size() != c->n_irr) return fail(c, LBM_ESTATE, "irregular-site set changed");
    // the compressed form was built and checked against the full table when
    // the buffers were sized; only its mode-dependent parts change here
    Compressed& cm = c->comp;
    refresh_compressed(bl, t32, c->np, cm);
    {
        int rc = upload(c, c->nbr32, t32.data(), t32.size() * 4);
        if (rc) return rc;
    }
    const int64_t ni = c->n_irr;
    c->nb = (int64_t)bl.ghost.size();
    int rc = upload(c, c->bj, bl.ghost.data(), c->nb * 4);
    rc = rc ? rc : upload(c, c->rsite, bl.site.data(), ni * 4);
    rc = rc ? rc : upload(c, c->bidx, bl.rec_of_site.data(), c->plan.N * 4);
    rc = rc ? rc : upload(c, c->bwall, bl.wall.data(), ni * 4);
    rc = rc ? rc : upload(c, c->bio, bl.io.data(), ni * 4);
    rc = rc ? rc : upload(c, c->bk, bl.kidx.data(), ni * 4);
    rc = rc ? rc : upload(c, c->bw, bl.weight.data(), ni * 4);
    const int64_t nwf = c->np / 64;
    rc = rc ? rc : upload(c, c->wf, cm.wf.data(), nwf * sizeof(WfRec));
    rc = rc ? rc : upload(c, c->stretch, cm.stretch.data(), cm.stretch.size() * 4);
    rc = rc ? rc : upload(c, c->nfm, cm.nfm.data(), cm.nfm.size() * 4);
    rc = rc ? rc : upload(c, c->exc, cm.exc.data(), cm.exc.size() * 4);
    if (rc) return rc;
    c->tables_dirty = false;
    drop_graphs(c);
    return LBM_OK;
}

int sync_params(lbm_ctx* c) {
    if (!c->params_dirty) return LBM_OK;
    const int ni = (int)c->ist.size();
    std::vector<InstParams> ip(ni);
    std::vector<IoletParams> iop(std::max(1, c->n_iolet_slots));
    std::vector<double> kinv(std::max(1, c->n_k), 1.0);
    for (int k = 0; k < ni; ++k) {
        const InstState& s = c->ist[k];
        ip[k].F = s.F;
        ip[k].dp0 = 1.0 / 3.0 - s.P0;
        ip[k].t0 = s.t0;
        ip[k].elastic = s.mode == LBM_WALL_ELASTIC;
        ip[k].pad = 0;
        for (size_t j = 0; j < s.k.size(); ++j) kinv[c->seg_off[k] + j] = 1.0 / s.k[j];
        for (size_t j = 0; j < s.iolets.size(); ++j) iop[c->iolet_off[k] + j] = s.iolets[j];
    }
    int rc = upload(c, c->ip, ip.data(), ip.size() * sizeof(InstParams));
    rc = rc ? rc : upload(c, c->iop, iop.data(), iop.size() * sizeof(IoletParams));
    rc = rc ? rc : upload(c, c->kinv, kinv.data(), kinv.size() * sizeof(double));
    {
        // elastic-wall coefficients per boundary record
        std::vector<WallCoef> bq(std::max<size_t>(1, c->rec_k.size()));
        for (size_t j = 0; j < c->rec_k.size(); ++j) {
            const InstState& s = c->ist[c->rec_inst[j]];
            const double ki = kinv[c->rec_k[j]];
            bq[j].c1 = ki / 3.0;
            bq[j].c0 = (1.0 / 3.0 - s.P0) * ki;
            bq[j].F = s.Fseg[c->rec_k[j] - c->seg_off[c->rec_inst[j]]];
            bq[j].pad = 0.0;
        }
        rc = rc ? rc : upload(c, c->bq, bq.data(), c->rec_k.size() * sizeof(WallCoef));
        // single-precision copy (rounded to nearest, as a conversion on the
        // device would round)
        std::vector<WallCoefF> bqf(bq.size());
        for (size_t j = 0; j < bq.size(); ++j)
            bqf[j] = WallCoefF{(float)bq[j].c1, (float)bq[j].c0, (float)bq[j].F, 0.0f};
        rc = rc ? rc : upload(c, c->bqf, bqf.data(), c->rec_k.size() * sizeof(WallCoefF));
    }
    if (rc) return rc;
    c->params_dirty = false;
    return LBM_OK;
}

int check_ready(lbm_ctx* c) {
    for (size_t k = 0; k < c->ist.size(); ++k) {
        const InstanceGeom& g = c->plan.inst[k];
        for (int id = 0; id < g.n_iolet; ++id)
            if (g.iolet_used[id] && !c->ist[k].iolet_set[id])
                return fail(c, LBM_ESTATE, "instance %zu: iolet %d is used but has no parameters",
                            k, id);
    }
    int rc = sync_tables(c);
    return rc ? rc : sync_params(c);
}

const void* nbr_ptr(const lbm_ctx* c) { return c->ibits == 16 ? c->nbr16 : c->nbr32; }
// read-out, initialisation and checkpoint kernels always use the 32-bit table
const void* nbr_rd(const lbm_ctx* c) { return c->nbr32; }

StepArgs step_args(const lbm_ctx* c, int parity) {
    StepArgs a;
    a.A = c->buf[parity];
    a.B = c->buf[parity ^ 1];
    a.nbr = nbr_ptr(c);
    a.np = c->np;
    a.n = (int32_t)c->plan.N;
    a.n_int_blocks = (int32_t)((c->plan.N + (int64_t)c->block * c->spt - 1) / ((int64_t)c->block * c->spt));
    a.nb = (int32_t)c->nb;
    a.xcd_remap = c->xcd;
    a.nontemporal = c->nt;
    a.clock_in = parity;
    a.fused = c->fused;
    a.spt = c->spt;
    a.omega = 1.0 / c->tau;
    a.bj = c->bj;
    a.rsite = c->rsite;
    a.bidx = c->bidx;
    a.bwall = c->bwall;
    a.bio = c->bio;
    a.bq = c->bq;
    a.bqf = c->bqf;
    a.bw = c->bw;
    a.ip = c->ip;
    a.iop = c->iop;
    a.clock = c->clock;
    a.wf = c->wf;
    a.stretch = c->stretch;
    a.nfm = c->nfm;
    a.exc = c->exc;
    a.n_exc_pad = c->n_exc_pad;
    return a;
}

int enqueue_step(lbm_ctx* c) {
    const int parity = (int)(c->step & 1);
    hipError_t e = launch_step(c->dtype, c->ibits, step_args(c, parity), c->block, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "update launch failed: %s", hipGetErrorString(e));
    c->step += 1;
    return LBM_OK;
}

int get_graph(lbm_ctx* c, int parity, hipGraphExec_t* out) {
    if (c->graph[parity]) {
        *out = c->graph[parity];
        return LBM_OK;
    }
    // captured on a private stream (the caller's stream may be the null
    // stream, which cannot be captured) and launched on the context's stream
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int k = 0; k < GRAPH_STEPS && le == hipSuccess; ++k)
        le = launch_step(c->dtype, c->ibits, step_args(c, (parity + k) & 1), c->block, c->cap_stream);
    hipError_t ce = hipStreamEndCapture(c->cap_stream, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(c, LBM_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ce));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(c, LBM_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
    c->graph[parity] = ex;
    *out = ex;
    return LBM_OK;
}

int run_steps(lbm_ctx* c, int64_t n) {
    while (n > 0) {
        if (c->use_graph && n >= GRAPH_STEPS) {
            hipGraphExec_t ex;
            int rc = get_graph(c, (int)(c->step & 1), &ex);
            if (rc) return rc;
            HIP_TRY(c, hipGraphLaunch(ex, c->stream));
            c->step += GRAPH_STEPS;
            n -= GRAPH_STEPS;
        } else {
            int rc = enqueue_step(c);
            if (rc) return rc;
            n -= 1;
        }
    }
    return LBM_OK;
}

int check_inst(lbm_ctx* c, int inst) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (inst < 0 || inst >= (int)c->ist.size())
        return fail(c, LBM_EINVAL, "instance %d out of range [0, %zu)", inst, c->ist.size());
    return LBM_OK;
}

size_t elem_size(int dtype) {
    switch (dtype) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16DEV:
        case LBM_BF16DEV: return 2;
    }
    return 0;
}

// Component of the caller's frame that internal component m holds when axes
// x and `axis` are exchanged (an involution).
inline int comp_src(int m, int axis) { return axis == 0 ? m : (m == 0 ? axis : (m == axis ? 0 : m)); }

// Direction of the caller's frame whose velocity is internal direction i's
// with the components exchanged (an involution on 0..18).
int dir_swap(int i, int axis) {
    if (axis == 0) return i;
    const int v[3] = {CX[i], CY[i], CZ[i]};
    const int w[3] = {v[comp_src(0, axis)], v[comp_src(1, axis)], v[comp_src(2, axis)]};
    for (int j = 0; j < Q; ++j)
        if (CX[j] == w[0] && CY[j] == w[1] && CZ[j] == w[2]) return j;
    return -1;
}

// LBM_FAST_AXIS: "x", "y" or "z" forces the fast axis of every instance;
// unset, empty or "auto" lets the library choose.  -2 for anything else.
int forced_axis() {
    const char* e = std::getenv("LBM_FAST_AXIS");
    if (!e || !*e || !std::strcmp(e, "auto")) return -1;
    if (!std::strcmp(e, "x")) return 0;
    if (!std::strcmp(e, "y")) return 1;
    if (!std::strcmp(e, "z")) return 2;
    return -2;
}

int init_instance(lbm_ctx* c, int inst, const double* rho, const double* u, const float* rho_u_dev,
                  const double* f) {
    int rc = sync_tables(c);
    if (rc) return rc;
    const InstanceGeom& g = c->plan.inst[inst];
    const int64_t n = g.n;
    // caller's order and frame -> internal
    const int ax = c->axis[inst];
    std::vector<double> prho, pu, pf;
    if (ax) {
        const std::vector<int32_t>& m = c->c2i[inst];
        if (f) {
            pf.resize((size_t)n * Q);
            int dm[Q];
            for (int i = 0; i < Q; ++i) dm[i] = dir_swap(i, ax);
            for (int64_t k = 0; k < n; ++k)
                for (int i = 0; i < Q; ++i) pf[(size_t)m[k] * Q + i] = f[(size_t)k * Q + dm[i]];
            f = pf.data();
        }
        if (rho) {
            prho.resize((size_t)n);
            for (int64_t k = 0; k < n; ++k) prho[(size_t)m[k]] = rho[k];
            rho = prho.data();
        }
        if (u) {
            pu.resize((size_t)n * 3);
            for (int64_t k = 0; k < n; ++k)
                for (int a = 0; a < 3; ++a) pu[(size_t)m[k] * 3 + a] = u[3 * k + comp_src(a, ax)];
            u = pu.data();
        }
    }
    InitArgs a;
    a.A = c->buf[c->step & 1];
    a.nbr = nbr_rd(c);
    a.np = c->np;
    a.first = (int32_t)g.offset;
    a.n = (int32_t)n;
    a.rho = nullptr;
    a.u = nullptr;
    a.rho_u = rho_u_dev;
    a.f = nullptr;
    size_t need = 0;
    if (f) need = (size_t)n * Q * 8;
    else need = (size_t)n * 4 * 8;
    rc = ensure_scratch(c, need);
    if (rc) return rc;
    double* s = (double*)c->scratch.p;
    if (ax && rho_u_dev) {
        // the device array is in the caller's order: permute it on the device
        // (n * 16 bytes of permuted values, then n * 4 bytes of site map)
        float* perm = (float*)c->scratch.p;
        int32_t* map = (int32_t*)(perm + 4 * n);
        HIP_TRY(c, hipMemcpyAsync(map, c->c2i[inst].data(), (size_t)n * 4, hipMemcpyHostToDevice,
                                  c->stream));
        hipError_t pe = launch_permute_rho_u(rho_u_dev, perm, map, (int)n, ax, c->stream);
        if (pe != hipSuccess)
            return fail(c, LBM_EDEVICE, "permute launch failed: %s", hipGetErrorString(pe));
        a.rho_u = perm;
    }
    if (f) {
        HIP_TRY(c, hipMemcpyAsync(s, f, (size_t)n * Q * 8, hipMemcpyHostToDevice, c->stream));
        a.f = s;
    } else if (!rho_u_dev) {
        if (rho) {
            HIP_TRY(c, hipMemcpyAsync(s, rho, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
            a.rho = s;
        }
        if (u) {
            HIP_TRY(c, hipMemcpyAsync(s + n, u, (size_t)n * 24, hipMemcpyHostToDevice, c->stream));
            a.u = s + n;
        }
    }
    hipError_t e = launch_init(c->dtype, 32, a, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "init launch failed: %s", hipGetErrorString(e));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(const lbm_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_last_error.c_str();
}

int lbm_copy_probe(void* dst, const void* src, size_t bytes, int nontemporal, int reps,
                   void* stream, double* ms) {
    if (!dst || !src || !ms || bytes == 0 || bytes % 16 || reps < 1 ||
        ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(nullptr, LBM_EINVAL, "lbm_copy_probe: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(nullptr, launch_copy(dst, src, bytes, nontemporal, s));  // warm-up
    HIP_TRY(nullptr, hipEventCreate(&e0));
    HIP_TRY(nullptr, hipEventCreate(&e1));
    HIP_TRY(nullptr, hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIP_TRY(nullptr, launch_copy(dst, src, bytes, nontemporal, s));
    HIP_TRY(nullptr, hipEventRecord(e1, s));
    HIP_TRY(nullptr, hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(nullptr, hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / reps;
    return LBM_OK;
}

int lbm_plan_export(const lbm_instance_desc* inst, int n_inst, const int* wall_mode,
                    int64_t* counts, int32_t* nbr, int32_t* boundary, uint32_t* bmask) {
    Plan p;
    std::string e = build_plan(inst, n_inst, p);
    if (!e.empty()) return fail(nullptr, LBM_EINVAL, "%s", e.c_str());
    std::vector<int> m(n_inst, LBM_WALL_BOUNCEBACK), so(n_inst, 0), io(n_inst, 0);
    if (wall_mode)
        for (int k = 0; k < n_inst; ++k) m[k] = wall_mode[k];
    BoundaryList bl;
    build_boundary(p, m, so, io, bl);
    if (counts) {
        counts[0] = p.N;
        counts[1] = (int64_t)bl.ghost.size();
        counts[2] = (int64_t)p.wall_site.size();
        counts[3] = p.n_wall_links;
        counts[4] = p.n_iolet_links;
        counts[5] = p.max_abs_offset;
    }
    if (nbr) {
        std::vector<int32_t> t;
        build_device_nbr<int32_t>(p, m, p.N, t);
        std::memcpy(nbr, t.data(), t.size() * 4);
    }
    for (size_t j = 0; j < bl.ghost.size(); ++j) {
        const int32_t id = bl.ghost[j];
        if (boundary) boundary[j] = bl.site[id];
        if (bmask) bmask[j] = (bl.wall[id] & 0x7FFFEu) | (bl.io[id] & 0x7FFFEu);
    }
    return LBM_OK;
}

int lbm_plan_compressed(const lbm_instance_desc* inst, int n_inst, const int* wall_mode,
                        int64_t* stats) {
    if (!stats) return fail(nullptr, LBM_EINVAL, "stats is NULL");
    Plan p;
    std::string e = build_plan(inst, n_inst, p);
    if (!e.empty()) return fail(nullptr, LBM_EINVAL, "%s", e.c_str());
    std::vector<int> m(n_inst, LBM_WALL_BOUNCEBACK), so(n_inst, 0), io(n_inst, 0);
    if (wall_mode)
        for (int k = 0; k < n_inst; ++k) m[k] = wall_mode[k];
    const int64_t np = std::max<int64_t>(256, (p.N + 255) / 256 * 256);
    std::vector<int32_t> t32;
    build_device_nbr<int32_t>(p, m, np, t32);
    BoundaryList bl;
    build_boundary(p, m, so, io, bl);
    Compressed cm;
    e = build_compressed(p, bl, t32, np, cm);
    if (!e.empty()) return fail(nullptr, LBM_EINVAL, "%s", e.c_str());
    // the runtime builds the form once for all-bounce-back walls and then
    // refreshes it for the actual modes: both routes must agree
    {
        const std::vector<int> m0(n_inst, LBM_WALL_BOUNCEBACK);
        std::vector<int32_t> t0;
        build_device_nbr<int32_t>(p, m0, np, t0);
        BoundaryList b0;
        build_boundary(p, m0, so, io, b0);
        Compressed c0;
        e = build_compressed(p, b0, t0, np, c0);
        if (!e.empty()) return fail(nullptr, LBM_EINVAL, "%s", e.c_str());
        refresh_compressed(bl, t32, np, c0);
        if (c0.nfm != cm.nfm || c0.exc != cm.exc || c0.stretch != cm.stretch ||
            c0.wf.size() != cm.wf.size() ||
            std::memcmp(c0.wf.data(), cm.wf.data(), cm.wf.size() * sizeof(WfRec)) != 0)
            return fail(nullptr, LBM_EINVAL, "compressed addressing: refresh for the wall modes "
                                             "differs from a direct build");
    }
    stats[0] = cm.n_stretch;
    stats[1] = cm.n_irr;
    stats[2] = cm.n_exc;
    stats[3] = (int64_t)cm.wf.size();
    return LBM_OK;
}

int lbm_fast_axis(const lbm_instance_desc* inst, int n_inst, int* axis) {
    if (!inst || !axis || n_inst <= 0) return fail(nullptr, LBM_EINVAL, "invalid arguments");
    const int forced = forced_axis();
    if (forced == -2) return fail(nullptr, LBM_EINVAL, "LBM_FAST_AXIS must be x, y, z or auto");
    for (int k = 0; k < n_inst; ++k) axis[k] = choose_fast_axis(inst[k], forced);
    return LBM_OK;
}

int lbm_create_geometry(lbm_ctx** out, const lbm_instance_desc* inst, int n_inst, int dtype,
                        double tau) {
    return lbm_create_geometry_ex(out, inst, n_inst, dtype, tau, nullptr);
}

int lbm_create_geometry_ex(lbm_ctx** out, const lbm_instance_desc* inst, int n_inst, int dtype,
                           double tau, const lbm_resources* res) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    if (res && (!res->alloc) != (!res->free))
        return fail(nullptr, LBM_EINVAL, "the allocator needs both alloc and free (or neither)");
    *out = nullptr;
    if (!(tau > 0.5)) return fail(nullptr, LBM_EINVAL, "tau must exceed 1/2 (got %g)", tau);
    if (elem_size(dtype) == 0) return fail(nullptr, LBM_EINVAL, "unknown dtype %d", dtype);
    if (n_inst <= 0 || n_inst > 8191) return fail(nullptr, LBM_EINVAL, "n_inst out of range");
    const int forced = forced_axis();
    if (forced == -2) return fail(nullptr, LBM_EINVAL, "LBM_FAST_AXIS must be x, y, z or auto");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "out of host memory");
    if (res) {
        c->alloc_fn = res->alloc;
        c->free_fn = res->free;
        c->alloc_user = res->user;
        if (res->use_stream) {
            c->stream = (hipStream_t)res->stream;
            c->own_stream = false;
        }
    }
    // site order: instances whose fluid runs are longest along y or z are
    // stored with that axis exchanged for x
    std::vector<lbm_instance_desc> descs(inst, inst + n_inst);
    std::vector<SwappedGeom> swapped((size_t)n_inst);
    c->axis.assign((size_t)n_inst, 0);
    c->c2i.resize((size_t)n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const int a = choose_fast_axis(inst[k], forced);
        if (!a || !inst[k].labels || inst[k].nx <= 0 || inst[k].ny <= 0 || inst[k].nz <= 0) continue;
        c->axis[k] = a;
        swap_axes(inst[k], a, swapped[k]);
        descs[k] = swapped[k].desc;
        site_map(inst[k], a, swapped[k], c->c2i[k]);
    }
    std::string e = build_plan(descs.data(), n_inst, c->plan);
    swapped.clear();
    if (!e.empty()) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "%s", e.c_str());
    }
    c->dtype = dtype;
    c->tau = tau;
    c->esize = elem_size(dtype);
    c->np = (c->plan.N + 255) / 256 * 256;
    c->ist.resize(n_inst);
    c->seg_off.resize(n_inst);
    c->iolet_off.resize(n_inst);
    int so = 0, io = 0;
    for (int k = 0; k < n_inst; ++k) {
        const InstanceGeom& g = c->plan.inst[k];
        InstState& s = c->ist[k];
        s.k.assign(g.n_seg, 1.0);
        s.Fseg.assign(g.n_seg, 0.0);
        s.iolets.assign(std::max(g.n_iolet, 0), IoletParams());
        s.iolet_set.assign(std::max(g.n_iolet, 0), 0);
        c->seg_off[k] = so;
        c->iolet_off[k] = io;
        so += g.n_seg;
        io += std::max(g.n_iolet, 0);
    }
    c->n_k = so;
    c->n_iolet_slots = io;
    if (io >= 8192) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "too many iolets (%d) in one context", io);
    }
    c->have16 = c->plan.max_abs_offset <= Sentinel<int16_t>::MAXABS - 1;
    c->ibits = 0;  // compressed addressing by default
    if (c->own_stream) {
        hipError_t he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (he != hipSuccess) {
            delete c;
            return fail(nullptr, LBM_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(he));
        }
    }
    int rc = 0;
    {
        hipError_t de = hipGetDevice(&c->device);
        hipError_t se = de;
        if (de == hipSuccess) c->noalloc = scratch_ptr(c->device, &se);
        if (de != hipSuccess || se != hipSuccess) {
            if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(nullptr, LBM_EDEVICE, "device set-up failed: %s",
                        hipGetErrorString(de != hipSuccess ? de : se));
        }
    }
    const size_t pop_bytes = (size_t)Q * c->np * c->esize;
    rc = rc ? rc : dalloc(c, &c->buf[0], pop_bytes);
    rc = rc ? rc : dalloc(c, &c->buf[1], pop_bytes);
    rc = rc ? rc : dalloc(c, &c->nbr32, (size_t)18 * c->np * 4);
    if (!rc) {
        // sizes of the boundary records and of the compressed addressing do
        // not depend on the wall modes; build once to size the buffers
        const std::vector<int> m0(n_inst, LBM_WALL_BOUNCEBACK);
        std::vector<int32_t> t32;
        build_device_nbr<int32_t>(c->plan, m0, c->np, t32);
        BoundaryList bl;
        build_boundary(c->plan, m0, c->seg_off, c->iolet_off, bl);
        Compressed& cm = c->comp;
        std::string ce = build_compressed(c->plan, bl, t32, c->np, cm);
        if (!ce.empty()) rc = fail(c, LBM_EINVAL, "%s", ce.c_str());
        c->n_irr = (int64_t)bl.site.size();
        c->n_exc = cm.n_exc;
        c->n_exc_pad = cm.n_exc_pad;
        c->n_stretch = cm.n_stretch;
        const int64_t ni = c->n_irr, nwf = c->np / 64;
        rc = rc ? rc : dalloc(c, (void**)&c->bj, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->rsite, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->bidx, c->plan.N * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->bwall, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->bio, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->bk, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->bq, std::max<int64_t>(1, ni) * sizeof(WallCoef));
        rc = rc ? rc : dalloc(c, (void**)&c->bqf, std::max<int64_t>(1, ni) * sizeof(WallCoefF));
        c->rec_k.assign(bl.kidx.begin(), bl.kidx.end());
        c->rec_inst.resize(bl.wall.size());
        for (size_t j = 0; j < bl.wall.size(); ++j) c->rec_inst[j] = (int32_t)(bl.wall[j] >> 19);
        rc = rc ? rc : dalloc(c, (void**)&c->bw, ni * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->wf, nwf * sizeof(WfRec));
        rc = rc ? rc : dalloc(c, (void**)&c->stretch, cm.stretch.size() * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->nfm, cm.nfm.size() * 4);
        rc = rc ? rc : dalloc(c, (void**)&c->exc, cm.exc.size() * 4);
    }
    if (c->have16) rc = rc ? rc : dalloc(c, &c->nbr16, (size_t)18 * c->np * 2);
    const int64_t nw = (int64_t)c->plan.wall_site.size();
    rc = rc ? rc : dalloc(c, (void**)&c->wsite, nw * 4);
    rc = rc ? rc : dalloc(c, (void**)&c->wnormal, nw * 24);
    rc = rc ? rc : dalloc(c, (void**)&c->wk, nw * 4);
    rc = rc ? rc : dalloc(c, (void**)&c->ip, n_inst * sizeof(InstParams));
    rc = rc ? rc : dalloc(c, (void**)&c->iop, std::max(1, io) * sizeof(IoletParams));
    rc = rc ? rc : dalloc(c, (void**)&c->kinv, std::max(1, so) * sizeof(double));
    rc = rc ? rc : dalloc(c, (void**)&c->clock, 2 * sizeof(int64_t));
    rc = rc ? rc : dalloc(c, (void**)&c->maxes, 4 * sizeof(unsigned int));
    if (rc) {
        g_last_error = c->err;
        lbm_destroy(c);
        return rc;
    }
    // internal -> canonical site maps of exchanged instances
    c->i2c_dev.assign((size_t)n_inst, nullptr);
    for (int k = 0; k < n_inst && !rc; ++k) {
        if (!c->axis[k]) continue;
        const std::vector<int32_t>& m = c->c2i[k];
        std::vector<int32_t> inv(m.size());
        for (size_t j = 0; j < m.size(); ++j) inv[(size_t)m[j]] = (int32_t)j;
        rc = dalloc(c, (void**)&c->i2c_dev[k], inv.size() * 4);
        rc = rc ? rc : upload(c, c->i2c_dev[k], inv.data(), inv.size() * 4);
    }
    if (rc) {
        g_last_error = c->err;
        lbm_destroy(c);
        return rc;
    }
    // wall-site arrays (fixed by the geometry)
    std::vector<int32_t> wk(nw);
    for (int64_t j = 0; j < nw; ++j) {
        const int32_t x = c->plan.wall_site[j];
        const uint32_t k = c->plan.site_inst[x];
        wk[j] = c->seg_off[k] + c->plan.site_seg[x];
    }
    const int64_t zero2[2] = {0, 0};
    rc = rc ? rc : upload(c, c->wsite, c->plan.wall_site.data(), nw * 4);
    rc = rc ? rc : upload(c, c->wnormal, c->plan.wall_normal.data(), nw * 24);
    rc = rc ? rc : upload(c, c->wk, wk.data(), nw * 4);
    rc = rc ? rc : upload(c, c->clock, zero2, sizeof(zero2));
    // padding / unused slots start at zero deviation
    if (!rc) {
        hipError_t z0 = hipMemsetAsync(c->buf[0], 0, pop_bytes, c->stream);
        hipError_t z1 = hipMemsetAsync(c->buf[1], 0, pop_bytes, c->stream);
        if (z0 != hipSuccess || z1 != hipSuccess) rc = fail(c, LBM_EDEVICE, "hipMemset failed");
    }
    for (int k = 0; k < n_inst && !rc; ++k) rc = init_instance(c, k, nullptr, nullptr, nullptr, nullptr);
    rc = rc ? rc : sync_params(c);
    if (rc) {
        g_last_error = c->err;
        lbm_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    if (c->stream || !c->own_stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto& b : c->owned) release(c, b.p);
    c->owned.clear();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return LBM_OK;
}

int lbm_set_wall_params(lbm_ctx* c, int inst, int mode, double F, double P0,
                        const double* k_per_segment, int n_seg) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (mode != LBM_WALL_BOUNCEBACK && mode != LBM_WALL_ELASTIC)
        return fail(c, LBM_EINVAL, "unknown wall mode %d", mode);
    if (!(F >= 0.0 && F < 1.0)) return fail(c, LBM_EINVAL, "F must lie in [0, 1) (got %g)", F);
    if (!std::isfinite(P0)) return fail(c, LBM_EINVAL, "P0 must be finite");
    const InstanceGeom& g = c->plan.inst[inst];
    if (n_seg < g.n_seg || !k_per_segment)
        return fail(c, LBM_EINVAL, "instance %d uses %d segments, got %d stiffness values", inst,
                    g.n_seg, n_seg);
    for (int s = 0; s < g.n_seg; ++s)
        if (!(k_per_segment[s] > 0.0))
            return fail(c, LBM_EINVAL, "stiffness of segment %d must be > 0 (got %g)", s,
                        k_per_segment[s]);
    InstState& s = c->ist[inst];
    if (s.mode != mode) c->tables_dirty = true;
    s.mode = mode;
    s.F = F;
    s.P0 = P0;
    for (int j = 0; j < g.n_seg; ++j) s.k[j] = k_per_segment[j];
    s.Fseg.assign(g.n_seg, F);
    c->params_dirty = true;
    return LBM_OK;
}

int lbm_set_wall_F(lbm_ctx* c, int inst, const double* F_per_segment, int n_seg) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const InstanceGeom& g = c->plan.inst[inst];
    if (n_seg < g.n_seg || !F_per_segment)
        return fail(c, LBM_EINVAL, "instance %d uses %d segments, got %d slip ratios", inst,
                    g.n_seg, n_seg);
    for (int s = 0; s < g.n_seg; ++s)
        if (!(F_per_segment[s] >= 0.0 && F_per_segment[s] < 1.0))
            return fail(c, LBM_EINVAL, "F of segment %d must lie in [0, 1) (got %g)", s,
                        F_per_segment[s]);
    InstState& s = c->ist[inst];
    for (int j = 0; j < g.n_seg; ++j) s.Fseg[j] = F_per_segment[j];
    c->params_dirty = true;
    return LBM_OK;
}

int lbm_set_iolet(lbm_ctx* c, int inst, int id, int kind, double a0, double amp, double period,
                  double phase, const double* dir) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstState& s = c->ist[inst];
    if (id < 0 || id >= (int)s.iolets.size())
        return fail(c, LBM_EINVAL, "instance %d has no iolet %d adjacent to a fluid site", inst, id);
    if (kind != LBM_IOLET_DENSITY && kind != LBM_IOLET_VELOCITY)
        return fail(c, LBM_EINVAL, "unknown iolet kind %d", kind);
    if (!std::isfinite(a0) || !std::isfinite(amp) || !std::isfinite(phase))
        return fail(c, LBM_EINVAL, "iolet parameters must be finite");
    if (amp != 0.0 && !(period > 0.0)) return fail(c, LBM_EINVAL, "period must be > 0 when amp != 0");
    if (kind == LBM_IOLET_DENSITY && !(a0 > 0.0)) return fail(c, LBM_EINVAL, "density must be > 0");
    IoletParams q{};
    q.a0 = a0;
    q.amp = amp;
    q.inv_period = amp != 0.0 ? 1.0 / period : 0.0;
    q.phase = phase;
    q.kind = kind;
    const double nn = dir ? std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]) : 0.0;
    if (dir && !std::isfinite(nn)) return fail(c, LBM_EINVAL, "direction must be finite");
    if (kind == LBM_IOLET_VELOCITY) {
        if (!dir) return fail(c, LBM_EINVAL, "velocity iolet needs a direction");
        if (!(nn > 0.0)) return fail(c, LBM_EINVAL, "direction must be non-zero");
        for (int a = 0; a < 3; ++a) q.dir[a] = dir[comp_src(a, c->axis[inst])];
    } else if (nn > 0.0) {
        // density iolet with an inward normal: the velocity along it is kept
        for (int a = 0; a < 3; ++a) q.dir[a] = dir[comp_src(a, c->axis[inst])] / nn;
        q.pad = 1;
    }
    s.iolets[id] = q;
    s.iolet_set[id] = 1;
    c->params_dirty = true;
    return LBM_OK;
}

int lbm_init_fields(lbm_ctx* c, int inst, const double* rho, const double* u) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = init_instance(c, inst, rho, u, nullptr, nullptr);
    if (rc) return rc;
    c->ist[inst].t0 = c->step;
    c->ist[inst].has_snap = false;
    c->params_dirty = true;
    return sync_params(c);
}

int lbm_init_fields_device(lbm_ctx* c, int inst, const float* rho_u_dev) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!rho_u_dev) return fail(c, LBM_EINVAL, "rho_u_dev is NULL");
    rc = init_instance(c, inst, nullptr, nullptr, rho_u_dev, nullptr);
    if (rc) return rc;
    c->ist[inst].t0 = c->step;
    c->ist[inst].has_snap = false;
    c->params_dirty = true;
    return sync_params(c);
}

int lbm_step(lbm_ctx* c, int64_t n) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
    int rc = check_ready(c);
    if (rc) return rc;
    return run_steps(c, n);
}

int lbm_uses_caller_resources(const lbm_ctx* c, int* allocator, int* stream) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (allocator) *allocator = c->alloc_fn != nullptr;
    if (stream) *stream = !c->own_stream;
    return LBM_OK;
}

int lbm_sync(lbm_ctx* c) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_get_stream(lbm_ctx* c, void** stream) {
    if (!c || !stream) return fail(c, LBM_EINVAL, "NULL argument");
    *stream = (void*)c->stream;
    return LBM_OK;
}

int lbm_time_steps(lbm_ctx* c, int64_t n, double* ms) {
    if (!c || !ms) return fail(c, LBM_EINVAL, "NULL argument");
    int rc = check_ready(c);
    if (rc) return rc;
    if (c->use_graph && n >= GRAPH_STEPS) {  // capture outside the timed region
        hipGraphExec_t ex;
        rc = get_graph(c, (int)(c->step & 1), &ex);
        if (rc) return rc;
    }
    struct Events {  // destroyed on every exit path
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    HIP_TRY(c, hipEventCreate(&ev.e[0]));
    HIP_TRY(c, hipEventCreate(&ev.e[1]));
    HIP_TRY(c, hipEventRecord(ev.e[0], c->stream));
    rc = run_steps(c, n);
    HIP_TRY(c, hipEventRecord(ev.e[1], c->stream));
    HIP_TRY(c, hipEventSynchronize(ev.e[1]));
    float t = 0;
    HIP_TRY(c, hipEventElapsedTime(&t, ev.e[0], ev.e[1]));
    *ms = t;
    return rc;
}

int lbm_read_fields(lbm_ctx* c, int inst, double* rho, double* u, double* wss, float* wall_dr) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = sync_tables(c);
    rc = rc ? rc : sync_params(c);
    if (rc) return rc;
    const InstanceGeom& g = c->plan.inst[inst];
    const int64_t n = g.n;
    rc = ensure_scratch(c, (size_t)n * (8 * 5) + (size_t)n * 4 + 256);
    if (rc) return rc;
    double* s_rho = (double*)c->scratch.p;
    double* s_u = s_rho + n;
    double* s_wss = s_u + 3 * n;
    float* s_dr = (float*)(s_wss + n);
    const void* A = c->buf[c->step & 1];
    FieldArgs fa{A, nbr_rd(c), c->np, (int32_t)g.offset, (int32_t)n, 1.0 / c->tau, s_rho, s_u};
    hipError_t e = launch_fields(c->dtype, 32, fa, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "read-out launch failed: %s", hipGetErrorString(e));
    if (wss || wall_dr) {
        HIP_TRY(c, hipMemsetAsync(s_wss, 0, (size_t)n * 8, c->stream));
        HIP_TRY(c, hipMemsetAsync(s_dr, 0, (size_t)n * 4, c->stream));
        const InstState& st = c->ist[inst];
        WallArgs wa;
        wa.A = A;
        wa.nbr = nbr_rd(c);
        wa.np = c->np;
        wa.first = (int32_t)g.offset;
        wa.nw = (int32_t)(g.wall_end - g.wall_begin);
        wa.wsite = c->wsite + g.wall_begin;
        wa.wnormal = c->wnormal + 3 * g.wall_begin;
        wa.wk = c->wk + g.wall_begin;
        wa.omega = 1.0 / c->tau;
        wa.stress_fac = 1.0 - 1.0 / (2.0 * c->tau);
        wa.dp0 = 1.0 / 3.0 - st.P0;
        wa.elastic = st.mode == LBM_WALL_ELASTIC;
        wa.kinv = c->kinv;
        wa.wss = s_wss;
        wa.dr = s_dr;
        e = launch_wall(c->dtype, 32, wa, c->stream);
        if (e != hipSuccess) return fail(c, LBM_EDEVICE, "wall read-out launch failed: %s", hipGetErrorString(e));
    }
    // internal order and frame; exchanged instances go through host copies
    const int ax = c->axis[inst];
    std::vector<double> hr, hu, hw;
    std::vector<float> hd;
    double* prho = rho;
    double* pu = u;
    double* pw = wss;
    float* pd = wall_dr;
    if (!prho || ax) { hr.resize(n); prho = hr.data(); }
    if (!pu || ax) { hu.resize(3 * n); pu = hu.data(); }
    if (wss && ax) { hw.resize(n); pw = hw.data(); }
    if (wall_dr && ax) { hd.resize(n); pd = hd.data(); }
    HIP_TRY(c, hipMemcpyAsync(prho, s_rho, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pu, s_u, (size_t)n * 24, hipMemcpyDeviceToHost, c->stream));
    if (wss) HIP_TRY(c, hipMemcpyAsync(pw, s_wss, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    if (wall_dr) HIP_TRY(c, hipMemcpyAsync(pd, s_dr, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // outputs are written in canonical order first, then checked, so a
    // diverged state is still returned in full
    if (ax) {
        const std::vector<int32_t>& m = c->c2i[inst];
        for (int64_t k = 0; k < n; ++k) {
            const size_t j = (size_t)m[k];
            if (rho) rho[k] = prho[j];
            if (u)
                for (int a = 0; a < 3; ++a) u[3 * k + a] = pu[3 * j + comp_src(a, ax)];
            if (wss) wss[k] = pw[j];
            if (wall_dr) wall_dr[k] = pd[j];
        }
    }
    for (int64_t k = 0; k < n; ++k)
        if (!std::isfinite(prho[k]) || !std::isfinite(pu[3 * k]) || !std::isfinite(pu[3 * k + 1]) ||
            !std::isfinite(pu[3 * k + 2]))
            return fail(c, LBM_EDIVERGED, "non-finite field in instance %d (step %lld)", inst,
                        (long long)c->step);
    return LBM_OK;
}

int lbm_read_fields_noalloc(lbm_ctx* c, int inst, double* rho, double* u, double* wss,
                            float* wall_dr) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (c->tables_dirty || c->params_dirty)
        return fail(c, LBM_ESTATE, "wall or iolet parameters changed since the last step: call "
                                   "lbm_step or lbm_read_fields first");
    const InstanceGeom& g = c->plan.inst[inst];
    const int64_t n = g.n;
    if (n > LBM_NOALLOC_MAX_SITES)
        return fail(c, LBM_EINVAL, "instance %d has %lld sites; lbm_read_fields_noalloc takes at most %lld",
                    inst, (long long)n, (long long)LBM_NOALLOC_MAX_SITES);
    int dev = -1;
    HIP_TRY(c, hipGetDevice(&dev));
    if (dev != c->device)
        return fail(c, LBM_ESTATE, "current device %d is not the context's device %d", dev, c->device);
    // staging in the device's static array: flag | rho | u | wss | dr
    unsigned char* base = (unsigned char*)c->noalloc;
    unsigned int* bad = (unsigned int*)base;
    double* s_rho = (double*)(base + 256);
    double* s_u = s_rho + n;
    double* s_wss = s_u + 3 * n;
    float* s_dr = (float*)(s_wss + n);
    const void* A = c->buf[c->step & 1];
    const int ax = c->axis[inst];
    hipError_t e = launch_zero_u32(bad, 1, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    FieldArgs fa{A, nbr_rd(c), c->np, (int32_t)g.offset, (int32_t)n, 1.0 / c->tau, s_rho, s_u};
    fa.i2c = c->i2c_dev[inst];
    fa.axis = ax;
    fa.bad = bad;
    e = launch_fields(c->dtype, 32, fa, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "read-out launch failed: %s", hipGetErrorString(e));
    if (wss || wall_dr) {
        // zero by a fill kernel (the wall kernel writes wall sites only)
        e = launch_zero_u32((unsigned int*)s_wss, 2 * n + n, c->stream);
        if (e != hipSuccess) return fail(c, LBM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
        const InstState& st = c->ist[inst];
        WallArgs wa;
        wa.A = A;
        wa.nbr = nbr_rd(c);
        wa.np = c->np;
        wa.first = (int32_t)g.offset;
        wa.nw = (int32_t)(g.wall_end - g.wall_begin);
        wa.wsite = c->wsite + g.wall_begin;
        wa.wnormal = c->wnormal + 3 * g.wall_begin;
        wa.wk = c->wk + g.wall_begin;
        wa.omega = 1.0 / c->tau;
        wa.stress_fac = 1.0 - 1.0 / (2.0 * c->tau);
        wa.dp0 = 1.0 / 3.0 - st.P0;
        wa.elastic = st.mode == LBM_WALL_ELASTIC;
        wa.kinv = c->kinv;
        wa.wss = s_wss;
        wa.dr = s_dr;
        wa.i2c = c->i2c_dev[inst];
        e = launch_wall(c->dtype, 32, wa, c->stream);
        if (e != hipSuccess) return fail(c, LBM_EDEVICE, "wall read-out launch failed: %s", hipGetErrorString(e));
    }
    unsigned int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, bad, sizeof(flag), hipMemcpyDeviceToHost, c->stream));
    if (rho) HIP_TRY(c, hipMemcpyAsync(rho, s_rho, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    if (u) HIP_TRY(c, hipMemcpyAsync(u, s_u, (size_t)n * 24, hipMemcpyDeviceToHost, c->stream));
    if (wss) HIP_TRY(c, hipMemcpyAsync(wss, s_wss, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    if (wall_dr) HIP_TRY(c, hipMemcpyAsync(wall_dr, s_dr, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag)
        return fail(c, LBM_EDIVERGED, "non-finite field in instance %d (step %lld)", inst,
                    (long long)c->step);
    return LBM_OK;
}

int lbm_read_populations(lbm_ctx* c, int inst, double* f) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!f) return fail(c, LBM_EINVAL, "f is NULL");
    rc = sync_tables(c);
    if (rc) return rc;
    const InstanceGeom& g = c->plan.inst[inst];
    rc = ensure_scratch(c, (size_t)g.n * Q * 8);
    if (rc) return rc;
    PopArgs a{c->buf[c->step & 1], nbr_rd(c), c->np, (int32_t)g.offset, (int32_t)g.n,
              (double*)c->scratch.p};
    hipError_t e = launch_read_pop(c->dtype, 32, a, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    const int ax = c->axis[inst];
    std::vector<double> hf;
    double* pf = f;
    if (ax) { hf.resize((size_t)g.n * Q); pf = hf.data(); }
    HIP_TRY(c, hipMemcpyAsync(pf, c->scratch.p, (size_t)g.n * Q * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (ax) {
        const std::vector<int32_t>& m = c->c2i[inst];
        int dm[Q];
        for (int i = 0; i < Q; ++i) dm[i] = dir_swap(i, ax);
        for (int64_t k = 0; k < g.n; ++k)
            for (int i = 0; i < Q; ++i) f[(size_t)k * Q + i] = pf[(size_t)m[k] * Q + dm[i]];
    }
    return LBM_OK;
}

int lbm_write_populations(lbm_ctx* c, int inst, const double* f) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!f) return fail(c, LBM_EINVAL, "f is NULL");
    return init_instance(c, inst, nullptr, nullptr, nullptr, f);
}

int lbm_cycle_delta(lbm_ctx* c, int inst, double* delta_u, double* delta_p) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = sync_tables(c);
    if (rc) return rc;
    InstState& st = c->ist[inst];
    const InstanceGeom& g = c->plan.inst[inst];
    if (!st.snap.p) {
        rc = dalloc(c, &st.snap.p, (size_t)g.n * 16);
        if (rc) return rc;
        st.snap.bytes = (size_t)g.n * 16;
    }
    hipError_t e = launch_zero_u32(c->maxes, 4, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    DeltaArgs a{c->buf[c->step & 1], nbr_rd(c), c->np, (int32_t)g.offset, (int32_t)g.n,
                1.0 / 3.0 - st.P0, (float*)st.snap.p, st.has_snap ? 1 : 0, c->maxes};
    e = launch_delta(c->dtype, 32, a, c->stream);
    if (e != hipSuccess) return fail(c, LBM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    unsigned int m[4];
    HIP_TRY(c, hipMemcpyAsync(m, c->maxes, sizeof(m), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float v[4];
    std::memcpy(v, m, sizeof(v));
    const bool first = !st.has_snap;
    st.has_snap = true;
    const double inf = std::numeric_limits<double>::infinity();
    if (delta_u) *delta_u = first ? inf : (v[1] > 0 ? v[0] / v[1] : (v[0] > 0 ? inf : 0.0));
    if (delta_p) *delta_p = first ? inf : (v[3] > 0 ? v[2] / v[3] : (v[2] > 0 ? inf : 0.0));
    if (!std::isfinite(v[0]) || !std::isfinite(v[1]) || !std::isfinite(v[2]) || !std::isfinite(v[3]))
        return fail(c, LBM_EDIVERGED, "non-finite velocity or pressure in instance %d", inst);
    return LBM_OK;
}

int lbm_get_info(const lbm_ctx* c, lbm_info* info) {
    if (!c || !info) return fail(nullptr, LBM_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_sites = c->plan.N;
    info->n_boundary = c->nb;
    info->n_wall_sites = (int64_t)c->plan.wall_site.size();
    info->n_wall_links = c->plan.n_wall_links;
    info->n_iolet_links = c->plan.n_iolet_links;
    info->step = c->step;
    info->n_instances = (int32_t)c->ist.size();
    info->dtype = c->dtype;
    info->index_bits = c->ibits;
    info->block_size = c->block;
    info->use_graph = c->use_graph;
    info->xcd_remap = c->xcd;
    info->nontemporal = c->nt;
    info->boundary_fused = c->fused;
    info->sites_per_lane = c->spt;
    info->bytes_per_site_algorithmic = 2.0 * Q * (double)c->esize;
    const double N = (double)std::max<int64_t>(1, c->plan.N);
    if (c->ibits == 0)
        // populations; wavefront records; stretches; link mask per
        // irregular site; wall and iolet words and wall coefficients per
        // site with boundary-rule links; full offsets of exceptional sites
        info->bytes_per_site_model = 2.0 * Q * (double)c->esize + 48.0 / 64.0 +
                                     32.0 * (double)c->n_stretch / N +
                                     4.0 * (double)c->n_irr / N +
                                     (8.0 + (c->dtype == LBM_F64 ? sizeof(WallCoef) : sizeof(WallCoefF))) *
                                         (double)c->nb / N +
                                     72.0 * (double)c->n_exc / N;
    else
        info->bytes_per_site_model = 2.0 * Q * (double)c->esize + 18.0 * (c->ibits / 8) +
                                     (double)c->nb / N * 24.0;
    info->device_bytes = c->device_bytes;
    return LBM_OK;
}

int lbm_instance_sites(const lbm_ctx* c, int inst, int64_t* n) {
    if (!c || !n) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (inst < 0 || inst >= (int)c->ist.size())
        return fail(c, LBM_EINVAL, "instance %d out of range [0, %zu)", inst, c->ist.size());
    *n = c->plan.inst[inst].n;
    return LBM_OK;
}

// The two-sites-per-lane update forms 32-bit slot offsets (bytes below
// 2 GiB, elements above) of up to about 3 np + 2 elements.
static bool pair_offsets_fit(int64_t np) { return 3 * np + 4096 < (int64_t)1 << 32; }

int lbm_set_launch(lbm_ctx* c, int block_size, int index_bits, int use_graph, int xcd_remap,
                   int nontemporal, int boundary_fused, int sites_per_lane) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (block_size != -1 && block_size != 64 && block_size != 128 && block_size != 256 &&
        block_size != 512 && block_size != 1024)
        return fail(c, LBM_EINVAL, "block size %d not supported", block_size);
    if (index_bits != -1 && index_bits != 0 && index_bits != 16 && index_bits != 32)
        return fail(c, LBM_EINVAL, "index_bits must be 0 (compressed), 16 or 32");
    if (sites_per_lane != -1 && sites_per_lane != 1 && sites_per_lane != 2)
        return fail(c, LBM_EINVAL, "sites_per_lane must be 1 or 2");
    {
        // two sites per lane: FP32 storage, compressed addressing, the fused
        // boundary mode, and 32-bit element offsets (they reach about 3 np)
        const int spt = sites_per_lane != -1 ? sites_per_lane : c->spt;
        const int ib = index_bits != -1 ? index_bits : c->ibits;
        const int fu = boundary_fused != -1 ? (boundary_fused ? 1 : 0) : c->fused;
        if (spt == 2 && (c->dtype != LBM_F32 || ib != 0 || !fu || !pair_offsets_fit(c->np)))
            return fail(c, LBM_EINVAL, "sites_per_lane 2 needs FP32 storage, index_bits 0, "
                                       "boundary_fused 1 and fewer than 1.4e9 padded sites");
    }
    if (xcd_remap != -1 && xcd_remap != 0 && xcd_remap != 1 &&
        (xcd_remap < 2 || xcd_remap > 4096 || (xcd_remap & (xcd_remap - 1))))
        return fail(c, LBM_EINVAL, "xcd_remap must be 0, 1 or a power of two up to 4096");
    if (index_bits == 16 && !c->have16)
        return fail(c, LBM_EINVAL, "a neighbour offset exceeds the 16-bit range (max %lld)",
                    (long long)c->plan.max_abs_offset);
    if (block_size != -1) c->block = block_size;
    if (index_bits != -1) c->ibits = index_bits;
    if (use_graph != -1) c->use_graph = use_graph ? 1 : 0;
    if (xcd_remap != -1) c->xcd = xcd_remap;
    if (nontemporal != -1) c->nt = nontemporal & 3;
    if (boundary_fused != -1) c->fused = boundary_fused ? 1 : 0;
    if (sites_per_lane != -1) c->spt = sites_per_lane;
    drop_graphs(c);
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* c, int steps_per_trial, double* best_rate) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (steps_per_trial < 2) return fail(c, LBM_EINVAL, "steps_per_trial must be >= 2");
    int rc = check_ready(c);
    if (rc) return rc;
    const TuneKey key{c->plan.N, c->nb, c->dtype};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && !best_rate) {
            const TuneVal& v = it->second;
            return lbm_set_launch(c, v.block, v.ibits, -1, v.xcd, v.nt, v.fused, v.spt);
        }
    }
    // save the state: both buffers and the clock
    const size_t pop_bytes = (size_t)Q * c->np * c->esize;
    ScopedDev s0(c), s1(c);
    rc = dalloc(c, &s0.p, pop_bytes);
    rc = rc ? rc : dalloc(c, &s1.p, pop_bytes);
    if (rc) return rc;
    void* const save0 = s0.p;
    void* const save1 = s1.p;
    int64_t clock_save[2];
    HIP_TRY(c, hipMemcpyAsync(save0, c->buf[0], pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(save1, c->buf[1], pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(clock_save, c->clock, sizeof(clock_save), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int64_t step_save = c->step;
    const int old_block = c->block, old_ibits = c->ibits, old_xcd = c->xcd, old_nt = c->nt,
              old_fused = c->fused, old_spt = c->spt;
    TuneVal best{old_block, old_ibits, old_xcd, old_nt, old_fused, old_spt};
    double best_ms = std::numeric_limits<double>::infinity();
    double best_score = std::numeric_limits<double>::infinity();
    const int blocks[] = {128, 256, 512, 1024};
    const int ibits_list[] = {0, 16, 32};
    // pass 1: every configuration once (non-temporal loads are left out:
    // the gathers share cache lines between neighbouring wavefronts)
    // (block orders: launch order, one range per XCD, and for compressed
    // addressing in the fused mode also runs of 4 and 16 blocks per XCD)
    std::vector<std::pair<double, TuneVal>> cand;
    std::vector<TuneVal> trials;
    for (int ib : ibits_list) {
        if (ib == 16 && !c->have16) continue;
        for (int fu = 0; fu < 2; ++fu)
            for (int bs : blocks)
                for (int xr : {0, 1, 4, 16}) {
                    if (xr > 1 && (ib != 0 || !fu)) continue;
                    for (int ntv = 0; ntv < 2; ++ntv) trials.push_back(TuneVal{bs, ib, xr, ntv, fu, 1});
                }
    }
    // two sites per lane where they apply (FP32, compressed, fused)
    if (c->dtype == LBM_F32 && pair_offsets_fit(c->np))
        for (int bs : {128, 256, 512})
            for (int xr : {0, 1, 4, 16})
                for (int ntv = 0; ntv < 2; ++ntv) trials.push_back(TuneVal{bs, 0, xr, ntv, 1, 2});
    for (const TuneVal& v : trials) {
        rc = lbm_set_launch(c, v.block, v.ibits, -1, v.xcd, v.nt, v.fused, v.spt);
        if (rc) break;
        double ms = 0;
        rc = run_steps(c, 2);  // warm-up (and graph build)
        rc = rc ? rc : lbm_time_steps(c, steps_per_trial, &ms);
        if (rc) break;
        cand.push_back({ms, v});
    }
    // pass 2: the six fastest again, three times each with twice the steps
    // (single short trials are noisy: clocks and cache contents vary).  The
    // block orders that keep neighbouring blocks on one XCD move fewer
    // bytes (neighbouring wavefronts share lines in one L2; the tree in FP32
    // reads 1.08 instead of 1.19 times the algorithmic bytes with one range
    // per XCD), so they are kept unless the launch order is more than 2 %
    // faster
    if (!rc) {
        std::sort(cand.begin(), cand.end(),
                  [](const std::pair<double, TuneVal>& a, const std::pair<double, TuneVal>& b) {
                      return a.first < b.first;
                  });
        const size_t top = std::min<size_t>(6, cand.size());
        for (size_t k = 0; k < top && !rc; ++k) {
            const TuneVal& v = cand[k].second;
            rc = lbm_set_launch(c, v.block, v.ibits, -1, v.xcd, v.nt, v.fused, v.spt);
            double t = std::numeric_limits<double>::infinity();
            for (int r = 0; r < 3 && !rc; ++r) {
                double ms = 0;
                rc = lbm_time_steps(c, 2 * steps_per_trial, &ms);
                t = std::min(t, ms / 2.0);
            }
            const double score = t * (v.xcd ? 0.98 : 1.0);
            if (!rc && score < best_score) {
                best_score = score;
                best_ms = t;
                best = v;
            }
        }
    }
    // restore
    HIP_TRY(c, hipMemcpyAsync(c->buf[0], save0, pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->buf[1], save1, pop_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->clock, clock_save, sizeof(clock_save), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = step_save;
    if (rc) {
        lbm_set_launch(c, old_block, old_ibits, -1, old_xcd, old_nt, old_fused, old_spt);
        return rc;
    }
    rc = lbm_set_launch(c, best.block, best.ibits, -1, best.xcd, best.nt, best.fused, best.spt);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (best_rate) *best_rate = steps_per_trial / (best_ms * 1e-3);
    return LBM_OK;
}

}  // extern "C"
