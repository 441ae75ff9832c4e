/*
 * lbm.h -- C ABI of the MI355X (gfx950) elastic-wall D3Q19 lattice Boltzmann
 * library.
 *
 * The method is that of McCullough & Coveney, "An efficient, localised
 * approach for the simulation of elastic blood vessels using the lattice
 * Boltzmann method" (2021):
 *   - D3Q19 lattice, single-relaxation-time (BGK) collision and streaming
 *     over the fluid sites of a sparse vessel geometry (Sec. 2.1, eqs.
 *     LBE_SRT, feq, Density, Momentum, Pressure);
 *   - the localised elastic wall: a GZS-type link rule with Delta = 1 whose
 *     wall-node velocity U_w = U_R + ((Delta r - Delta x)/Delta r)(U_f - U_R),
 *     U_R = F U_f, with Delta r = Delta x + Delta E and the extension
 *     Delta E following the local pressure (Sec. 2.3 and the extension law of
 *     Sec. 2.4);
 *   - bounce-back rigid walls (Sec. 2.4), velocity inlets with a profile
 *     weight map and fixed-pressure (density) outlets (Sec. 3).
 *
 * Conventions
 *   - Every function returns an int status: LBM_OK (0) or a negative
 *     LBM_E* code.  No C++ exception crosses this boundary.  The message of
 *     the last failure is returned by lbm_last_error(ctx) (ctx may be NULL
 *     for failures of lbm_create_geometry / lbm_plan_*).
 *   - Lattice units throughout: Delta x = Delta t = 1, C_s^2 = 1/3,
 *     pressure p = rho / 3.
 *   - Voxel arrays are nx*ny*nz, x fastest, then y, then z.
 *   - Sites are the fluid voxels.  The canonical site order is the raster
 *     order of each instance's fluid voxels, instances concatenated; every
 *     per-site array exchanged through this API is in that order and covers
 *     one instance.
 *   - Population order (checkpoint calls): 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *     7..18 = face diagonals (x,y), (x,z), (y,z) families, each ordered
 *     (+,+), (-,-), (+,-), (-,+).
 *   - Host arrays passed in are read during the call and never retained;
 *     host arrays passed out are written before the call returns.  All
 *     device memory is owned by the context and freed by lbm_destroy; it is
 *     obtained from hipMalloc, or from the caller's allocator when one is
 *     given to lbm_create_geometry_ex.
 *   - A context is thread-compatible, not thread-safe: one host thread at a
 *     time.  All work is enqueued on the context's HIP stream: the caller's
 *     stream when one is given to lbm_create_geometry_ex, else a stream the
 *     context creates (lbm_get_stream).  lbm_step is asynchronous, the read
 *     calls synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or geometry                  */
#define LBM_ENOMEM (-2)    /* host or device allocation failed              */
#define LBM_EDEVICE (-3)   /* HIP runtime / launch failure                  */
#define LBM_EDIVERGED (-4) /* a non-finite value was read back              */
#define LBM_ESTATE (-5)    /* call not valid in the current state           */

/* ---- enums -------------------------------------------------------------- */
/* Storage type of the populations.  F64 and F32 store f_i - w_i in the
 * named type and collide in that type; F16DEV and BF16DEV store the
 * deviation f_i - w_i in 16 bits (round to nearest even) and collide in
 * FP32.  Wall distance and pressure are always evaluated in FP32 or
 * better. */
enum lbm_dtype { LBM_F64 = 0, LBM_F32 = 1, LBM_F16DEV = 2, LBM_BF16DEV = 3 };

/* Wall rule of an instance (Sec. 2.3 elastic; Sec. 2.4 bounce-back). */
enum lbm_wall_mode { LBM_WALL_BOUNCEBACK = 0, LBM_WALL_ELASTIC = 1 };

/* Inlet/outlet kind (Sec. 3): a DENSITY iolet prescribes rho and keeps the
 * fluid node's velocity (only its component along the iolet's inward normal
 * n, when n is given), a VELOCITY iolet prescribes u = weight * value * dir
 * and keeps the fluid node's density.  Both set the iolet node to the
 * equilibrium at those moments (zeroth order: unlike the elastic wall, no
 * non-equilibrium part is carried over).  Without the non-equilibrium part,
 * and with the tangential velocity removed at density iolets, the paper's
 * R = 50 cylinder stays stable at its tau = 0.537; with either kept, it
 * diverges there. */
enum lbm_iolet_kind { LBM_IOLET_DENSITY = 0, LBM_IOLET_VELOCITY = 1 };

/* Voxel labels. */
#define LBM_LABEL_WALL 0
#define LBM_LABEL_FLUID 1
#define LBM_LABEL_IOLET0 2 /* label 2 + id, id = 0..253 */

typedef struct lbm_ctx lbm_ctx;

/* One vessel instance.  labels: 0 wall/solid, 1 fluid, 2+id iolet.  A fluid
 * voxel must not lie on the array border.  The type of each link of a fluid
 * site is decided by the label of its upstream voxel x - c_i.
 *   segment      optional (NULL: all 0): wall segment id per voxel, selects
 *                the stiffness k of lbm_set_wall_params at fluid voxels;
 *   normal       optional (NULL: normalised sum of -c_i over the site's wall
 *                links): outward unit normal, 3 floats per voxel, used for
 *                the wall shear stress;
 *   iolet_weight optional (NULL: 1): profile weight per voxel, multiplies a
 *                velocity iolet's value at the fluid site next to it. */
typedef struct {
    int32_t nx, ny, nz;
    const uint8_t* labels;
    const uint16_t* segment;
    const float* normal;
    const float* iolet_weight;
} lbm_instance_desc;

typedef struct {
    int64_t n_sites;         /* fluid sites, all instances                   */
    int64_t n_boundary;      /* sites handled by the boundary pass           */
    int64_t n_wall_sites;    /* sites with at least one wall link            */
    int64_t n_wall_links;    /* links whose upstream voxel is a wall         */
    int64_t n_iolet_links;   /* links whose upstream voxel is an iolet       */
    int64_t step;            /* steps enqueued since creation                */
    int32_t n_instances;
    int32_t dtype;           /* enum lbm_dtype                               */
    int32_t index_bits;      /* 0 compressed addressing, 16/32 offset table  */
    int32_t block_size;      /* threads per block of the update kernel       */
    int32_t use_graph;       /* 1: lbm_step replays captured HIP graphs      */
    int32_t xcd_remap;       /* block -> XCD order (see lbm_set_launch)      */
    int32_t nontemporal;     /* bit 0 stores, bit 1 loads bypass the caches  */
    int32_t boundary_fused;  /* 1: boundary links applied inside the update   */
    int32_t sites_per_lane;  /* sites updated per lane in the update blocks   */
    int32_t reserved;
    double bytes_per_site_algorithmic; /* 2 * 19 * sizeof(stored type)       */
    double bytes_per_site_model;       /* + neighbour table + boundary data  */
    int64_t device_bytes;    /* device memory held by the context            */
} lbm_info;

/* Caller-supplied device resources (optional; see lbm_create_geometry_ex).
 *   alloc(bytes, user) returns device memory of the current device, at least
 *     `bytes` long and 256-byte aligned, or NULL on failure (reported as
 *     LBM_ENOMEM); free(ptr, user) returns a block obtained from alloc.  Both
 *     or neither must be set; with neither, hipMalloc / hipFree are used.
 *     The context calls them from the creating call, from calls that need
 *     read-out staging (first use, or a larger instance), from the first
 *     lbm_cycle_delta of an instance and from lbm_destroy, always on the
 *     calling thread.  Before it frees a block the context drains its
 *     stream.
 *   use_stream != 0: every operation of the context is enqueued on `stream`
 *     (a hipStream_t; NULL means the null stream), which the context never
 *     destroys and which must outlive it.  The step graphs are captured on
 *     a private stream of the context and launched on `stream`.
 *   user is passed through unchanged. */
typedef void* (*lbm_alloc_fn)(size_t bytes, void* user);
typedef void (*lbm_free_fn)(void* ptr, void* user);
typedef struct {
    lbm_alloc_fn alloc;
    lbm_free_fn free;
    void* user;
    int32_t use_stream;
    void* stream;
} lbm_resources;

/* ---- lifetime ----------------------------------------------------------- */

/* Builds the site list, the neighbour (pull) table and the compacted
 * boundary list of n_inst instances (Sec. 2.1 streaming over the fluid
 * nodes; Sec. 2.3 link classification), allocates device memory on the
 * current HIP device and initialises every instance to rho = 1, u = 0 with
 * bounce-back walls.  tau is the BGK relaxation time (Sec. 2.1), tau > 1/2.
 * Site order on the device: each instance is updated in raster order with
 * its fast axis innermost.  The fast axis is x unless the instance's fluid
 * voxels form clearly longer runs along y or z (lbm_fast_axis); then that
 * axis is exchanged with x internally.  This changes nothing at the
 * interface: every call takes and returns sites in canonical order and
 * vectors and directions in the caller's frame.  The environment variable
 * LBM_FAST_AXIS (x, y, z or auto) read here overrides the choice.
 * Errors: LBM_EINVAL (n_inst <= 0, tau <= 1/2, unknown dtype, no fluid
 * voxel, fluid on the border, a site touching two different iolets, more
 * than 2^31/19 sites, an invalid LBM_FAST_AXIS), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_create_geometry(lbm_ctx** out, const lbm_instance_desc* inst, int n_inst, int dtype,
                        double tau);

/* lbm_create_geometry with the caller's device allocator and/or stream
 * (res may be NULL: same as lbm_create_geometry).  Errors as
 * lbm_create_geometry, and LBM_EINVAL if only one of alloc / free is set or
 * the allocator returns a misaligned block. */
int lbm_create_geometry_ex(lbm_ctx** out, const lbm_instance_desc* inst, int n_inst, int dtype,
                           double tau, const lbm_resources* res);

/* Whether ctx allocates through the caller's allocator (*allocator = 1) and
 * enqueues on the caller's stream (*stream = 1); either pointer may be NULL. */
int lbm_uses_caller_resources(const lbm_ctx* ctx, int* allocator, int* stream);

/* Frees every resource of the context; NULL is accepted. */
int lbm_destroy(lbm_ctx* ctx);

/* Message of the last failure on ctx (or of the last context-less failure
 * of this thread when ctx is NULL).  Never NULL; owned by the library. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* ---- parameters --------------------------------------------------------- */

/* Wall rule of instance inst (Sec. 2.3, Sec. 2.4).  mode: enum
 * lbm_wall_mode.  F = U_R/U_f in [0, 1).  P0: pressure at which the
 * extension vanishes (lattice units).  k_per_segment[s] > 0: stiffness of
 * segment s, Delta E = max(0, (p - P0)/k) (k = Y h / ((1 - sigma^2) R^2) in
 * lattice units).  n_seg must cover every segment id present at the
 * instance's fluid voxels.  Takes effect for the next step.  Errors:
 * LBM_EINVAL. */
int lbm_set_wall_params(lbm_ctx* ctx, int inst, int mode, double F, double P0,
                        const double* k_per_segment, int n_seg);

/* Local slip ratio (the closing discussion of Sec. 4: F need not be global;
 * the Sec. 2.3 relation ties it to the local Womersley number and
 * Delta r / R).  F_per_segment[s] in [0, 1) replaces, for wall segment s of
 * instance inst, the single F of the last lbm_set_wall_params call, which
 * resets every segment to its F.  n_seg must cover every segment id present
 * at the instance's fluid voxels; the array is copied.  Takes effect for
 * the next step.  Errors: LBM_EINVAL. */
int lbm_set_wall_F(lbm_ctx* ctx, int inst, const double* F_per_segment, int n_seg);

/* Drive of iolet id of instance inst (Sec. 3).  value(t) = a0 (1 + amp
 * sin(2 pi t / period + phase)), t = steps since the instance's last
 * lbm_init_fields; amp = 0 gives a steady value (period is then ignored,
 * otherwise period > 0).  DENSITY: value is rho; dir, if not NULL and not
 * zero, is the iolet's inward normal n (normalised here): only the fluid
 * node's velocity along n enters the iolet node.  VELOCITY: the
 * prescribed velocity at fluid site x is iolet_weight(x) * value(t) * dir,
 * dir (3 doubles) the unit direction into the vessel.  Every iolet present
 * in the labels must be set before lbm_step.  Errors: LBM_EINVAL. */
int lbm_set_iolet(lbm_ctx* ctx, int inst, int id, int kind, double a0, double amp,
                  double period, double phase, const double* dir);

/* Sets f = feq(rho, u) at every site of instance inst (Sec. 2.1 eq. feq);
 * rho (n_inst_sites doubles) and u (3 * n_inst_sites doubles, xyz per site)
 * in canonical order; NULL means rho = 1 / u = 0.  Resets the instance's
 * drive clock to t = 0.  Errors: LBM_EINVAL, LBM_EDEVICE. */
int lbm_init_fields(lbm_ctx* ctx, int inst, const double* rho, const double* u);

/* Same as lbm_init_fields with a DEVICE array rho_u of 4 floats per site
 * (rho, ux, uy, uz) in canonical order for instance inst; the call is
 * enqueued on the context's stream after all previous work. */
int lbm_init_fields_device(lbm_ctx* ctx, int inst, const float* rho_u_dev);

/* ---- stepping ----------------------------------------------------------- */

/* Advances every instance by n >= 0 steps (Sec. 2.1 eq. LBE_SRT with the
 * boundary rules), asynchronously on the context's stream.  Errors:
 * LBM_ESTATE (an iolet without parameters), LBM_EDEVICE. */
int lbm_step(lbm_ctx* ctx, int64_t n);

/* Blocks until all work of the context has finished. */
int lbm_sync(lbm_ctx* ctx);

/* The context's HIP stream (hipStream_t) in *stream. */
int lbm_get_stream(lbm_ctx* ctx, void** stream);

/* Enqueues n steps between two HIP events recorded on the context's stream
 * and returns the elapsed milliseconds (synchronises). */
int lbm_time_steps(lbm_ctx* ctx, int64_t n, double* ms);

/* ---- read-out ----------------------------------------------------------- */

/* Fields of instance inst at the current time from f(t) (Sec. 2.1 eqs.
 * Density, Momentum, Pressure; p = rho/3).  Outputs (any may be NULL), in
 * canonical order of the instance's sites:
 *   rho     n doubles;
 *   u       3n doubles (xyz per site);
 *   wss     n doubles: |t - (t.n) n|, t = sigma n,
 *           sigma = -(1 - 1/(2 tau)) sum_i fneq_i c_i c_i, at sites with at
 *           least one wall link, 0 elsewhere;
 *   wall_dr n floats: Delta r = 1 + max(0, (p - P0)/k) at wall sites of an
 *           elastic instance, 0 elsewhere (Sec. 2.3, 2.4).
 * Synchronises.  Returns LBM_EDIVERGED if any rho or u is not finite (the
 * outputs are still written). */
int lbm_read_fields(lbm_ctx* ctx, int inst, double* rho, double* u, double* wss,
                    float* wall_dr);

/* Size of the per-device staging array of lbm_read_fields_noalloc, and the
 * largest instance (in sites) it can read: 44 bytes per site (rho, u, wss
 * as doubles, wall_dr as float) after a 256-byte flag block. */
#define LBM_NOALLOC_SCRATCH_BYTES (96u << 20)
#define LBM_NOALLOC_MAX_SITES (((int64_t)LBM_NOALLOC_SCRATCH_BYTES - 256) / 44)

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbm_read_fields
 * with the same arguments, outputs and result, that allocates nothing.
 * Its device staging lives in a fixed array of LBM_NOALLOC_SCRATCH_BYTES
 * per device, which the library reserves when it is loaded on a device and
 * holds until the process ends; sites of an instance whose fast axis is
 * exchanged are put in canonical order on the device.  Every call on one
 * device shares that array (the previous call's contents are overwritten;
 * what must start at zero is cleared by a kernel, not a memset), so calls
 * that overlap on one device, from different threads or from contexts with
 * different streams, race.  Errors: those of lbm_read_fields; LBM_EINVAL if
 * the instance has more than LBM_NOALLOC_MAX_SITES sites; LBM_ESTATE if
 * wall or iolet parameters were changed after the last lbm_step or
 * lbm_read_fields (the update that applies them would allocate), or if the
 * current device is not the context's. */
int lbm_read_fields_noalloc(lbm_ctx* ctx, int inst, double* rho, double* u, double* wss,
                            float* wall_dr);

/* Populations f_i(t) of instance inst, n * 19 doubles, site-major, in the
 * population order above (checkpoint).  Synchronises. */
int lbm_read_populations(lbm_ctx* ctx, int inst, double* f);

/* Overwrites f_i(t) of instance inst (same layout), keeping its clock. */
int lbm_write_populations(lbm_ctx* ctx, int inst, const double* f);

/* Periodicity monitor (cycle-to-cycle change).  Compares the current
 * velocity and pressure of instance inst with the snapshot taken by the
 * previous call and stores a new snapshot:
 *   delta_u = max_x |u(x) - u_prev(x)|_inf / max_x |u(x)|_inf,
 *   delta_p = max_x |p(x) - p_prev(x)| / max_x |p(x) - P0|.
 * The first call after creation or lbm_init_fields returns +inf for both.
 * The maxima are taken over the sites of the instance in FP32 (velocity
 * and p - 1/3 from the FP32 moments of f(t); the snapshot is FP32).
 * Synchronises.  Returns LBM_EDIVERGED if the velocity or pressure of any
 * site is not finite (the snapshot is replaced all the same). */
int lbm_cycle_delta(lbm_ctx* ctx, int inst, double* delta_u, double* delta_p);

/* ---- introspection / tuning ---------------------------------------------- */

int lbm_get_info(const lbm_ctx* ctx, lbm_info* info);

/* Number of sites of instance inst in *n. */
int lbm_instance_sites(const lbm_ctx* ctx, int inst, int64_t* n);

/* Launch configuration of the update kernel.  block_size in {64, 128, 256,
 * 512, 1024}; index_bits: 0 for compressed addressing (interior sites derive
 * their offsets from per-row offsets shared along runs of interior sites),
 * 16 or 32 for a per-site offset table (16 only if every neighbour offset
 * fits, else LBM_EINVAL); use_graph boolean; xcd_remap: 0 blocks in launch
 * order (the hardware deals them round-robin to the 8 XCDs), 1 one
 * contiguous site range per XCD, g = 2..4096 (a power of two) runs of g
 * neighbouring blocks per XCD, advancing together; nontemporal bit 0:
 * population stores bypass the caches, bit 1: population loads do;
 * boundary_fused 1: sites with elastic-wall or iolet links are updated by
 * the same blocks as all other sites, which apply the link rules in place;
 * 0: they are skipped there and updated by a compacted list of boundary
 * sites in blocks appended to the same launch.  Both modes compute the same
 * link rule.  sites_per_lane: 1, or 2 for FP32 storage with index_bits 0,
 * boundary_fused 1 and fewer than 1.4e9 padded sites (else LBM_EINVAL):
 * each wavefront then updates 128 consecutive sites, lane l the sites x and
 * x + 64, with the two loads of every direction issued back to back (the
 * 128-byte line they share is fetched once).  A value of -1 keeps the
 * current setting.  No setting changes the arithmetic. */
int lbm_set_launch(lbm_ctx* ctx, int block_size, int index_bits, int use_graph, int xcd_remap,
                   int nontemporal, int boundary_fused, int sites_per_lane);

/* Times every launch configuration on the context's own state for
 * steps_per_trial steps each (the populations are saved and restored), keeps
 * the fastest and writes its steps per second in *best_rate (may be NULL).
 * Results are cached in-process per (sites, boundary sites, dtype). */
int lbm_autotune(lbm_ctx* ctx, int steps_per_trial, double* best_rate);

/* ---- diagnostics ----------------------------------------------------------- */

/* Plain streaming device copy of `bytes` (a multiple of 16) from src to dst
 * (caller-owned device buffers, 16-byte aligned), `reps` times on `stream`
 * (hipStream_t, NULL = default), with 16-byte vector loads and stores,
 * optionally non-temporal.  Writes the average milliseconds per copy.  Used
 * as the reference for achievable HBM bandwidth and for scaling the
 * FETCH_SIZE / WRITE_SIZE counters; not part of the method.  Errors:
 * LBM_EINVAL, LBM_EDEVICE. */
int lbm_copy_probe(void* dst, const void* src, size_t bytes, int nontemporal, int reps,
                   void* stream, double* ms);

/* ---- host-only geometry plan (no device needed) -------------------------- */

/* Runs the host part of lbm_create_geometry for n_inst instances (wall mode
 * bounce-back for instances whose wall_mode[i] is 0, elastic for 1; NULL
 * means all bounce-back) and writes
 *   counts[6]  = {n_sites, n_boundary, n_wall_sites, n_wall_links,
 *                 n_iolet_links, max |neighbour offset|};
 *   nbr        = 18 * n_sites int32 if not NULL: for direction i = 1..18
 *                (row i-1) and site x, the offset d such that the upstream
 *                site is x + d, or INT32_MIN for a bounce-back link,
 *                INT32_MIN + 1 for a link handled by the boundary pass;
 *   boundary   = n_boundary int32 site indices if not NULL;
 *   bmask      = n_boundary uint32 if not NULL: bit i set for each link i
 *                whose upstream voxel is a wall (elastic) or an iolet.
 * No device call is made.  Errors: LBM_EINVAL. */
int lbm_plan_export(const lbm_instance_desc* inst, int n_inst, const int* wall_mode,
                    int64_t* counts, int32_t* nbr, int32_t* boundary, uint32_t* bmask);

/* Runs the host part of the compressed neighbour addressing of the update
 * kernel for n_inst instances (wall modes as for lbm_plan_export),
 * including its check that the compressed form reproduces the neighbour
 * table at every site, and writes
 *   stats[4] = {stretches, irregular sites, exceptional sites (rows of
 *               several fluid runs, full offsets kept), wavefront records}.
 * No device call is made.  Errors: LBM_EINVAL (invalid geometry, NULL
 * stats, or the check failed). */
int lbm_plan_compressed(const lbm_instance_desc* inst, int n_inst, const int* wall_mode,
                        int64_t* stats);

/* The fast axis lbm_create_geometry uses for each of n_inst instances:
 * axis[k] = 0 keeps x, 1 exchanges x and y, 2 exchanges x and z.  The axis
 * with the longest mean run of fluid voxels (fluid voxels per run of
 * consecutive fluid voxels along it) is chosen when its mean run is at
 * least 1.25 times that along x; LBM_FAST_AXIS overrides.  lbm_plan_export
 * and lbm_plan_compressed describe the geometry as given, without the
 * exchange.  No device call is made.  Errors: LBM_EINVAL. */
int lbm_fast_axis(const lbm_instance_desc* inst, int n_inst, int* axis);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
