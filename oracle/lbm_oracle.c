/*
 * Reference oracle for the elastic-wall D3Q19 lattice Boltzmann method of
 * McCullough & Coveney, "An efficient, localised approach for the simulation
 * of elastic blood vessels using the lattice Boltzmann method" (2021).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 CPU statement
 * of what the GPU library computes.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, tables or
 * headers with the HIP library.
 *
 * Route (deliberately different from the GPU one):
 *   - dense int32 index grid over the voxel box, coordinates -> site index;
 *   - populations stored array-of-structures f[site][19];
 *   - textbook order: collide every site, then stream every site;
 *   - boundary links are written from the PRE-collision non-equilibrium part,
 *     exactly as the wall rule is stated (Sec. 2.3), not from post-collision
 *     values.
 *
 * Readings of the paper taken here (the same readings the GPU side follows):
 *   R1  equilibrium (Sec. 2.1, eq. feq) with the standard factors 1/2 on the
 *       second-order terms; the printed form lacks them and would give a
 *       second moment of rho/3 I + 2 rho u u.
 *   R2  GZS wall-node density is the density of the fluid node (Sec. 2.3).
 *   R3  Delta r = Delta x + Delta E: the undeformed wall sits on the wall node
 *       (GZS with Delta = 1), Delta E is the pressure-driven extension.
 *   R4  Delta E = max(0, (p - P0)/k), k = Y h / ((1 - sigma^2) R^2) in lattice
 *       units (Sec. 2.4 law between extension and pressure).
 *   R5  U_w = U_R + ((Delta r - Delta x)/Delta r)(U_f - U_R), U_R = F U_f,
 *       applied to the full velocity vector of the fluid node (Sec. 2.3).
 *   R6  inlets/outlets (Sec. 3, fixed pressure after the cited pressure
 *       boundary scheme, prescribed velocity at the inlet): the iolet node
 *       is at equilibrium, without the non-equilibrium part the wall rule
 *       carries over (zeroth order); a density iolet prescribes rho and
 *       keeps the fluid node's u (only its component along the iolet's
 *       inward normal when the caller gives one); a velocity iolet
 *       prescribes u and keeps the fluid node's rho.  Carrying the
 *       non-equilibrium part or the tangential velocity over diverges at
 *       the paper's tau = 0.537 in its R = 50 cylinder.
 *   R7  the update from step n to n+1 uses the drive value at time n.
 *   R8  wall shear stress: sigma = -(1 - 1/(2 tau)) sum_i fneq_i c_i c_i,
 *       traction t = sigma n, WSS = |t - (t.n) n| at fluid sites that have at
 *       least one wall link; n is the caller's outward normal, else the
 *       normalised sum of -c_i over the site's wall links.
 *
 * Velocity set order (Sec. 2.1): 0 rest; 1..6 the axis directions
 * (+x,-x,+y,-y,+z,-z); 7..18 the face diagonals in the listed families
 * (x,y), (x,z), (y,z), each family ordered (+,+), (-,-), (+,-), (-,+).
 *
 * Voxel labels: 0 wall, 1 fluid, 2..255 iolet with id = label - 2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

/* Sec. 2.1: weights 1/3 (rest), 1/18 (axis), 1/36 (diagonal). */
static double weight(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

#define MAX_IOLETS 254

typedef struct {
    int nx, ny, nz;
    long nvox;
    int n;                 /* fluid sites */
    int *index;            /* nvox, site index or -1 */
    int *site_x, *site_y, *site_z;
    uint8_t *labels;       /* copy */
    int *seg;              /* per site */
    double *normal;        /* 3 per site; zero if absent */
    int has_normal;
    double *iolet_w;       /* per site */
    double tau;
    int mode;              /* 0 bounce-back, 1 elastic */
    double F, P0;
    double *k_seg;
    double *F_seg;         /* slip ratio per segment, F by default */
    int n_seg;
    int io_kind[MAX_IOLETS];
    double io_a0[MAX_IOLETS], io_amp[MAX_IOLETS], io_period[MAX_IOLETS], io_phase[MAX_IOLETS];
    double io_dir[MAX_IOLETS][3];
    int io_project[MAX_IOLETS];      /* density iolet with an inward normal */
    int io_set[MAX_IOLETS];
    double *f, *fnew, *fstar;   /* n*Q, array of structures */
    double *rho, *ux, *uy, *uz; /* pre-collision moments of the current step */
    long t;
} orc_t;

/* Sec. 2.1 eq. feq, reading R1. */
static double feq_i(int i, double rho, double ux, double uy, double uz) {
    const double cs2 = 1.0 / 3.0;
    double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
    double uu = ux * ux + uy * uy + uz * uz;
    return weight(i) * rho * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

/* Sec. 2.1 eqs. Density and Momentum. */
static void moments(const double *f, double *rho, double *ux, double *uy, double *uz) {
    double r = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
        jz += f[i] * CZ[i];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
    *uz = jz / r;
}

static long vox(const orc_t *o, int x, int y, int z) {
    return ((long)z * o->ny + y) * o->nx + x;
}

/* Drive value a0 (1 + amp sin(2 pi t / period + phase)), reading R7. */
static double drive(const orc_t *o, int id, long t) {
    double v = o->io_a0[id];
    if (o->io_amp[id] != 0.0)
        v *= 1.0 + o->io_amp[id] * sin(2.0 * M_PI * (double)t / o->io_period[id] + o->io_phase[id]);
    return v;
}

void orc_destroy(void *h) {
    orc_t *o = (orc_t *)h;
    if (!o) return;
    free(o->index); free(o->site_x); free(o->site_y); free(o->site_z); free(o->labels);
    free(o->seg); free(o->normal); free(o->iolet_w); free(o->k_seg); free(o->F_seg);
    free(o->f); free(o->fnew); free(o->fstar);
    free(o->rho); free(o->ux); free(o->uy); free(o->uz);
    free(o);
}

/* Returns NULL if a fluid voxel touches the array border (its neighbours
 * would be undefined) or if there is no fluid voxel. */
void *orc_create(int nx, int ny, int nz, const uint8_t *labels, const uint16_t *segment,
                 const float *normal, const float *iolet_weight, double tau) {
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->nx = nx; o->ny = ny; o->nz = nz;
    o->nvox = (long)nx * ny * nz;
    o->tau = tau;
    o->labels = (uint8_t *)malloc(o->nvox);
    memcpy(o->labels, labels, o->nvox);
    o->index = (int *)malloc(sizeof(int) * o->nvox);
    int n = 0;
    for (long v = 0; v < o->nvox; ++v) {
        if (labels[v] == 1) o->index[v] = n++;
        else o->index[v] = -1;
    }
    o->n = n;
    if (n == 0) { orc_destroy(o); return NULL; }
    o->site_x = (int *)malloc(sizeof(int) * n);
    o->site_y = (int *)malloc(sizeof(int) * n);
    o->site_z = (int *)malloc(sizeof(int) * n);
    o->seg = (int *)calloc(n, sizeof(int));
    o->normal = (double *)calloc(3 * (size_t)n, sizeof(double));
    o->iolet_w = (double *)malloc(sizeof(double) * n);
    o->has_normal = normal != NULL;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long v = vox(o, x, y, z);
                int s = o->index[v];
                if (s < 0) continue;
                if (x == 0 || y == 0 || z == 0 || x == nx - 1 || y == ny - 1 || z == nz - 1) {
                    orc_destroy(o);
                    return NULL;
                }
                o->site_x[s] = x; o->site_y[s] = y; o->site_z[s] = z;
                o->seg[s] = segment ? segment[v] : 0;
                if (normal) {
                    o->normal[3 * s + 0] = normal[3 * v + 0];
                    o->normal[3 * s + 1] = normal[3 * v + 1];
                    o->normal[3 * s + 2] = normal[3 * v + 2];
                }
                o->iolet_w[s] = iolet_weight ? iolet_weight[v] : 1.0;
            }
    size_t nq = (size_t)n * Q;
    o->f = (double *)calloc(nq, sizeof(double));
    o->fnew = (double *)calloc(nq, sizeof(double));
    o->fstar = (double *)calloc(nq, sizeof(double));
    o->rho = (double *)malloc(sizeof(double) * n);
    o->ux = (double *)malloc(sizeof(double) * n);
    o->uy = (double *)malloc(sizeof(double) * n);
    o->uz = (double *)malloc(sizeof(double) * n);
    o->mode = 0;
    o->F = 0.0;
    o->P0 = 1.0 / 3.0;
    o->n_seg = 1;
    o->k_seg = (double *)malloc(sizeof(double));
    o->k_seg[0] = 1.0;
    o->F_seg = (double *)malloc(sizeof(double));
    o->F_seg[0] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < Q; ++q) o->f[(size_t)i * Q + q] = weight(q);
    return o;
}

int orc_n_sites(void *h) { return ((orc_t *)h)->n; }

void orc_site_coords(void *h, int *xyz) {
    orc_t *o = (orc_t *)h;
    for (int s = 0; s < o->n; ++s) {
        xyz[3 * s] = o->site_x[s];
        xyz[3 * s + 1] = o->site_y[s];
        xyz[3 * s + 2] = o->site_z[s];
    }
}

void orc_velocity_set(int *c, double *w) {
    for (int i = 0; i < Q; ++i) {
        c[3 * i] = CX[i]; c[3 * i + 1] = CY[i]; c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
    }
}

void orc_feq(double rho, double ux, double uy, double uz, double *out) {
    for (int i = 0; i < Q; ++i) out[i] = feq_i(i, rho, ux, uy, uz);
}

void orc_set_wall(void *h, int mode, double F, double P0, const double *k, int n_seg) {
    orc_t *o = (orc_t *)h;
    o->mode = mode;
    o->F = F;
    o->P0 = P0;
    free(o->k_seg);
    free(o->F_seg);
    o->n_seg = n_seg;
    o->k_seg = (double *)malloc(sizeof(double) * (n_seg > 0 ? n_seg : 1));
    o->F_seg = (double *)malloc(sizeof(double) * (n_seg > 0 ? n_seg : 1));
    for (int s = 0; s < n_seg; ++s) {
        o->k_seg[s] = k[s];
        o->F_seg[s] = F;
    }
}

/* Slip ratio F per wall segment (the closing discussion of Sec. 4: F may be
 * set locally, e.g. per vessel of a tree from the Sec. 2.3 relation between
 * F, the Womersley number and Delta r / R).  Replaces the single F of
 * orc_set_wall for segments 0 .. n_seg-1; returns -1 if n_seg differs from
 * the count given to orc_set_wall. */
int orc_set_wall_F(void *h, const double *F, int n_seg) {
    orc_t *o = (orc_t *)h;
    if (n_seg != o->n_seg) return -1;
    for (int s = 0; s < n_seg; ++s) o->F_seg[s] = F[s];
    return 0;
}

void orc_set_iolet(void *h, int id, int kind, double a0, double amp, double period, double phase,
                   const double *dir) {
    orc_t *o = (orc_t *)h;
    o->io_kind[id] = kind;
    o->io_a0[id] = a0;
    o->io_amp[id] = amp;
    o->io_period[id] = period;
    o->io_phase[id] = phase;
    o->io_dir[id][0] = dir ? dir[0] : 0.0;
    o->io_dir[id][1] = dir ? dir[1] : 0.0;
    o->io_dir[id][2] = dir ? dir[2] : 0.0;
    o->io_project[id] = 0;
    if (kind == 0) {
        /* density iolet: a non-zero direction is its inward normal */
        double *d = o->io_dir[id];
        double nn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (nn > 0.0) {
            for (int a = 0; a < 3; ++a) d[a] /= nn;
            o->io_project[id] = 1;
        }
    }
    o->io_set[id] = 1;
}

/* f = feq(rho, u) at every site (canonical order); NULL means rho=1 / u=0.
 * Resets the time to 0. */
void orc_init_fields(void *h, const double *rho, const double *u) {
    orc_t *o = (orc_t *)h;
    for (int s = 0; s < o->n; ++s) {
        double r = rho ? rho[s] : 1.0;
        double ux = u ? u[3 * s] : 0.0, uy = u ? u[3 * s + 1] : 0.0, uz = u ? u[3 * s + 2] : 0.0;
        for (int i = 0; i < Q; ++i) o->f[(size_t)s * Q + i] = feq_i(i, r, ux, uy, uz);
    }
    o->t = 0;
}

void orc_set_populations(void *h, const double *f) {
    orc_t *o = (orc_t *)h;
    memcpy(o->f, f, sizeof(double) * (size_t)o->n * Q);
}

void orc_get_populations(void *h, double *f) {
    orc_t *o = (orc_t *)h;
    memcpy(f, o->f, sizeof(double) * (size_t)o->n * Q);
}

long orc_time(void *h) { return ((orc_t *)h)->t; }

/* Extension of the wall beyond the wall node and the link ratio
 * Delta r = Delta x + Delta E (readings R3, R4); Delta x = 1. */
static double wall_dr(const orc_t *o, int s, double rho) {
    double p = rho / 3.0; /* Sec. 2.1 eq. Pressure, C_s^2 = 1/3 */
    double k = o->k_seg[o->seg[s]];
    double dE = (p - o->P0) / k;
    if (dE < 0.0) dE = 0.0;
    return 1.0 + dE;
}

/* One time step t -> t+1. */
static void step_once(orc_t *o) {
    const int n = o->n;
    const double omega = 1.0 / o->tau;
    /* Collision (Sec. 2.1 eq. LBE_SRT) at every fluid site. */
#pragma omp parallel for schedule(static)
    for (int s = 0; s < n; ++s) {
        const double *f = o->f + (size_t)s * Q;
        double rho, ux, uy, uz;
        moments(f, &rho, &ux, &uy, &uz);
        o->rho[s] = rho; o->ux[s] = ux; o->uy[s] = uy; o->uz[s] = uz;
        for (int i = 0; i < Q; ++i) {
            double fe = feq_i(i, rho, ux, uy, uz);
            o->fstar[(size_t)s * Q + i] = f[i] - omega * (f[i] - fe);
        }
    }
    /* Streaming with the boundary rules for links whose upstream voxel is not
     * fluid. */
#pragma omp parallel for schedule(static)
    for (int s = 0; s < n; ++s) {
        const int x = o->site_x[s], y = o->site_y[s], z = o->site_z[s];
        const double rho = o->rho[s], ux = o->ux[s], uy = o->uy[s], uz = o->uz[s];
        const double *f = o->f + (size_t)s * Q;
        double *out = o->fnew + (size_t)s * Q;
        out[0] = o->fstar[(size_t)s * Q + 0];
        for (int i = 1; i < Q; ++i) {
            long v = vox(o, x - CX[i], y - CY[i], z - CZ[i]);
            int lab = o->labels[v];
            if (lab == 1) {
                out[i] = o->fstar[(size_t)o->index[v] * Q + i];
                continue;
            }
            if (lab == 0) {
                /* Non-equilibrium part of the fluid node, carried to the
                 * wall node (GZS, Sec. 2.3). */
                double fneq = f[i] - feq_i(i, rho, ux, uy, uz);
                if (o->mode == 0) {
                    /* Bounce-back (Sec. 2.4, rigid comparison). */
                    out[i] = o->fstar[(size_t)s * Q + opposite(i)];
                } else {
                    /* Elastic wall (Sec. 2.3): wall-node velocity from the
                     * linear profile between the fluid node and the extended
                     * wall at distance Delta r. */
                    double dr = wall_dr(o, s, rho);
                    double F = o->F_seg[o->seg[s]];
                    double URx = F * ux, URy = F * uy, URz = F * uz;
                    double a = (dr - 1.0) / dr;
                    double Uwx = URx + a * (ux - URx);
                    double Uwy = URy + a * (uy - URy);
                    double Uwz = URz + a * (uz - URz);
                    out[i] = feq_i(i, rho, Uwx, Uwy, Uwz) + (1.0 - omega) * fneq;
                }
            } else {
                /* Iolet (Sec. 3, reading R6): equilibrium at the prescribed
                 * density and the fluid node's velocity (along the iolet's
                 * inward normal, if one is set), or at the fluid node's
                 * density and the prescribed velocity. */
                int id = lab - 2;
                double val = drive(o, id, o->t);
                if (o->io_kind[id] == 0 && o->io_project[id]) {
                    const double *nv = o->io_dir[id];
                    double un = ux * nv[0] + uy * nv[1] + uz * nv[2];
                    out[i] = feq_i(i, val, un * nv[0], un * nv[1], un * nv[2]);
                } else if (o->io_kind[id] == 0) {
                    out[i] = feq_i(i, val, ux, uy, uz);
                } else {
                    double sp = o->iolet_w[s] * val;
                    out[i] = feq_i(i, rho, sp * o->io_dir[id][0], sp * o->io_dir[id][1],
                                   sp * o->io_dir[id][2]);
                }
            }
        }
    }
    double *tmp = o->f;
    o->f = o->fnew;
    o->fnew = tmp;
    o->t += 1;
}

void orc_step(void *h, long nsteps) {
    orc_t *o = (orc_t *)h;
    for (long k = 0; k < nsteps; ++k) step_once(o);
}

/* Fields at the current time from f(t) (Sec. 2.1 eqs. Density, Momentum and
 * Pressure); WSS by reading R8; wall_dr = Delta r at elastic wall sites, 0
 * elsewhere.  Any output pointer may be NULL. */
void orc_read(void *h, double *rho_out, double *u_out, double *wss_out, double *dr_out) {
    orc_t *o = (orc_t *)h;
    const double taufac = 1.0 - 1.0 / (2.0 * o->tau);
#pragma omp parallel for schedule(static)
    for (int s = 0; s < o->n; ++s) {
        const double *f = o->f + (size_t)s * Q;
        double rho, ux, uy, uz;
        moments(f, &rho, &ux, &uy, &uz);
        if (rho_out) rho_out[s] = rho;
        if (u_out) { u_out[3 * s] = ux; u_out[3 * s + 1] = uy; u_out[3 * s + 2] = uz; }
        int x = o->site_x[s], y = o->site_y[s], z = o->site_z[s];
        int nwall = 0;
        double gx = 0, gy = 0, gz = 0;
        for (int i = 1; i < Q; ++i) {
            if (o->labels[vox(o, x - CX[i], y - CY[i], z - CZ[i])] == 0) {
                nwall++;
                gx -= CX[i]; gy -= CY[i]; gz -= CZ[i];
            }
        }
        if (dr_out) dr_out[s] = (nwall > 0 && o->mode == 1) ? wall_dr(o, s, rho) : 0.0;
        if (!wss_out) continue;
        if (nwall == 0) { wss_out[s] = 0.0; continue; }
        double nxv, nyv, nzv;
        if (o->has_normal) {
            nxv = o->normal[3 * s]; nyv = o->normal[3 * s + 1]; nzv = o->normal[3 * s + 2];
        } else {
            nxv = gx; nyv = gy; nzv = gz;
        }
        double nn = sqrt(nxv * nxv + nyv * nyv + nzv * nzv);
        if (nn == 0.0) { wss_out[s] = 0.0; continue; }
        nxv /= nn; nyv /= nn; nzv /= nn;
        double S[3][3] = {{0}};
        for (int i = 0; i < Q; ++i) {
            double fneq = f[i] - feq_i(i, rho, ux, uy, uz);
            int c[3] = {CX[i], CY[i], CZ[i]};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) S[a][b] += fneq * c[a] * c[b];
        }
        double nv[3] = {nxv, nyv, nzv}, tr[3];
        for (int a = 0; a < 3; ++a) {
            tr[a] = 0;
            for (int b = 0; b < 3; ++b) tr[a] += -taufac * S[a][b] * nv[b];
        }
        double tn = tr[0] * nv[0] + tr[1] * nv[1] + tr[2] * nv[2];
        double wx = tr[0] - tn * nv[0], wy = tr[1] - tn * nv[1], wz = tr[2] - tn * nv[2];
        wss_out[s] = sqrt(wx * wx + wy * wy + wz * wz);
    }
}

/* Number of threads the OpenMP runtime will use (for reporting). */
int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
