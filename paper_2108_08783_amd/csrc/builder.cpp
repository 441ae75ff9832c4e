// Host-side geometry plan (see builder.hpp).
#include "builder.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <sstream>
#include <thread>

#include "d3q19.hpp"

namespace lbm {

namespace {

// Host worker threads for the O(N) passes (at most 16: the CPU share of one
// GPU on a shared host).
int n_workers(int64_t work) {
    const unsigned h = std::thread::hardware_concurrency();
    const int t = (int)std::min<unsigned>(h ? h : 1u, 16u);
    return work < (int64_t)1 << 16 ? 1 : t;
}

// Runs f(t, begin, end) on contiguous chunks [begin, end) of [0, n), one per
// worker, in order of t.
template <typename F>
void parallel_chunks(int64_t n, int workers, F f) {
    if (workers <= 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + workers - 1) / workers;
    for (int t = 0; t < workers; ++t) {
        const int64_t b = std::min(n, t * chunk), e = std::min(n, (t + 1) * chunk);
        th.emplace_back([=, &f] { f(t, b, e); });
    }
    for (auto& x : th) x.join();
}

}  // namespace

std::string build_plan(const lbm_instance_desc* desc, int n_inst, Plan& plan) {
    if (n_inst <= 0) return "n_inst must be positive";
    if (!desc) return "instance descriptor array is NULL";
    plan = Plan();
    plan.inst.resize(n_inst);
    int64_t total = 0;
    // pass 1: fluid voxels per z-slice (parallel over slices), validation
    std::vector<std::vector<int64_t>> slice_start(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const lbm_instance_desc& d = desc[k];
        if (!d.labels) return "instance " + std::to_string(k) + ": labels is NULL";
        if (d.nx < 3 || d.ny < 3 || d.nz < 3)
            return "instance " + std::to_string(k) + ": every dimension must be >= 3";
        InstanceGeom& g = plan.inst[k];
        g.nx = d.nx; g.ny = d.ny; g.nz = d.nz;
        g.offset = total;
        const int64_t nxy = (int64_t)d.nx * d.ny;
        std::vector<int64_t> cnt(d.nz, 0);
        std::vector<std::string> err(16);
        const int W = n_workers(nxy * d.nz);
        parallel_chunks(d.nz, W, [&](int t, int64_t z0, int64_t z1) {
            for (int64_t z = z0; z < z1 && err[t].empty(); ++z)
                for (int y = 0; y < d.ny; ++y) {
                    const uint8_t* row = d.labels + z * nxy + (int64_t)y * d.nx;
                    const bool edge = (z == 0 || z == d.nz - 1 || y == 0 || y == d.ny - 1);
                    for (int x = 0; x < d.nx; ++x) {
                        if (row[x] != LBM_LABEL_FLUID) continue;
                        if (edge || x == 0 || x == d.nx - 1) {
                            std::ostringstream m;
                            m << "instance " << k << ": fluid voxel on the array border at (" << x
                              << "," << y << "," << z << ")";
                            err[t] = m.str();
                            break;
                        }
                        ++cnt[z];
                    }
                }
        });
        for (const auto& e : err)
            if (!e.empty()) return e;
        slice_start[k].assign(d.nz + 1, 0);
        for (int z = 0; z < d.nz; ++z) slice_start[k][z + 1] = slice_start[k][z] + cnt[z];
        const int64_t n = slice_start[k][d.nz];
        if (n == 0) return "instance " + std::to_string(k) + ": no fluid voxel";
        g.n = n;
        total += n;
    }
    if (total >= (int64_t)INT32_MAX - 1024) return "too many sites for 32-bit site indices";
    plan.N = total;
    const int64_t N = total;
    plan.nbr.assign((size_t)18 * N, 0);
    plan.site_iolet.assign(N, 255);
    plan.site_seg.assign(N, 0);
    plan.site_w.assign(N, 1.0f);
    plan.site_inst.assign(N, 0);
    // pass 2 per instance: index grid, then the link classification of every
    // site; z-slabs in parallel, per-slab results merged in slab order
    struct Part {
        std::string err;
        int64_t max_abs = 0, n_wall = 0, n_io = 0;
        int max_seg = 0, max_io = -1;
        std::vector<uint8_t> used;
        std::vector<int32_t> wall_site;
        std::vector<double> wall_normal;
    };
    for (int k = 0; k < n_inst; ++k) {
        const lbm_instance_desc& d = desc[k];
        InstanceGeom& g = plan.inst[k];
        const int64_t nxy = (int64_t)d.nx * d.ny, nvox = nxy * d.nz;
        const std::vector<int64_t>& ss = slice_start[k];
        std::vector<int32_t> index(nvox, -1);
        const int W = n_workers(nvox);
        parallel_chunks(d.nz, W, [&](int, int64_t z0, int64_t z1) {
            for (int64_t z = z0; z < z1; ++z) {
                int32_t next = (int32_t)ss[z];
                for (int64_t v = z * nxy; v < (z + 1) * nxy; ++v)
                    if (d.labels[v] == LBM_LABEL_FLUID) index[v] = next++;
            }
        });
        std::vector<Part> parts(W);
        parallel_chunks(d.nz - 2, W, [&](int t, int64_t b, int64_t e) {
            Part& P = parts[t];
            P.used.assign(254, 0);
            for (int64_t z = b + 1; z < e + 1 && P.err.empty(); ++z) {
                int64_t s = ss[z];
                for (int y = 1; y < d.ny - 1 && P.err.empty(); ++y)
                    for (int x = 1; x < d.nx - 1; ++x) {
                        const int64_t v = z * nxy + (int64_t)y * d.nx + x;
                        if (d.labels[v] != LBM_LABEL_FLUID) continue;
                        const int64_t gs = g.offset + s;
                        plan.site_inst[gs] = (uint32_t)k;
                        const uint16_t seg = d.segment ? d.segment[v] : 0;
                        plan.site_seg[gs] = seg;
                        if (seg > P.max_seg) P.max_seg = seg;
                        plan.site_w[gs] = d.iolet_weight ? d.iolet_weight[v] : 1.0f;
                        int nwall = 0, sid = -1;
                        float gx = 0, gy = 0, gz = 0;
                        for (int i = 1; i < Q; ++i) {
                            const int64_t u = v - CX[i] - (int64_t)CY[i] * d.nx - CZ[i] * nxy;
                            const uint8_t lab = d.labels[u];
                            int32_t code;
                            if (lab == LBM_LABEL_FLUID) {
                                const int64_t off = (int64_t)index[u] - s;
                                code = (int32_t)off;
                                const int64_t a = off < 0 ? -off : off;
                                if (a > P.max_abs) P.max_abs = a;
                            } else if (lab == LBM_LABEL_WALL) {
                                code = H_WALL;
                                ++nwall;
                                gx -= CX[i]; gy -= CY[i]; gz -= CZ[i];
                                ++P.n_wall;
                            } else {
                                const int id = lab - LBM_LABEL_IOLET0;
                                if (sid >= 0 && sid != id) {
                                    std::ostringstream m;
                                    m << "instance " << k << ": fluid site (" << x << "," << y << ","
                                      << z << ") touches iolets " << sid << " and " << id;
                                    P.err = m.str();
                                }
                                sid = id;
                                P.used[id] = 1;
                                if (id > P.max_io) P.max_io = id;
                                code = H_IOLET;
                                ++P.n_io;
                            }
                            plan.nbr[(size_t)(i - 1) * N + gs] = code;
                        }
                        if (sid >= 0) plan.site_iolet[gs] = (uint8_t)sid;
                        if (nwall > 0) {
                            P.wall_site.push_back((int32_t)gs);
                            double nxv, nyv, nzv;
                            if (d.normal) {
                                nxv = d.normal[3 * v]; nyv = d.normal[3 * v + 1]; nzv = d.normal[3 * v + 2];
                            } else {
                                nxv = gx; nyv = gy; nzv = gz;
                            }
                            const double nn = std::sqrt(nxv * nxv + nyv * nyv + nzv * nzv);
                            if (nn > 0) { nxv /= nn; nyv /= nn; nzv /= nn; }
                            P.wall_normal.push_back(nxv);
                            P.wall_normal.push_back(nyv);
                            P.wall_normal.push_back(nzv);
                        }
                        ++s;
                    }
            }
        });
        g.iolet_used.assign(254, 0);
        int max_seg = 0, max_io = -1;
        g.wall_begin = (int64_t)plan.wall_site.size();
        for (const Part& P : parts) {
            if (!P.err.empty()) return P.err;
            plan.max_abs_offset = std::max(plan.max_abs_offset, P.max_abs);
            plan.n_wall_links += P.n_wall;
            plan.n_iolet_links += P.n_io;
            max_seg = std::max(max_seg, P.max_seg);
            max_io = std::max(max_io, P.max_io);
            for (size_t j = 0; j < P.used.size(); ++j) g.iolet_used[j] |= P.used[j];
            plan.wall_site.insert(plan.wall_site.end(), P.wall_site.begin(), P.wall_site.end());
            plan.wall_normal.insert(plan.wall_normal.end(), P.wall_normal.begin(),
                                    P.wall_normal.end());
        }
        g.wall_end = (int64_t)plan.wall_site.size();
        g.n_seg = max_seg + 1;
        g.n_iolet = max_io + 1;
    }
    return "";
}

void build_boundary(const Plan& plan, const std::vector<int>& mode,
                    const std::vector<int>& seg_off, const std::vector<int>& iolet_off,
                    BoundaryList& out) {
    out = BoundaryList();
    const int64_t N = plan.N;
    out.rec_of_site.assign(N, -1);
    auto classify = [&](int64_t x, uint32_t& wmask, uint32_t& imask) {
        const uint32_t k = plan.site_inst[x];
        wmask = 0;
        imask = 0;
        bool irregular = false;
        for (int i = 1; i < Q; ++i) {
            const int32_t c = plan.nbr[(size_t)(i - 1) * N + x];
            if (c == H_WALL || c == H_IOLET) irregular = true;
            if (c == H_WALL && mode[k] == LBM_WALL_ELASTIC) wmask |= 1u << i;
            if (c == H_IOLET) imask |= 1u << i;
        }
        return irregular;
    };
    // irregular sites per chunk, then every record at its final position
    const int W = n_workers(N);
    std::vector<int64_t> cnt(W + 1, 0), gcnt(W + 1, 0);
    parallel_chunks(N, W, [&](int t, int64_t b, int64_t e) {
        uint32_t wm, im;
        for (int64_t x = b; x < e; ++x)
            if (classify(x, wm, im)) {
                ++cnt[t + 1];
                if (wm | im) ++gcnt[t + 1];
            }
    });
    for (int t = 0; t < W; ++t) {
        cnt[t + 1] += cnt[t];
        gcnt[t + 1] += gcnt[t];
    }
    const int64_t nr = cnt[W];
    out.site.resize(nr);
    out.wall.resize(nr);
    out.io.resize(nr);
    out.kidx.resize(nr);
    out.weight.resize(nr);
    out.ghost.resize(gcnt[W]);
    parallel_chunks(N, W, [&](int t, int64_t b, int64_t e) {
        int64_t id = cnt[t], gid = gcnt[t];
        uint32_t wmask, imask;
        for (int64_t x = b; x < e; ++x) {
            if (!classify(x, wmask, imask)) continue;
            const uint32_t k = plan.site_inst[x];
            out.rec_of_site[x] = (int32_t)id;
            out.site[id] = (int32_t)x;
            out.wall[id] = wmask | (k << 19);
            const uint32_t slot = imask ? (uint32_t)(iolet_off[k] + plan.site_iolet[x]) : 0u;
            out.io[id] = imask | (slot << 19);
            out.kidx[id] = seg_off[k] + plan.site_seg[x];
            out.weight[id] = plan.site_w[x];
            if (wmask | imask) out.ghost[gid++] = (int32_t)id;
            ++id;
        }
    });
}

namespace {

// Stretch slot of direction i's upstream row (y - cy, z - cz); -1 for the
// site's own row.
int row_of(int i) {
    if (CY[i] == 0 && CZ[i] == 0) return -1;
    for (int r = 0; r < 8; ++r)
        if (ROW8[r][0] == -CY[i] && ROW8[r][1] == -CZ[i]) return r;
    return -1;
}

bool is_sentinel(int32_t v) { return v <= Sentinel<int32_t>::GHOST; }

}  // namespace

std::string build_compressed(const Plan& plan, const BoundaryList& bl,
                             const std::vector<int32_t>& nbr_dev32, int64_t n_pad, Compressed& out) {
    out = Compressed();
    const int64_t N = plan.N;
    const int64_t nwf = n_pad / 64;
    int rowi[Q];
    for (int i = 0; i < Q; ++i) rowi[i] = row_of(i);
    auto tab = [&](int i, int64_t x) { return nbr_dev32[(size_t)(i - 1) * n_pad + x]; };

    // pass 1: row constraints of every site; exceptional sites
    out.n_irr = (int64_t)bl.site.size();
    out.nfm.assign((size_t)std::max<int64_t>(out.n_irr, 1), 0u);
    std::vector<int32_t> exc_sites;
    std::vector<uint8_t> exceptional(N, 0);
    for (int64_t j = 0; j < out.n_irr; ++j) {
        const int64_t x = bl.site[j];
        uint32_t m = 0;
        bool ghost = false, bad = false;
        int32_t C[8];
        bool has[8] = {false};
        for (int i = 1; i < Q; ++i) {
            const int32_t v = tab(i, x);
            if (is_sentinel(v)) {
                m |= 1u << (i - 1);
                ghost |= v == Sentinel<int32_t>::GHOST;
                continue;
            }
            const int r = rowi[i];
            if (r < 0) {
                bad |= v != -CX[i];
            } else if (has[r]) {
                bad |= C[r] != v + CX[i];
            } else {
                has[r] = true;
                C[r] = v + CX[i];
            }
        }
        out.nfm[j] = m | (ghost ? 1u << 31 : 0u);
        if (bad) {
            exceptional[x] = 1;
            exc_sites.push_back((int32_t)x);
        }
    }
    out.n_exc = (int64_t)exc_sites.size();
    out.n_exc_pad = std::max<int64_t>(256, (out.n_exc + 255) / 256 * 256);
    out.exc.assign((size_t)18 * out.n_exc_pad, Sentinel<int32_t>::BB);
    for (int64_t e = 0; e < out.n_exc; ++e)
        for (int i = 1; i < Q; ++i) out.exc[(size_t)(i - 1) * out.n_exc_pad + e] = tab(i, exc_sites[e]);

    // pass 2: stretches (greedy: a site joins the current stretch when its
    // fluid row links agree with the entries already set) and the records
    out.wf.assign((size_t)nwf, WfRec{});
    int32_t cur = -1, nirr = 0, nexc = 0;
    int32_t D[8] = {0};
    bool known[8] = {false};
    for (int64_t w = 0; w < nwf; ++w) {
        WfRec& R = out.wf[w];
        R.cur = cur;
        R.firr = nirr;
        R.fexc = nexc;
        R.pad = 0;
        R.smask = R.imask = R.emask = R.pad2 = 0;
        for (int l = 0; l < 64; ++l) {
            const int64_t x = w * 64 + l;
            if (x >= N) break;
            const bool irr = bl.rec_of_site[x] >= 0;
            if (irr) {
                R.imask |= 1ull << l;
                ++nirr;
            }
            if (exceptional[x]) {
                R.emask |= 1ull << l;
                ++nexc;
                continue;
            }
            int32_t C[8];
            bool has[8] = {false};
            for (int i = 1; i < Q; ++i) {
                const int32_t v = tab(i, x);
                if (is_sentinel(v) || rowi[i] < 0) continue;
                has[rowi[i]] = true;
                C[rowi[i]] = v + CX[i];
            }
            bool fits = cur >= 0;
            for (int r = 0; r < 8 && fits; ++r) fits = !has[r] || !known[r] || D[r] == C[r];
            if (!fits) {
                ++cur;
                for (int r = 0; r < 8; ++r) {
                    known[r] = has[r];
                    D[r] = has[r] ? C[r] : 0;
                }
                out.stretch.insert(out.stretch.end(), D, D + 8);
                R.smask |= 1ull << l;
            } else {
                for (int r = 0; r < 8; ++r)
                    if (has[r] && !known[r]) {
                        known[r] = true;
                        D[r] = C[r];
                        out.stretch[(size_t)8 * cur + r] = C[r];
                    }
            }
        }
    }
    out.n_stretch = cur + 1;
    if (out.stretch.empty()) out.stretch.assign(8, 0);
    if (nirr != out.n_irr) return "compressed addressing: irregular-site count mismatch";

    auto check_range = [&](int64_t b0, int64_t e0) -> std::string {
    for (int64_t x = b0; x < e0; ++x) {
        const WfRec& R = out.wf[x >> 6];
        const int l = (int)(x & 63);
        const uint64_t bit = 1ull << l, below = bit - 1ull;
        int st = R.cur + __builtin_popcountll(R.smask & (bit | below));
        st = st < 0 ? 0 : st;
        uint32_t nf = 0;
        if (R.imask & bit) {
            const int64_t id = R.firr + __builtin_popcountll(R.imask & below);
            if (bl.site[id] != x) return "compressed addressing: irregular id mismatch at site " +
                                         std::to_string(x);
            nf = out.nfm[id];
        }
        const bool exc = (R.emask & bit) != 0;
        const int64_t eid = R.fexc + __builtin_popcountll(R.emask & below);
        bool ghost_tab = false, ghost_rec = false;
        for (int i = 1; i < Q; ++i) {
            const int32_t want = tab(i, x);
            ghost_tab |= want == Sentinel<int32_t>::GHOST;
            int32_t got;
            if (exc) {
                got = out.exc[(size_t)(i - 1) * out.n_exc_pad + eid];
            } else if ((nf >> (i - 1)) & 1u) {
                got = (nf >> 31) ? Sentinel<int32_t>::GHOST : Sentinel<int32_t>::BB;
            } else {
                got = (rowi[i] < 0 ? 0 : out.stretch[(size_t)8 * st + rowi[i]]) - CX[i];
            }
            ghost_rec |= got == Sentinel<int32_t>::GHOST;
            const bool ok = is_sentinel(want) ? is_sentinel(got) : got == want;
            if (!ok)
                return "compressed addressing: derived offset mismatch at site " + std::to_string(x);
        }
        if (ghost_tab != ghost_rec)
            return "compressed addressing: boundary-link flag mismatch at site " + std::to_string(x);
    }
        return std::string();
    };
    // check: the device's reconstruction reproduces the table at every site
    const int W = n_workers(N);
    std::vector<std::string> errs(W);
    parallel_chunks(N, W, [&](int t, int64_t b, int64_t e) {
        errs[t] = check_range(b, e);
    });
    for (const auto& e : errs)
        if (!e.empty()) return e;
    return "";
}


void refresh_compressed(const BoundaryList& bl, const std::vector<int32_t>& nbr_dev32,
                        int64_t n_pad, Compressed& c) {
    auto tab = [&](int i, int64_t x) { return nbr_dev32[(size_t)(i - 1) * n_pad + x]; };
    for (int64_t j = 0; j < c.n_irr; ++j) {
        const int64_t x = bl.site[j];
        bool ghost = false;
        for (int i = 1; i < Q; ++i) ghost |= tab(i, x) == Sentinel<int32_t>::GHOST;
        c.nfm[j] = (c.nfm[j] & 0x7FFFFFFFu) | (ghost ? 1u << 31 : 0u);
    }
    int64_t e = 0;
    for (const WfRec& R : c.wf) {
        uint64_t m = R.emask;
        const int64_t base = (int64_t)(&R - c.wf.data()) * 64;
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            for (int i = 1; i < Q; ++i) c.exc[(size_t)(i - 1) * c.n_exc_pad + e] = tab(i, base + l);
            ++e;
        }
    }
}

template <typename I>
void build_device_nbr(const Plan& plan, const std::vector<int>& mode, int64_t n_pad,
                      std::vector<I>& out) {
    const int64_t N = plan.N;
    out.assign((size_t)18 * n_pad, (I)0);
    parallel_chunks(18, std::min(18, n_workers(18 * N)), [&](int, int64_t i0, int64_t i1) {
    for (int i = (int)i0 + 1; i < (int)i1 + 1; ++i) {
        const int32_t* src = plan.nbr.data() + (size_t)(i - 1) * N;
        I* dst = out.data() + (size_t)(i - 1) * n_pad;
        for (int64_t x = 0; x < N; ++x) {
            const int32_t c = src[x];
            if (c == H_WALL)
                dst[x] = mode[plan.site_inst[x]] == LBM_WALL_ELASTIC ? Sentinel<I>::GHOST
                                                                     : Sentinel<I>::BB;
            else if (c == H_IOLET)
                dst[x] = Sentinel<I>::GHOST;
            else
                dst[x] = (I)c;
        }
        // padding sites read their own rest slot (never stored back)
        for (int64_t x = N; x < n_pad; ++x) dst[x] = Sentinel<I>::BB;
    }
    });
}

template void build_device_nbr<int32_t>(const Plan&, const std::vector<int>&, int64_t,
                                        std::vector<int32_t>&);
template void build_device_nbr<int16_t>(const Plan&, const std::vector<int>&, int64_t,
                                        std::vector<int16_t>&);


int choose_fast_axis(const lbm_instance_desc& d, int forced) {
    if (forced >= 0 && forced <= 2) return forced;
    if (!d.labels || d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return 0;
    const int64_t nx = d.nx, ny = d.ny, nxy = nx * ny;
    const int W = n_workers(nxy * d.nz);
    std::vector<std::array<int64_t, 4>> acc(W, std::array<int64_t, 4>{0, 0, 0, 0});
    parallel_chunks(d.nz, W, [&](int t, int64_t z0, int64_t z1) {
        std::array<int64_t, 4>& a = acc[t];   // fluid, runs along x, y, z
        for (int64_t z = z0; z < z1; ++z)
            for (int64_t y = 0; y < ny; ++y) {
                const uint8_t* L = d.labels + z * nxy + y * nx;
                for (int64_t x = 0; x < nx; ++x) {
                    if (L[x] != 1) continue;
                    ++a[0];
                    a[1] += x == 0 || L[x - 1] != 1;
                    a[2] += y == 0 || L[x - nx] != 1;
                    a[3] += z == 0 || L[x - nxy] != 1;
                }
            }
    });
    int64_t f = 0, r[3] = {0, 0, 0};
    for (const auto& a : acc) {
        f += a[0];
        for (int k = 0; k < 3; ++k) r[k] += a[k + 1];
    }
    if (f == 0) return 0;
    double mean[3];
    for (int k = 0; k < 3; ++k) mean[k] = (double)f / (double)std::max<int64_t>(1, r[k]);
    const int best = mean[2] > mean[1] ? 2 : 1;
    return mean[best] >= 1.25 * mean[0] ? best : 0;
}

void swap_axes(const lbm_instance_desc& d, int axis, SwappedGeom& out) {
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz;
    // new dimensions and the old coordinates of new voxel (x', y', z')
    const int64_t mx = axis == 1 ? ny : nz, my = axis == 1 ? nx : ny, mz = axis == 1 ? nz : nx;
    const int64_t nvox = nx * ny * nz;
    out.labels.assign((size_t)nvox, 0);
    if (d.segment) out.segment.assign((size_t)nvox, 0);
    if (d.normal) out.normal.assign((size_t)nvox * 3, 0.0f);
    if (d.iolet_weight) out.iolet_weight.assign((size_t)nvox, 0.0f);
    const int W = n_workers(nvox);
    parallel_chunks(mz, W, [&](int, int64_t z0, int64_t z1) {
        for (int64_t zp = z0; zp < z1; ++zp)
            for (int64_t yp = 0; yp < my; ++yp)
                for (int64_t xp = 0; xp < mx; ++xp) {
                    const int64_t x = axis == 1 ? yp : zp, y = axis == 1 ? xp : yp,
                                  z = axis == 1 ? zp : xp;
                    const int64_t o = (z * ny + y) * nx + x, v = (zp * my + yp) * mx + xp;
                    out.labels[v] = d.labels[o];
                    if (d.segment) out.segment[v] = d.segment[o];
                    if (d.iolet_weight) out.iolet_weight[v] = d.iolet_weight[o];
                    if (d.normal)
                        for (int a = 0; a < 3; ++a) {
                            const int src = a == 0 ? axis : (a == axis ? 0 : a);
                            out.normal[3 * v + a] = d.normal[3 * o + src];
                        }
                }
    });
    out.desc.nx = (int32_t)mx;
    out.desc.ny = (int32_t)my;
    out.desc.nz = (int32_t)mz;
    out.desc.labels = out.labels.data();
    out.desc.segment = d.segment ? out.segment.data() : nullptr;
    out.desc.normal = d.normal ? out.normal.data() : nullptr;
    out.desc.iolet_weight = d.iolet_weight ? out.iolet_weight.data() : nullptr;
}

void site_map(const lbm_instance_desc& d, int axis, const SwappedGeom& sw,
              std::vector<int32_t>& c2i) {
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz;
    // canonical index of the first fluid voxel of every original row (y, z)
    std::vector<int64_t> start((size_t)(ny * nz) + 1, 0);
    for (int64_t r = 0; r < ny * nz; ++r) {
        const uint8_t* L = d.labels + r * nx;
        int64_t n = 0;
        for (int64_t x = 0; x < nx; ++x) n += L[x] == 1;
        start[r + 1] = start[r] + n;
    }
    c2i.assign((size_t)start[ny * nz], 0);
    // internal order visits the voxels of one original row with increasing x
    // (x is the slowest or the middle loop of the exchanged raster), so a
    // counter per row gives each voxel's canonical rank within its row
    std::vector<int64_t> cnt((size_t)(ny * nz), 0);
    const int64_t mx = sw.desc.nx, my = sw.desc.ny, mz = sw.desc.nz;
    int64_t j = 0;
    for (int64_t zp = 0; zp < mz; ++zp)
        for (int64_t yp = 0; yp < my; ++yp) {
            const uint8_t* L = sw.labels.data() + (zp * my + yp) * mx;
            for (int64_t xp = 0; xp < mx; ++xp) {
                if (L[xp] != 1) continue;
                const int64_t y = axis == 1 ? xp : yp, z = axis == 1 ? zp : xp;
                const int64_t r = z * ny + y;
                c2i[(size_t)(start[r] + cnt[r]++)] = (int32_t)j++;
            }
        }
}

}  // namespace lbm
