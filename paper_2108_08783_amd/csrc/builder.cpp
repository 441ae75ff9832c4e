// Host-side geometry plan (see builder.hpp).
#include "builder.hpp"

#include <cmath>
#include <cstring>
#include <sstream>

#include "d3q19.hpp"

namespace lbm {

std::string build_plan(const lbm_instance_desc* desc, int n_inst, Plan& plan) {
    if (n_inst <= 0) return "n_inst must be positive";
    if (!desc) return "instance descriptor array is NULL";
    plan = Plan();
    plan.inst.resize(n_inst);
    int64_t total = 0;
    // pass 1: counts and validation
    for (int k = 0; k < n_inst; ++k) {
        const lbm_instance_desc& d = desc[k];
        if (!d.labels) return "instance " + std::to_string(k) + ": labels is NULL";
        if (d.nx < 3 || d.ny < 3 || d.nz < 3)
            return "instance " + std::to_string(k) + ": every dimension must be >= 3";
        InstanceGeom& g = plan.inst[k];
        g.nx = d.nx; g.ny = d.ny; g.nz = d.nz;
        g.offset = total;
        int64_t n = 0;
        const int64_t nxy = (int64_t)d.nx * d.ny;
        for (int z = 0; z < d.nz; ++z)
            for (int y = 0; y < d.ny; ++y) {
                const uint8_t* row = d.labels + z * nxy + (int64_t)y * d.nx;
                const bool edge = (z == 0 || z == d.nz - 1 || y == 0 || y == d.ny - 1);
                for (int x = 0; x < d.nx; ++x) {
                    if (row[x] != LBM_LABEL_FLUID) continue;
                    if (edge || x == 0 || x == d.nx - 1) {
                        std::ostringstream s;
                        s << "instance " << k << ": fluid voxel on the array border at (" << x
                          << "," << y << "," << z << ")";
                        return s.str();
                    }
                    ++n;
                }
            }
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
    // pass 2: index grid and link classification per instance
    for (int k = 0; k < n_inst; ++k) {
        const lbm_instance_desc& d = desc[k];
        InstanceGeom& g = plan.inst[k];
        const int64_t nxy = (int64_t)d.nx * d.ny, nvox = nxy * d.nz;
        std::vector<int32_t> index(nvox, -1);
        int32_t next = 0;
        for (int64_t v = 0; v < nvox; ++v)
            if (d.labels[v] == LBM_LABEL_FLUID) index[v] = next++;
        g.iolet_used.assign(254, 0);
        int max_seg = 0, max_io = -1;
        g.wall_begin = (int64_t)plan.wall_site.size();
        int64_t s = 0;
        for (int z = 1; z < d.nz - 1; ++z)
            for (int y = 1; y < d.ny - 1; ++y)
                for (int x = 1; x < d.nx - 1; ++x) {
                    const int64_t v = z * nxy + (int64_t)y * d.nx + x;
                    if (d.labels[v] != LBM_LABEL_FLUID) continue;
                    const int64_t gs = g.offset + s;
                    plan.site_inst[gs] = (uint32_t)k;
                    const uint16_t seg = d.segment ? d.segment[v] : 0;
                    plan.site_seg[gs] = seg;
                    if (seg > max_seg) max_seg = seg;
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
                            if (a > plan.max_abs_offset) plan.max_abs_offset = a;
                        } else if (lab == LBM_LABEL_WALL) {
                            code = H_WALL;
                            ++nwall;
                            gx -= CX[i]; gy -= CY[i]; gz -= CZ[i];
                            ++plan.n_wall_links;
                        } else {
                            const int id = lab - LBM_LABEL_IOLET0;
                            if (sid >= 0 && sid != id) {
                                std::ostringstream m;
                                m << "instance " << k << ": fluid site (" << x << "," << y << ","
                                  << z << ") touches iolets " << sid << " and " << id;
                                return m.str();
                            }
                            sid = id;
                            g.iolet_used[id] = 1;
                            if (id > max_io) max_io = id;
                            code = H_IOLET;
                            ++plan.n_iolet_links;
                        }
                        plan.nbr[(size_t)(i - 1) * N + gs] = code;
                    }
                    if (sid >= 0) plan.site_iolet[gs] = (uint8_t)sid;
                    if (nwall > 0) {
                        plan.wall_site.push_back((int32_t)gs);
                        double nxv, nyv, nzv;
                        if (d.normal) {
                            nxv = d.normal[3 * v]; nyv = d.normal[3 * v + 1]; nzv = d.normal[3 * v + 2];
                        } else {
                            nxv = gx; nyv = gy; nzv = gz;
                        }
                        const double nn = std::sqrt(nxv * nxv + nyv * nyv + nzv * nzv);
                        if (nn > 0) { nxv /= nn; nyv /= nn; nzv /= nn; }
                        plan.wall_normal.push_back(nxv);
                        plan.wall_normal.push_back(nyv);
                        plan.wall_normal.push_back(nzv);
                    }
                    ++s;
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
    for (int64_t x = 0; x < N; ++x) {
        const uint32_t k = plan.site_inst[x];
        uint32_t wmask = 0, imask = 0;
        for (int i = 1; i < Q; ++i) {
            const int32_t c = plan.nbr[(size_t)(i - 1) * N + x];
            if (c == H_WALL && mode[k] == LBM_WALL_ELASTIC) wmask |= 1u << i;
            if (c == H_IOLET) imask |= 1u << i;
        }
        if (!(wmask | imask)) continue;
        out.site.push_back((int32_t)x);
        out.wall.push_back(wmask | (k << 19));
        const uint32_t slot = imask ? (uint32_t)(iolet_off[k] + plan.site_iolet[x]) : 0u;
        out.io.push_back(imask | (slot << 19));
        out.kidx.push_back(seg_off[k] + plan.site_seg[x]);
        out.weight.push_back(plan.site_w[x]);
    }
}

template <typename I>
void build_device_nbr(const Plan& plan, const std::vector<int>& mode, int64_t n_pad,
                      std::vector<I>& out) {
    const int64_t N = plan.N;
    out.assign((size_t)18 * n_pad, (I)0);
    for (int i = 1; i < Q; ++i) {
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
}

template void build_device_nbr<int32_t>(const Plan&, const std::vector<int>&, int64_t,
                                        std::vector<int32_t>&);
template void build_device_nbr<int16_t>(const Plan&, const std::vector<int>&, int64_t,
                                        std::vector<int16_t>&);

}  // namespace lbm
