// Host-side geometry plan: fluid-site enumeration, the per-link
// classification of Sec. 2.3 (fluid / wall / iolet upstream voxel), the pull
// (neighbour) table and the compacted boundary list.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "d3q19.hpp"

namespace lbm {

// Host classification sentinels (before the wall mode is applied).
constexpr int32_t H_WALL = INT32_MIN;
constexpr int32_t H_IOLET = INT32_MIN + 1;

struct InstanceGeom {
    int nx = 0, ny = 0, nz = 0;
    int64_t offset = 0;   // first global site
    int64_t n = 0;        // sites
    int n_seg = 1;        // max segment id at fluid voxels + 1
    int n_iolet = 0;      // max iolet id adjacent to a fluid site + 1
    std::vector<uint8_t> iolet_used;  // per id: some link reads it
    int64_t wall_begin = 0, wall_end = 0;  // range in the wall-site list
};

struct Plan {
    int64_t N = 0;
    std::vector<InstanceGeom> inst;
    // nbr[(i-1)*N + x]: offset d (upstream = x + d) or H_WALL / H_IOLET.
    std::vector<int32_t> nbr;
    std::vector<uint8_t> site_iolet;   // iolet id of the site's iolet links, 255 if none
    std::vector<uint16_t> site_seg;
    std::vector<float> site_w;         // iolet profile weight
    std::vector<uint32_t> site_inst;
    // sites with at least one wall link, ascending
    std::vector<int32_t> wall_site;
    std::vector<double> wall_normal;   // 3 per wall site (unit, normalised in FP64)
    int64_t n_wall_links = 0, n_iolet_links = 0;
    int64_t max_abs_offset = 0;
};

// Returns an empty string on success, else the reason.
std::string build_plan(const lbm_instance_desc* desc, int n_inst, Plan& plan);

// Site order of an instance.  Sites are updated in raster order with x
// fastest, and the compressed addressing and the boundary work favour long
// runs of fluid voxels along that axis.  An instance whose fluid runs are
// clearly longer along y or z (mean run at least 1.25 times that along x)
// is therefore stored with that axis exchanged for x; the exchange is an
// involution on positions, velocities and directions, applied at the C ABI.
// Returns 0 (keep x), 1 (exchange x and y) or 2 (exchange x and z); forced
// in {0, 1, 2} overrides the choice, -1 chooses.  An instance without
// labels or with empty dimensions keeps 0 (build_plan reports it).
int choose_fast_axis(const lbm_instance_desc& d, int forced);

// The instance with axes x and `axis` exchanged, in owning arrays (desc
// points into them; optional arrays stay NULL; normals have their
// components exchanged too).
struct SwappedGeom {
    std::vector<uint8_t> labels;
    std::vector<uint16_t> segment;
    std::vector<float> normal, iolet_weight;
    lbm_instance_desc desc{};
};
void swap_axes(const lbm_instance_desc& d, int axis, SwappedGeom& out);

// c2i[canonical local site] = internal local site: canonical order is the
// raster order (x fastest) of the fluid voxels of d, internal order the
// raster order of the exchanged geometry (sw, built by swap_axes).
void site_map(const lbm_instance_desc& d, int axis, const SwappedGeom& sw,
              std::vector<int32_t>& c2i);

// Irregular sites: every site with at least one non-fluid link, in site
// order.  Each carries a boundary record; the records with elastic-wall or
// iolet links (the boundary pass) are listed in `ghost`.  The wall mode per
// instance (0 bounce-back, 1 elastic) decides which wall links are
// bounce-back redirects and which go through the boundary rule.
struct BoundaryList {
    std::vector<int32_t> site;    // irregular site indices
    std::vector<uint32_t> wall;   // bits 1..18 elastic wall links | inst << 19
    std::vector<uint32_t> io;     // bits 1..18 iolet links | global iolet slot << 19
    std::vector<int32_t> kidx;    // index into the global stiffness table
    std::vector<float> weight;    // iolet profile weight
    std::vector<int32_t> ghost;   // record ids with boundary-pass links
    std::vector<int32_t> rec_of_site;  // per site: record id or -1
};

void build_boundary(const Plan& plan, const std::vector<int>& mode,
                    const std::vector<int>& seg_off, const std::vector<int>& iolet_off,
                    BoundaryList& out);

// Compressed addressing.  Offsets of a site follow from the 8 offsets
// d(dy,dz) to the voxel at the same x in the neighbouring rows (y+dy, z+dz):
// the upstream voxel of direction c is at d(-cy,-cz) - cx, and the
// x-neighbours in a row are consecutive sites.  Along a row that is one run
// of fluid voxels these 8 offsets are constant, also at the row's irregular
// sites for the links that reach fluid (a "stretch"); a stretch may leave
// entries unset that none of its sites uses.  Every site belongs to the
// current stretch unless it starts a new one; an irregular site carries an
// 18-bit mask of its non-fluid links (bit i-1 for direction i; bit 31: at
// least one of them is handled by the boundary rule).  The rare irregular
// sites whose fluid links disagree with any single stretch ("exceptional":
// a row of several runs) keep all 18 offsets.  Per wavefront of 64
// consecutive sites one record holds
//   cur    id of the stretch in effect before the wavefront
//   firr   id of the first irregular site at or after the wavefront start
//   fexc   id of the first exceptional site at or after the wavefront start
//   smask  bit l: site l starts a new stretch
//   imask  bit l: site l is irregular
//   emask  bit l: site l is exceptional (a subset of imask)
// so stretch(l) = cur + popcount(smask & bits 0..l), irregular id(l) =
// firr + popcount(imask & bits 0..l-1) (also the boundary record id) and
// exceptional id(l) = fexc + popcount(emask & bits 0..l-1).
struct Compressed {
    std::vector<WfRec> wf;
    std::vector<int32_t> stretch;  // 8 per stretch, (dy, dz) in order of ROW8
    std::vector<uint32_t> nfm;     // per irregular site: non-fluid link mask
    std::vector<int32_t> exc;      // 18 planes x n_exc_pad, Sentinel<int32_t> codes
    int64_t n_irr = 0, n_exc = 0, n_exc_pad = 0, n_stretch = 0;
};

// (dy, dz) of the 8 neighbouring rows, in stretch-table order.
constexpr int ROW8[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};

// Builds the compressed form from the device table (Sentinel<int32_t>
// codes, n_pad sites per plane) and checks that it reproduces the table at
// every site.  Returns an empty string on success.
std::string build_compressed(const Plan& plan, const BoundaryList& bl,
                             const std::vector<int32_t>& nbr_dev32, int64_t n_pad, Compressed& out);

// Rewrites the parts of a compressed form that depend on the wall modes
// (the boundary-rule flag of each link mask and the sentinels of the
// exceptional sites' offsets) from the device table of the current modes;
// which links are non-fluid, the stretches and the records do not change.
void refresh_compressed(const BoundaryList& bl, const std::vector<int32_t>& nbr_dev32,
                        int64_t n_pad, Compressed& c);

// Device neighbour table of width I for the given wall modes.
template <typename I>
void build_device_nbr(const Plan& plan, const std::vector<int>& mode, int64_t n_pad,
                      std::vector<I>& out);

}  // namespace lbm
