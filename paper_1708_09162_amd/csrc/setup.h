// Host-side structures of libigabem: geometry, element tiles, cluster tree,
// block partition and the element-pair work lists handed to the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/igabem.h"

namespace igb {

struct Patch {
    int pu, pv, nu, nv;
    std::vector<double> U, V;
    std::vector<double> cpw;  // nv*nu*4, (x,y,z,w)
};

struct Geometry {
    std::vector<Patch> patches;
};

// Element-pair classes (same numbering as the exported diagnostics).
enum PairClass { kRegular = 0, kIdentical = 1, kEdge = 2, kVertex = 3 };

// One near-field element pair, E <= F in global row-major element order.
// frames: canonical (0,0), (1,0), (0,1) corners of E and of F (Sec. 4 item 4 rules).
struct PairRec {
    int32_t E, F;
    int32_t cls, order;
    int32_t blk1;   // near block (leaf(E), leaf(F)), sub-block (elE, elF)
    int32_t blk2;   // near block (leaf(F), leaf(E)), or -1 when E == F
    int8_t elE, elF;
    int8_t oE, aE, bE, oF, aF, bF;
};

struct Setup {
    // parameters
    int kernel = 0;
    double kappa = 0.0;
    int p = 0, m = 0, q = 1, d = 0, L = 0;
    double eta = 1.0;
    double kappa_diam = 0.0;  // > 0: blocks with kappa max(diam) above it are not admissible
    double hull_c[3] = {0.0, 0.0, 0.0}, hull_r = 0.0;  // ball around the control points' bounding box
    int g0 = 6, gs = 8, grhs = 6;
    int mode = 0;
    // derived sizes
    int npatch = 0, ne = 1, nelem = 0, nloc = 1, ns1 = 1;
    int64_t nsup = 0, ndof = 0;
    int side = 1;        // elements per leaf side (2^d)
    int nl = 1;          // superspace functions per leaf (4^d nloc)
    int n1 = 1;          // 1D leaf functions per direction (2^d (p+1))
    int nleaf = 0;       // clusters at level L
    // element geometry: homogeneous rational Bezier tiles, stride tile_stride doubles
    int tile_degree = 1;             // common bidegree of all tiles (1, 2, 4 or 8)
    int tile_stride = 0;
    std::vector<int32_t> tile_deg;   // per element: pu, pv
    std::vector<double> tiles;
    // B-spline -> Bernstein band: Tb[(e*(p+1) + r)*(p+1) + jj] = T1[e+jj, (e,r)]
    std::vector<double> Tb;
    // Chebyshev nodes, moments and transfers
    std::vector<double> z;           // q
    std::vector<double> M1;          // n1 x q, leaf moments
    std::vector<double> E2;          // 2 x q x q: E_c[nu][mu] = L_mu((c + z_nu)/2)
    std::vector<double> Mlev;        // per level l: (2^(m-l) (p+1)) x q direct 1D moments (diag kernel)
    std::vector<int64_t> Mlev_off;   // offsets into Mlev per level
    // level layout of clusters: global index = cl_off[l] + id
    std::vector<int64_t> cl_off;     // size L+2
    // partition (sorted)
    std::vector<int32_t> near;       // pairs (tgt, src)
    std::vector<int32_t> far;        // triples (level, tgt, src)
    std::vector<int64_t> near_ptr;   // CSR over target leaves (nleaf+1)
    std::vector<int32_t> near_src;
    std::vector<int64_t> far_ptr;    // CSR over global clusters
    std::vector<int32_t> far_src;    // global cluster index of sources
    // element corners (4 x 3), 3x3 grids (9 x 3), grid diameters and the radius of
    // the grid about its centre point (grid point 4)
    std::vector<double> ecorner, egrid, ediam, erad;
    // near-field element pairs, grouped: regular pairs of Gauss order g0, g0 + 2, g0 + 4 (capped at 40),
    // then the touching pairs; group k is pairs[pair_off[k] .. pair_off[k + 1])
    std::vector<PairRec> pairs;
    int64_t pair_off[5] = {0, 0, 0, 0, 0};
    int64_t npairs_class[4] = {0, 0, 0, 0};
    // Gauss rules on [0,1], orders 1..40, concatenated: gx[goff[n] + i]
    std::vector<double> gx, gw;
    std::vector<int32_t> goff;
    double setup_seconds = 0.0;
};

// Validation + copy of the patches; returns empty string or an error message.
std::string make_geometry(int32_t n, const igb_nurbs_patch *in, Geometry &out);

// Build everything host-side for the given parameters; returns "" or an error message.
// build_setup = build_setup_geometry (build_setup_tiles: parameters, element tiles,
// tables; then build_setup_elements: element corners, grids, diameters) followed by
// build_setup_plan (cluster tree, partition, near-field pairs).
std::string build_setup(const Geometry &g, const igb_params &prm, Setup &s);
std::string build_setup_geometry(const Geometry &g, const igb_params &prm, Setup &s);
std::string build_setup_tiles(const Geometry &g, const igb_params &prm, Setup &s);
void build_setup_elements(Setup &s);
std::string build_setup_plan(Setup &s);

// Bounds of the clusters of level l (level-local index patch 4^l + k2 2^l + k1), five doubles each: the
// centre (the cluster's mid parameter point), the largest distance from it to the cluster's 5 x 5 grid of
// surface points, and the grid's diameter (the quantities of the block admissibility).
void cluster_spheres(const Setup &s, int l, std::vector<double> &out);

// Touching element pairs (common edge, common vertex, and identical ones when
// with_identical; E <= F, sorted) from physical corner coincidence alone, without
// the partition.  Every touching pair lies in the near field, so this list equals
// the touching part of the plan.  Needs the element geometry.
std::string enumerate_touching(const Setup &s, std::vector<PairRec> &out, bool with_identical);
// "" if the touching pairs of the plan, sorted by (E, F), are exactly `touch`
// (class, order, frames); the sorted plan records (with their block indices)
// are returned through plan_touch when it is not null.
std::string check_touching(const Setup &s, const std::vector<PairRec> &touch, std::vector<PairRec> *plan_touch = nullptr);
// n_pairs x 4 (E, F, class, order) of the near-field pairs, sorted by (E, F).
void sorted_pair_classes(const Setup &s, int32_t *out);

// Host evaluation of an element tile: point and surface measure w.r.t. element-local coordinates.
void tile_eval(const Setup &s, int E, double u, double v, double X[3], double *kap_local);

// Gauss-Legendre rule on [0,1] with n points (ascending).
void gauss_rule(int n, double *x, double *w);

}  // namespace igb
