// libigabem: HIP kernels and C-ABI entry points for the isogeometric
// single-layer BEM with nested-basis (H2) interpolation compression.
// Target: gfx950 (MI355X), FP64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <atomic>
#include <mutex>
#include <set>
#include <thread>
#include <type_traits>
#include <string>
#include <type_traits>
#include <vector>

#include "cnn.h"
#include "kernels.h"
#include "setup.h"

using namespace igb;

static thread_local std::string g_err;

static igb_status fail(igb_status s, const std::string &m)
{
    g_err = m;
    return s;
}

void igb_set_error(const std::string &msg) { g_err = msg; }

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? IGB_ENOMEM : IGB_EHIP,                         \
                        std::string(#x) + ": " + hipGetErrorString(e_));                           \
    } while (0)

#define LAUNCHCHK()                                                                                \
    do {                                                                                           \
        hipError_t e_ = hipGetLastError();                                                         \
        if (e_ != hipSuccess) return fail(IGB_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

struct igb_geometry {
    Geometry g;
};

// ===========================================================================
// kernels: geometry
// ===========================================================================

// Geometry at the tensor Gauss nodes of order g of every element:
// out[(E*g*g + j*g + i)*4 + {0,1,2,3}] = x, y, z, kappa_local * w_i * w_j.
__global__ void k_gauss_geom(int nelem, int stride, const double *__restrict__ tiles, const int32_t *__restrict__ tdeg,
                             int g, const double *__restrict__ x, const double *__restrict__ w, double *__restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int gg = g * g;
    if (idx >= (int64_t)nelem * gg) return;
    int E = (int)(idx / gg), k = (int)(idx % gg), j = k / g, i = k % g;
    double X[3], kap;
    tile_point(tiles + (size_t)E * stride, tdeg[2 * E], tdeg[2 * E + 1], x[i], x[j], X, &kap);
    out[idx * 4 + 0] = X[0];
    out[idx * 4 + 1] = X[1];
    out[idx * 4 + 2] = X[2];
    out[idx * 4 + 3] = kap * w[i] * w[j];
}

// Chebyshev-node geometry of every cluster (all levels): point and surface
// measure times the affine Jacobian 4^-l of the cluster map,
// nodes[(gc*q2 + mu)*4 + c], mu = mu2*q + mu1.
__global__ void k_cluster_nodes(int64_t ncl_all, int L, const int64_t *__restrict__ cl_off, int q, int m, int ne,
                                const double *__restrict__ z, int stride, const double *__restrict__ tiles,
                                const int32_t *__restrict__ tdeg, double *__restrict__ nodes)
{
    int q2 = q * q;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncl_all * q2) return;
    int64_t gc = idx / q2;
    int mu = (int)(idx % q2), mu2 = mu / q, mu1 = mu % q;
    int l = 0;
    while (l < L && gc >= cl_off[l + 1]) ++l;
    int id = (int)(gc - cl_off[l]);
    int n = 1 << l;
    int patch = id / (n * n), r = id % (n * n), k2 = r / n, k1 = r % n;
    double a = (k1 + z[mu1]) * (double)(ne >> l), b = (k2 + z[mu2]) * (double)(ne >> l);
    int e1 = (int)floor(a), e2 = (int)floor(b);
    e1 = e1 < 0 ? 0 : (e1 > ne - 1 ? ne - 1 : e1);
    e2 = e2 < 0 ? 0 : (e2 > ne - 1 ? ne - 1 : e2);
    int E = patch * ne * ne + e2 * ne + e1;
    double X[3], kap;
    tile_point(tiles + (size_t)E * stride, tdeg[2 * E], tdeg[2 * E + 1], a - e1, b - e2, X, &kap);
    // kappa_patch = kappa_local * ne^2; times 4^-l  ->  kappa_local * 4^(m-l)
    double sc = (double)(1LL << (2 * (m - l)));
    nodes[idx * 4 + 0] = X[0];
    nodes[idx * 4 + 1] = X[1];
    nodes[idx * 4 + 2] = X[2];
    nodes[idx * 4 + 3] = kap * sc;
}

// ===========================================================================
// kernels: near-field quadrature
// ===========================================================================

// Position of entry (row a of element elE, column b of element elF) in a
// column-major leaf block of nl columns with column stride ld (ld >= nl).
__device__ inline int64_t blk_pos(int ld, int nloc, int elE, int a, int elF, int b)
{
    return (int64_t)(elF * nloc + b) * ld + elE * nloc + a;
}

// Near-field storage: only the leaf blocks (t, s) with t <= s are kept (the
// Galerkin matrix is symmetric, complex symmetric for Helmholtz, so block
// (s, t) is the transpose of block (t, s)).  sb[e] is the stored block of CSR
// near entry e, or -1 for an entry with t > s.  A pair record writes its entry
// (E row, F column) into sb[blk1] and the mirrored entry into sb[blk2]; the
// lower one of the two is absent, and both land in the same block when
// leaf(E) == leaf(F).
template <class T>
__device__ inline void near_targets(const int32_t *sb, const PairRec &R, int64_t bsz, T *blocks, T *&out1, T *&out2)
{
    const int32_t b1 = sb[R.blk1], b2 = R.blk2 >= 0 ? sb[R.blk2] : -1;
    out1 = b1 >= 0 ? blocks + (int64_t)b1 * bsz : nullptr;
    out2 = b2 >= 0 ? blocks + (int64_t)b2 * bsz : nullptr;
}

// entries (sin, cos) of the sine/cosine table of the complex kernels (sincos_tab)
constexpr int kSinCosTab = 256;

// 1/sqrt(r2) for finite r2 > 0: the hardware estimate refined by the
// second-order expansion of (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8, e = 1 - r2 y^2.
__device__ inline double rsqrt_pos(double r2)
{
    double y = __builtin_amdgcn_rsq(r2);
    double e = fma(-r2 * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Well separated pairs: tensor Gauss of order g in all four variables.
// One workgroup per pair; kernel rows K(x_i, .) are formed by thread i and
// contracted with the Bernstein values of F, then with those of E.
template <class T, int P>
__global__ void __launch_bounds__(128) k_near_regular(const PairRec *__restrict__ pairs, int npairs, int g,
                                                      const double *__restrict__ gp, const double *__restrict__ btab,
                                                      double kappa, int nl, int ld, const int32_t *__restrict__ sb,
                                                      T *__restrict__ blocks, const double *__restrict__ sctab)
{
    constexpr int P1 = P + 1, NLOC = P1 * P1, TS = NLOC + 1;  // tmp row stride: rows on distinct banks
    extern __shared__ double sh[];
    int gg = g * g;
    double *X = sh;                        // gg*4
    double *Y = X + gg * 4;                // gg*4
    double *psi = Y + gg * 4;              // gg*NLOC
    T *tmp = (T *)(psi + (size_t)gg * NLOC);  // gg*TS
    PairRec R = pairs[blockIdx.x];
    const double *gE = gp + (size_t)R.E * gg * 4, *gF = gp + (size_t)R.F * gg * 4;
    for (int k = threadIdx.x; k < gg * 4; k += blockDim.x) {
        X[k] = gE[k];
        Y[k] = gF[k];
    }
    for (int k = threadIdx.x; k < gg * NLOC; k += blockDim.x) {
        int j = k / NLOC, b = k % NLOC;
        int j2 = j / g, j1 = j % g, b2 = b / P1, b1 = b % P1;
        psi[k] = btab[j1 * P1 + b1] * btab[j2 * P1 + b2];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < gg; i += blockDim.x) {
        T acc[NLOC];
#pragma unroll
        for (int b = 0; b < NLOC; ++b) acc[b] = zero<T>();
        double x0 = X[4 * i], x1 = X[4 * i + 1], x2 = X[4 * i + 2];
        for (int j = 0; j < gg; ++j) {
            double d0 = x0 - Y[4 * j], d1 = x1 - Y[4 * j + 1], d2 = x2 - Y[4 * j + 2];
            // the kernel value (eq. fundament1 / fundament2) from one refined reciprocal square root
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2, ir = rsqrt_pos(r2);
            const double f = 0.07957747154594767 * ir * Y[4 * j + 3];
            T k;
            if constexpr (NComp<T>::value == 2) {
                double sn, cs;
                sincos_tab(kappa * (r2 * ir), sctab, &sn, &cs);  // the 4 KB table stays in the L1 cache
                k = T{cs * f, sn * f};
            } else {
                k = f;
            }
            const double *ps = psi + j * NLOC;
#pragma unroll
            for (int b = 0; b < NLOC; ++b) acc[b] += k * ps[b];
        }
        double kw = X[4 * i + 3];
#pragma unroll
        for (int b = 0; b < NLOC; ++b) tmp[i * TS + b] = acc[b] * kw;
    }
    __syncthreads();
    T *out1, *out2;
    near_targets(sb, R, (int64_t)nl * ld, blocks, out1, out2);
    for (int o = threadIdx.x; o < NLOC * NLOC; o += blockDim.x) {
        int a = o / NLOC, b = o % NLOC;
        T s = zero<T>();
        for (int i = 0; i < gg; ++i) s += psi[i * NLOC + a] * tmp[i * TS + b];
        if (out1) out1[blk_pos(ld, NLOC, R.elE, a, R.elF, b)] = s;
        if (out2) out2[blk_pos(ld, NLOC, R.elF, b, R.elE, a)] = s;
    }
}

// Line-contraction tiles (see tile_fix): for every element, the tile with both
// parameters converted by cm (monomial basis, or identity), stored as itself
// (out[0]) and with the two parameters exchanged (out[1]).  One thread per entry.
__global__ void k_tline(int nelem, int G1, const double *__restrict__ cm, const double *__restrict__ tiles,
                        double *__restrict__ out)
{
    const int64_t ts = (int64_t)G1 * G1 * 4;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)nelem * ts) return;
    const int64_t E = x / ts;
    const int r = (int)(x % ts), c = r & 3, j = (r >> 2) / G1, i = (r >> 2) % G1;
    const double *H = tiles + E * ts;
    double acc = 0.0;
    for (int jj = 0; jj <= j; ++jj)
        for (int ii = 0; ii <= i; ++ii) acc += cm[j * G1 + jj] * cm[i * G1 + ii] * H[(jj * G1 + ii) * 4 + c];
    out[E * ts + (j * G1 + i) * 4 + c] = acc;
    out[((int64_t)nelem + E) * ts + (i * G1 + j) * 4 + c] = acc;
}

// 1/x for finite x != 0: the hardware estimate refined by two Newton steps.
__device__ inline double rcp_nz(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}

// Line contraction of an element tile (rational, bidegree (PG, PG), homogeneous
// (x w, y w, z w, w)).  M holds the tile with the parameter to be fixed
// fastest, M[(k*(PG+1) + l)*4 + c] (the tile itself to fix u, its transpose to
// fix v), in the monomial basis t^l of both parameters when PG <= 4 (Horner
// evaluation; the conversion from Bernstein form is exact up to rounding) and
// in Bernstein form otherwise.  Returns A[k] = sum_l b_l(f) M[k][l] and
// dA[k] = sum_l b_l'(f) M[k][l], k along the parameter that remains free.
template <int PG>
__device__ inline void tile_fix(const double *M, double f, double A[PG + 1][4], double dA[PG + 1][4])
{
    constexpr int G1 = PG + 1;
    if constexpr (PG <= 4) {
#pragma unroll
        for (int k = 0; k < G1; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double x = M[(k * G1 + PG) * 4 + c], d = 0.0;
#pragma unroll
                for (int l = PG - 1; l >= 0; --l) {
                    d = fma(d, f, x);
                    x = fma(x, f, M[(k * G1 + l) * 4 + c]);
                }
                A[k][c] = x;
                dA[k][c] = d;
            }
    } else {
        double B[G1], dB[G1];
        bernstein_d_t<PG>(f, B, dB);
#pragma unroll
        for (int k = 0; k < G1; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double x = 0.0, d = 0.0;
#pragma unroll
                for (int l = 0; l < G1; ++l) {
                    const double h = M[(k * G1 + l) * 4 + c];
                    x += B[l] * h;
                    d += dB[l] * h;
                }
                A[k][c] = x;
                dA[k][c] = d;
            }
    }
}

// Point and surface measure of the tile at value w of the remaining parameter,
// from its line contraction (the measure |X_u x X_v| does not depend on the
// order of the two tangents).  With homogeneous S, tangents D1, D2 and
// X = S_xyz / S_w, |X_u x X_v| = |(D1 - X D1_w) x (D2 - X D2_w)| / S_w^2.
template <int PG>
__device__ inline void tile_line_point(const double A[PG + 1][4], const double dA[PG + 1][4], double w, double X[3],
                                       double *kap)
{
    constexpr int G1 = PG + 1;
    double S[4], D1[4], D2[4];
    if constexpr (PG <= 4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double x = A[PG][c], d = 0.0, e = dA[PG][c];
#pragma unroll
            for (int k = PG - 1; k >= 0; --k) {
                d = fma(d, w, x);
                x = fma(x, w, A[k][c]);
                e = fma(e, w, dA[k][c]);
            }
            S[c] = x;
            D1[c] = d;
            D2[c] = e;
        }
    } else {
        double B[G1], dB[G1];
        bernstein_d_t<PG>(w, B, dB);
#pragma unroll
        for (int c = 0; c < 4; ++c) S[c] = D1[c] = D2[c] = 0.0;
#pragma unroll
        for (int k = 0; k < G1; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                S[c] += B[k] * A[k][c];
                D1[c] += dB[k] * A[k][c];
                D2[c] += B[k] * dA[k][c];
            }
    }
    const double iw = rcp_nz(S[3]);
    const double x0 = S[0] * iw, x1 = S[1] * iw, x2 = S[2] * iw;
    const double a0 = D1[0] - x0 * D1[3], a1 = D1[1] - x1 * D1[3], a2 = D1[2] - x2 * D1[3];
    const double b0 = D2[0] - x0 * D2[3], b1 = D2[1] - x1 * D2[3], b2 = D2[2] - x2 * D2[3];
    X[0] = x0;
    X[1] = x1;
    X[2] = x2;
    const double n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
    const double nn = n0 * n0 + n1 * n1 + n2 * n2;
    *kap = nn > 0.0 ? nn * rsqrt_pos(nn) * (iw * iw) : 0.0;
}

// One element's reference point along a quadrature line: (u, v) = (u0, v0) +
// w (du, dv), where only the coordinate that is not fixed moves (fix_u: u
// stays u0).  For a canonical frame (o, a, b) and local (s, t) = (s0, t0) +
// w (ds, dt) with only s or only t moving.
struct Line {
    double u0, v0, du, dv;
};

__device__ inline Line frame_line(int o, int a, int b, double s0, double ds, double t0, double dt)
{
    const double cx[4] = {0.0, 1.0, 1.0, 0.0}, cy[4] = {0.0, 0.0, 1.0, 1.0};
    const double xa = cx[a] - cx[o], ya = cy[a] - cy[o], xb = cx[b] - cx[o], yb = cy[b] - cy[o];
    return Line{cx[o] + s0 * xa + t0 * xb, cy[o] + s0 * ya + t0 * yb, ds * xa + dt * xb, ds * ya + dt * yb};
}

// Whether u stays fixed along the line when the moving local coordinate is s
// (move_s) or t of the frame (o, a, b).
__device__ inline bool frame_fix_u(int o, int a, int b, bool move_s)
{
    const double cx[4] = {0.0, 1.0, 1.0, 0.0};
    return (move_s ? cx[a] : cx[b]) == cx[o];
}

// Value of the neighbouring lane of the pair (lane ^ 1), by DPP quad_perm [1,0,3,2].
__device__ inline double from_pair_lane(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int plo = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
    const int phi = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false);
    return __hiloint2double(phi, plo);
}

// Touching pairs (identical / common edge / common vertex): regularising
// Duffy-type substitutions of [0,1]^4 (8 / 6 / 4 regions), Gauss of order gs
// per variable.  One workgroup per pair.  A line of the rule has its first
// three variables (xi and two more) fixed and the fourth running over its gs
// nodes; along a line each element's reference point moves in one parameter
// only (in the vertex case the point of E does not move at all).  Every pair
// of lanes (2k, 2k+1) owns one line, lane 2k element E and lane 2k+1 element
// F: the lane contracts its tile once over the fixed parameter and then
// evaluates the points of the line at the cost of a curve.
//
// With the fixed parameter of E at f_E and of F at f_F, the basis function
// (a1, a2) of E factors on the line into b(f_E) times b(moving), so the line's
// contribution to the block is the Kronecker product of the fixed-parameter
// factor p[aF][bF] = b_aF(f_E) b_bF(f_F) with the line factor
// C[aM][bM] = sum over the line's points of w K(x, y) b_aM(.) b_bM(.).  Each
// line is therefore one rank-1 term of the block reordered by (aF, bF) x
// (aM, bM): the lane pair forms C on the vector units (lane 2k rows 0 .. H-1,
// lane 2k+1 rows H .. P, with the partner's Bernstein values passed by DPP),
// stages p and C of its line in LDS (same row split), and a wave accumulates
// its 32 lines with FP64 MFMA (v_mfma_f64_16x16x4f64: 4 lines per step),
// complex kernels as two real accumulations.  The reordered block depends on
// which parameter of F is fixed (the vertex rule has both kinds of lines), so
// there is one accumulator per kind; waves are reduced through LDS at the end
// and the reordering is undone on output.
typedef double v4d __attribute__((ext_vector_type(4)));

// VTX: this launch integrates the common-vertex pairs of its list (the others
// the remaining classes); a workgroup whose pair belongs to the other launch
// returns at once.  The two rules are separate instantiations so that neither
// carries the other's registers.
template <class T, int P, int PG, int WAVES, bool VTX>
__global__ void __launch_bounds__(64 * WAVES, NComp<T>::value == 1 ? 2 : 1) k_near_singular(
    const PairRec *__restrict__ pairs, int gs, const double *__restrict__ gxs, const double *__restrict__ gws,
    const double *__restrict__ tfix_u, const double *__restrict__ tfix_v, double kappa, T *__restrict__ pairbuf,
    const double *__restrict__ sctab)
{
    constexpr int P1 = P + 1, NLOC = P1 * P1, NT = (NLOC + 15) / 16, NPAD = 16 * NT;
    constexpr int NC = NComp<T>::value;
    constexpr int G1 = PG + 1, TS = G1 * G1 * 4;
    constexpr int H = (P1 + 1) / 2;  // rows (lane 2k) / columns (lane 2k+1) of C per lane
    constexpr int HALF = 32;         // lines staged per step
    // staging rows of RS = NPAD + 1 doubles, V after U with an 8-double shift:
    // the 16 lanes of a pass read 16 different 8-byte bank pairs
    constexpr int RS = NPAD + 1;
    constexpr int STAGE = HALF * (NC + 1) * RS + 8;  // doubles per wave
    extern __shared__ double sh[];
    double *nx = sh, *nw = nx + 64;
    double *stg = nw + 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *Ub = stg + wave * STAGE;  // [HALF][RS]: p of each line
    double *Vb = Ub + HALF * RS + 8;  // [NC][HALF][RS]: C of each line
    const PairRec R = pairs[blockIdx.x];
    if ((R.cls == 3) != VTX) return;  // the other launch's pair (uniform: no barrier passed yet)
    const int role = lane & 1, pl = lane >> 1;  // role 0: element E, 1: element F; pl: line slot
    const int elem = role ? R.F : R.E;
    for (int k = threadIdx.x; k < gs; k += blockDim.x) {
        nx[k] = gxs[k];
        nw[k] = gws[k];
    }
    // complex kernel: the sine/cosine table (sincos_tab) next to the nodes, before the first barrier
    __shared__ __attribute__((aligned(16))) double tabs[NC == 2 ? 2 * kSinCosTab : 1];
    if constexpr (NC == 2)
        for (int k = threadIdx.x; k < 2 * kSinCosTab; k += blockDim.x) tabs[k] = sctab[k];
    if constexpr (NPAD > NLOC) {
        for (int k = lane; k < HALF * (NPAD - NLOC); k += 64) {
            int pt = k / (NPAD - NLOC), a = NLOC + k % (NPAD - NLOC);
            Ub[pt * RS + a] = 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) Vb[c * HALF * RS + pt * RS + a] = 0.0;
        }
    }
    __syncthreads();
    const int g = gs, g2 = g * g, g3 = g2 * g;
    // identical pairs: the region with both signs flipped is the x <-> y mirror of
    // the one with (sg1, sg2 = 0) (same weights, the two points exchanged), so with
    // a symmetric kernel its block is the transpose; only the four regions with
    // sg2 = 0 are integrated and the output is S + S^T (the symmetrised sum of all
    // eight)
    const int nreg = R.cls == 1 ? 4 : (R.cls == 2 ? 6 : 4);
    const int chunks = (g3 + HALF - 1) / HALF;
    // acc[h]: lines on which F's fixed parameter is u (h = 1) or v (h = 0)
    v4d acc[2][NC][NT][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int i = 0; i < NT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[h][c][i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int col = lane & 15, sub = lane >> 4;
    for (int unit = wave; unit < nreg * chunks; unit += WAVES) {
        const int ureg = unit / chunks, line = (unit - ureg * chunks) * HALF + pl;
        const int reg = R.cls == 1 ? (ureg & 1) | ((ureg >> 1) << 2) : ureg;
        // the pair's line: fixed nodes (ia, ib, ic), weight Wl of the fixed part;
        // inactive lines get two distinct fixed points and zero weight
        Line LE{0.25, 0.25, 0.0, 0.0}, LF{0.75, 0.75, 0.0, 0.0};
        double Wl = 0.0;
        bool fixE_u = true, fixF_u = true, constE = false;
        {
            const bool valid = line < g3;
            const int ln = valid ? line : 0;
            const int ia = ln / g2, ib = (ln / g) % g, ic = ln % g;
            const double va = nx[ia], vb = nx[ib], vc = nx[ic], w3 = nw[ia] * nw[ib] * nw[ic];
            if (R.cls == 1) {
                // identical: (x1 - y1, x2 - y2) = (+-z1, +-z2); x1, y1 fixed, x2, y2 move with the 4th node
                const int sg1 = reg & 1, sg2 = (reg >> 1) & 1, tri = reg >> 2;
                const double xi = va, eta = vb;
                const double z1 = tri == 0 ? xi : xi * eta, z2 = tri == 0 ? xi * eta : xi;
                const double lo1 = (1 - z1) * vc;
                const double xs = sg1 == 0 ? lo1 : lo1 + z1, ys = sg1 == 0 ? lo1 + z1 : lo1;
                if (valid) {
                    LE = Line{xs, sg2 == 0 ? 0.0 : z2, 0.0, 1 - z2};
                    LF = Line{ys, sg2 == 0 ? z2 : 0.0, 0.0, 1 - z2};
                    Wl = w3 * xi * (1 - z1) * (1 - z2);
                }
            } else if (R.cls == 2) {
                // common edge: local s moves with the 4th node, t is fixed
                const int sg = reg & 1, pyr = reg >> 1;
                const double xi = va, e1 = vb, e2 = vc;
                double zz, ct, dt;
                if (pyr == 0) { zz = xi; ct = xi * e1; dt = xi * e2; }
                else if (pyr == 1) { ct = xi; zz = xi * e1; dt = xi * e2; }
                else { dt = xi; zz = xi * e1; ct = xi * e2; }
                const double cs0 = sg == 0 ? 0.0 : zz, ds0 = sg == 0 ? zz : 0.0;
                fixE_u = frame_fix_u(R.oE, R.aE, R.bE, true);
                fixF_u = frame_fix_u(R.oF, R.aF, R.bF, true);
                if (valid) {
                    LE = frame_line(R.oE, R.aE, R.bE, cs0, 1 - zz, ct, 0.0);
                    LF = frame_line(R.oF, R.aF, R.bF, ds0, 1 - zz, dt, 0.0);
                    Wl = w3 * xi * xi * (1 - zz);
                }
            } else {
                // common vertex: E's point is fixed on the line, F's moves in s (region 3) or t
                const double xi = va;
                const double v0 = reg == 0 ? xi : xi * vb;
                const double v1 = reg == 1 ? xi : xi * (reg == 0 ? vb : vc);
                constE = true;
                fixF_u = frame_fix_u(R.oF, R.aF, R.bF, reg == 3);
                if (valid) {
                    LE = frame_line(R.oE, R.aE, R.bE, v0, 0.0, v1, 0.0);
                    if (reg == 3) LF = frame_line(R.oF, R.aF, R.bF, 0.0, xi, xi, 0.0);
                    else LF = frame_line(R.oF, R.aF, R.bF, reg == 2 ? xi : xi * vc, 0.0, 0.0, xi);
                    Wl = w3 * xi * xi * xi;
                }
            }
        }
        if constexpr (!VTX) {
            // this lane's element along the line
            const Line L = role ? LF : LE;
            const bool fix_u = role ? fixF_u : fixE_u;
            const bool cst = role == 0 && constE;
            const double f = fix_u ? L.u0 : L.v0;
            double A[G1][4], dA[G1][4];
            tile_fix<PG>((fix_u ? tfix_u : tfix_v) + (size_t)elem * TS, f, A, dA);
            // Bernstein values at the fixed (bf) and moving (bm) parameter; index P1
            // pads the last row of an odd P1 on lane 2k+1
            double bf[P1 + 1], bm[P1 + 1], X[3], kap = 0.0;
            bernstein_t<P>(f, bf);
            bf[P1] = bm[P1] = 0.0;
            if (cst) {  // vertex, element E: one point for the whole line
                const double wv = fix_u ? L.v0 : L.u0;
                tile_line_point<PG>(A, dA, wv, X, &kap);
                bernstein_t<P>(wv, bm);
            }
            // cl[i][j] = C[base + i][j]: rows base .. base+H-1 of the line factor
            const int base = role ? H : 0;
            double cl[H][P1][NC];
    #pragma unroll
            for (int i = 0; i < H; ++i)
    #pragma unroll
                for (int j = 0; j < P1; ++j)
    #pragma unroll
                    for (int c = 0; c < NC; ++c) cl[i][j][c] = 0.0;
            for (int id = 0; id < g; ++id) {
                const double w = nx[id];
                if (!cst) {
                    const double wv = fix_u ? L.v0 + L.dv * w : L.u0 + L.du * w;
                    tile_line_point<PG>(A, dA, wv, X, &kap);
                    bernstein_t<P>(wv, bm);
                }
                // the partner's point; the weighted kernel value comes out bitwise
                // the same on both lanes (x - y = -(y - x) exactly)
                const double Y0 = from_pair_lane(X[0]), Y1 = from_pair_lane(X[1]), Y2 = from_pair_lane(X[2]);
                const double ky = from_pair_lane(kap);
                const double d0 = X[0] - Y0, d1 = X[1] - Y1, d2 = X[2] - Y2;
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double ir = rsqrt_pos(r2);
                const double f0 = 0.07957747154594767 * ir * ((Wl * nw[id]) * (kap * ky));
                double wk[NC];
                if constexpr (NC == 2) {
                    double sn, cs;
                    sincos_tab(kappa * (r2 * ir), tabs, &sn, &cs);
                    wk[0] = cs * f0;
                    wk[1] = sn * f0;
                } else {
                    wk[0] = f0;
                }
                // E's values of this lane's rows and F's values of all columns
                double bo[P1 + 1], be[H], bF[P1];
    #pragma unroll
                for (int a = 0; a < P1; ++a) bo[a] = from_pair_lane(bm[a]);
                bo[P1] = 0.0;
    #pragma unroll
                for (int i = 0; i < H; ++i) be[i] = role ? bo[H + i] : bm[i];
    #pragma unroll
                for (int j = 0; j < P1; ++j) bF[j] = role ? bm[j] : bo[j];
    #pragma unroll
                for (int i = 0; i < H; ++i)
    #pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const double t = wk[c] * be[i];
    #pragma unroll
                        for (int j = 0; j < P1; ++j) cl[i][j][c] = fma(t, bF[j], cl[i][j][c]);
                    }
            }
            // stage p and C of this line (row pl), rows base .. base+H-1 of both, in
            // (fixed | moving) index order aX * P1 + bX
            {
                double bfo[P1 + 1];
    #pragma unroll
                for (int a = 0; a < P1; ++a) bfo[a] = from_pair_lane(bf[a]);
                bfo[P1] = 0.0;
                double *urow = Ub + pl * RS + base * P1;
    #pragma unroll
                for (int i = 0; i < H; ++i) {
                    if (P1 % 2 == 1 && i == H - 1 && role) continue;  // row P1 does not exist
                    const double fe = role ? bfo[H + i] : bf[i];
    #pragma unroll
                    for (int j = 0; j < P1; ++j) {
                        const double ff = role ? bf[j] : bfo[j];
                        urow[i * P1 + j] = fe * ff;
    #pragma unroll
                        for (int c = 0; c < NC; ++c) urow[(Vb - Ub) + c * HALF * RS + i * P1 + j] = cl[i][j][c];
                    }
                }
            }
        } else {
            // common vertex: E's point is the same on the whole line, so both lanes of
            // the pair evaluate F's points, lane 2k the even and lane 2k+1 the odd
            // nodes; E's Bernstein factors are constant along the line, so the line
            // factor has rank one, C = b(v_E) (x) sum over the nodes of w K b(moving of F)
            const int base = role ? H : 0;
            double bfE[P1 + 1], bmE[P1 + 1], bfF[P1], XE[3], kapE = 0.0;
            {
                double A[G1][4], dA[G1][4];
                tile_fix<PG>(tfix_u + (size_t)R.E * TS, LE.u0, A, dA);  // E fixes u on vertex lines
                tile_line_point<PG>(A, dA, LE.v0, XE, &kapE);
            }
            bernstein_t<P>(LE.u0, bfE);
            bernstein_t<P>(LE.v0, bmE);
            bfE[P1] = bmE[P1] = 0.0;
            const double fF = fixF_u ? LF.u0 : LF.v0;
            double A[G1][4], dA[G1][4];
            tile_fix<PG>((fixF_u ? tfix_u : tfix_v) + (size_t)R.F * TS, fF, A, dA);
            bernstein_t<P>(fF, bfF);
            double sF[P1][NC];
#pragma unroll
            for (int j = 0; j < P1; ++j)
#pragma unroll
                for (int c = 0; c < NC; ++c) sF[j][c] = 0.0;
            for (int id = role; id < g; id += 2) {
                const double w = nx[id];
                const double wv = fixF_u ? LF.v0 + LF.dv * w : LF.u0 + LF.du * w;
                double XF[3], kapF = 0.0, bmF[P1];
                tile_line_point<PG>(A, dA, wv, XF, &kapF);
                bernstein_t<P>(wv, bmF);
                const double d0 = XE[0] - XF[0], d1 = XE[1] - XF[1], d2 = XE[2] - XF[2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double ir = rsqrt_pos(r2);
                const double f0 = 0.07957747154594767 * ir * ((Wl * nw[id]) * (kapE * kapF));
                double wk[NC];
                if constexpr (NC == 2) {
                    double sn, cs;
                    sincos_tab(kappa * (r2 * ir), tabs, &sn, &cs);
                    wk[0] = cs * f0;
                    wk[1] = sn * f0;
                } else {
                    wk[0] = f0;
                }
#pragma unroll
                for (int j = 0; j < P1; ++j)
#pragma unroll
                    for (int c = 0; c < NC; ++c) sF[j][c] = fma(wk[c], bmF[j], sF[j][c]);
            }
            // both lanes: own half plus the partner's (the same sum on both)
#pragma unroll
            for (int j = 0; j < P1; ++j)
#pragma unroll
                for (int c = 0; c < NC; ++c) sF[j][c] += from_pair_lane(sF[j][c]);
            double *urow = Ub + pl * RS + base * P1;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                if (P1 % 2 == 1 && i == H - 1 && role) continue;  // row P1 does not exist
                const double fe = role ? bfE[H + i] : bfE[i], me = role ? bmE[H + i] : bmE[i];
#pragma unroll
                for (int j = 0; j < P1; ++j) {
                    urow[i * P1 + j] = fe * bfF[j];
#pragma unroll
                    for (int c = 0; c < NC; ++c) urow[(Vb - Ub) + c * HALF * RS + i * P1 + j] = me * sF[j][c];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        auto accumulate = [&](v4d (&a)[NC][NT][NT]) {
#pragma unroll
            for (int j = 0; j < HALF / 4; ++j) {
                const int pt = 4 * j + sub;
                double av[NT];
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) av[ta] = Ub[pt * RS + 16 * ta + col];
#pragma unroll
                for (int c2 = 0; c2 < NC; ++c2)
#pragma unroll
                    for (int tb = 0; tb < NT; ++tb) {
                        const double bv = Vb[c2 * HALF * RS + pt * RS + 16 * tb + col];
#pragma unroll
                        for (int ta = 0; ta < NT; ++ta)
                            a[c2][ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ta], bv, a[c2][ta][tb], 0, 0, 0);
                    }
            }
        };
        if (fixF_u) accumulate(acc[1]);
        else accumulate(acc[0]);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // E's fixed parameter is the same on every line of the pair; F's takes one
    // value (identical, edge) or both (vertex)
    const bool fixE = R.cls == 2 ? frame_fix_u(R.oE, R.aE, R.bE, true) : true;
    const int hF = R.cls == 1 ? 1 : (frame_fix_u(R.oF, R.aF, R.bF, true) ? 1 : 0);
    T *out = pairbuf + (int64_t)blockIdx.x * NLOC * NLOC;
    double *red = stg;  // red[((w*NC + c)*NPAD + row)*NPAD + col], reordered block of wave w
    bool first = true;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (R.cls != 3 && h != hF) continue;
        __syncthreads();
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2)
#pragma unroll
            for (int ta = 0; ta < NT; ++ta)
#pragma unroll
                for (int tb = 0; tb < NT; ++tb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        // v_mfma_f64_16x16x4f64 result layout: lane l, element e holds D[4e + l/16][l%16]
                        int row = 16 * ta + 4 * e + sub, cc = 16 * tb + col;
                        red[((size_t)(wave * NC + c2) * NPAD + row) * NPAD + cc] = acc[h][c2][ta][tb][e];
                    }
        __syncthreads();
        for (int o = threadIdx.x; o < NLOC * NLOC; o += blockDim.x) {
            // entry (a, b) with a = a2 P1 + a1 (a1: u index of E), b likewise for F
            const int a = o / NLOC, b = o % NLOC;
            const int a1 = a % P1, a2 = a / P1, b1 = b % P1, b2 = b / P1;
            const int aF = fixE ? a1 : a2, aM = fixE ? a2 : a1;
            const int bF = h ? b1 : b2, bM = h ? b2 : b1;
            const size_t rc = (size_t)(aF * P1 + bF) * NPAD + aM * P1 + bM;
            // the mirrored entry (b, a) of an identical pair (both fix u)
            const size_t rt = (size_t)(b1 * P1 + a1) * NPAD + b2 * P1 + a2;
            double sre = 0.0, sim = 0.0, tre = 0.0, tim = 0.0;
            for (int w = 0; w < WAVES; ++w) {
                const double *rw = red + (size_t)(w * NC) * NPAD * NPAD;
                sre += rw[rc];
                if (R.cls == 1) tre += rw[rt];
                if constexpr (NC == 2) {
                    sim += rw[NPAD * NPAD + rc];
                    if (R.cls == 1) tim += rw[NPAD * NPAD + rt];
                }
            }
            if (R.cls == 1) {  // S + S^T over the four integrated regions
                sre = sre + tre;
                sim = sim + tim;
            }
            T s;
            if constexpr (NC == 2) s = T{sre, sim};
            else s = sre;
            if (!first) s += out[o];
            out[o] = s;
        }
        first = false;
    }
}

// Places staged touching-pair blocks (row-major nloc x nloc per pair, in the
// order of `pairs`) into the near-field leaf blocks and their mirrors.
template <class T>
__global__ void k_scatter_pairs(const PairRec *__restrict__ pairs, int nloc, int nl, int ld,
                                const int32_t *__restrict__ sb, const T *__restrict__ pairbuf, T *__restrict__ blocks)
{
    const PairRec R = pairs[blockIdx.x];
    const T *in = pairbuf + (int64_t)blockIdx.x * nloc * nloc;
    T *out1, *out2;
    near_targets(sb, R, (int64_t)nl * ld, blocks, out1, out2);
    for (int o = threadIdx.x; o < nloc * nloc; o += blockDim.x) {
        int a = o / nloc, b = o % nloc;
        T v = in[o];
        if (out1) out1[blk_pos(ld, nloc, R.elE, a, R.elF, b)] = v;
        if (out2) out2[blk_pos(ld, nloc, R.elF, b, R.elE, a)] = v;
    }
}

// ===========================================================================
// kernels: far field
// ===========================================================================

// Coupling block of every admissible pair: the localised kernel at the
// Chebyshev node pairs (Sec. 4.2), stored column-major (col = source node).
template <class T>
__global__ void __launch_bounds__(256) k_coupling(int64_t nfar, const int32_t *__restrict__ far_tgt,
                                                  const int32_t *__restrict__ far_src, int q2,
                                                  const double *__restrict__ nodes, double kappa, T *__restrict__ coup)
{
    int64_t k = blockIdx.x;
    int tg = far_tgt[k], sc = far_src[k];
    const double *xt = nodes + (size_t)tg * q2 * 4, *xsrc = nodes + (size_t)sc * q2 * 4;
    T *out = coup + k * q2 * q2;
    for (int idx = threadIdx.x; idx < q2 * q2; idx += blockDim.x) {
        int nu = idx / q2, mu = idx % q2;
        double d0 = xt[4 * mu] - xsrc[4 * nu], d1 = xt[4 * mu + 1] - xsrc[4 * nu + 1], d2 = xt[4 * mu + 2] - xsrc[4 * nu + 2];
        double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        out[idx] = green<T>(r, kappa) * (xt[4 * mu + 3] * xsrc[4 * nu + 3]);
    }
}

// Two-level slices of the cluster tree in one workgroup (Sec. 4.2 nested
// bases).  A workgroup owns one cluster of level ls and the clusters below it
// down to level lb <= ls + 2.  k_up_tree: leaf moments (when lb is the leaf
// level) and the upward transfers from lb to ls; k_down_tree: the downward
// transfers from ls to lb and the leaf back-moments (when lb is the leaf
// level).  Leaf moments X^ = M1^T X M1 (X the leaf's coefficients as an
// n1 x n1 array) and back-moments y* += M1 Y^ M1^T are two 1D contractions
// each; a transfer is one (parent, child) item per wave, the four child
// contributions of a parent summed in child order through LDS.  Waves use
// LDS slices of SL elements of T, levels are separated by workgroup barriers.
struct TreeArgs {
    int ls, lb, L, q, n1, side, P1, nloc, nl;
    const double *M1, *E2;
    const int64_t *cl_off;
};

// global index of cluster (a2, a1) of level lv inside the slice of root
// (patch, r2, r1) at level ls
__device__ inline int64_t tree_cluster(const TreeArgs &A, int patch, int r2, int r1, int lv, int a2, int a1)
{
    const int w = 1 << (lv - A.ls), n = 1 << lv;
    return A.cl_off[lv] + (int64_t)patch * n * n + (int64_t)(r2 * w + a2) * n + r1 * w + a1;
}

// The leaf moment matrix M1 (n1 x q) and the two child transfers E2 (q x q
// each) copied to LDS by the whole workgroup (the inner products read them
// once per term).
__device__ inline void tree_stage_ops(const TreeArgs &A, double *M1, double *E2)
{
    const int nm = A.n1 * A.q, ne = 2 * A.q * A.q;
    for (int k = threadIdx.x; k < nm + ne; k += blockDim.x) {
        if (k < nm) M1[k] = A.M1[k];
        else E2[k - nm] = A.E2[k - nm];
    }
    __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(1024) k_up_tree(TreeArgs A, int SL, const T *__restrict__ xs, T *__restrict__ Xh)
{
    extern __shared__ double sh[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const int q = A.q, q2 = q * q, n1 = A.n1;
    T *W0 = (T *)sh + (size_t)wave * SL;
    T *slot = (T *)sh + (size_t)nwv * SL;  // [4 P][q2] child contributions
    double *M1 = (double *)(slot + (size_t)16 * q2), *E2 = M1 + n1 * q;  // staged operators
    tree_stage_ops(A, M1, E2);
    const int nr = 1 << A.ls, root = blockIdx.x;
    const int patch = root / (nr * nr), r2 = (root % (nr * nr)) / nr, r1 = root % nr;
    if (A.lb == A.L) {
        const int w = 1 << (A.L - A.ls);
        const int64_t leaf0 = A.cl_off[A.L];
        T *X = W0, *Z = W0 + n1 * n1;
        for (int i = wave; i < w * w; i += nwv) {
            const int64_t g = tree_cluster(A, patch, r2, r1, A.L, i / w, i % w), leaf = g - leaf0;
            for (int f = lane; f < A.nl; f += 64) {
                int el = f / A.nloc, r = f % A.nloc;
                int i1 = (el % A.side) * A.P1 + r % A.P1, i2 = (el / A.side) * A.P1 + r / A.P1;
                X[i2 * n1 + i1] = xs[leaf * A.nl + f];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int o = lane; o < n1 * q; o += 64) {
                int i2 = o / q, mu1 = o % q;
                T s = zero<T>();
                for (int i1 = 0; i1 < n1; ++i1) s += M1[i1 * q + mu1] * X[i2 * n1 + i1];
                Z[o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int o = lane; o < q2; o += 64) {
                int mu2 = o / q, mu1 = o % q;
                T s = zero<T>();
                for (int i2 = 0; i2 < n1; ++i2) s += M1[i2 * q + mu2] * Z[i2 * q + mu1];
                Xh[g * q2 + o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
    }
    // X^_P = 1/4 sum_c (E_c1 (x) E_c2)^T X^_c, children c = (c2, c1) in order
    for (int lv = A.lb - 1; lv >= A.ls; --lv) {
        __syncthreads();
        const int w = 1 << (lv - A.ls), np = w * w;
        T *Xc = W0, *Z = W0 + q2;
        for (int it = wave; it < 4 * np; it += nwv) {
            const int i = it >> 2, c1 = it & 1, c2 = (it >> 1) & 1, a2 = i / w, a1 = i % w;
            const int64_t gc = tree_cluster(A, patch, r2, r1, lv + 1, 2 * a2 + c2, 2 * a1 + c1);
            for (int o = lane; o < q2; o += 64) Xc[o] = Xh[gc * q2 + o];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const double *Ec1 = E2 + c1 * q2, *Ec2 = E2 + c2 * q2;
            for (int o = lane; o < q2; o += 64) {
                int nu2 = o / q, mu1 = o % q;
                T s = zero<T>();
                for (int nu1 = 0; nu1 < q; ++nu1) s += Ec1[nu1 * q + mu1] * Xc[nu2 * q + nu1];
                Z[o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int o = lane; o < q2; o += 64) {
                int mu2 = o / q, mu1 = o % q;
                T s = zero<T>();
                for (int nu2 = 0; nu2 < q; ++nu2) s += Ec2[nu2 * q + mu2] * Z[nu2 * q + mu1];
                slot[(size_t)it * q2 + o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
        __syncthreads();
        for (int o = threadIdx.x; o < np * q2; o += blockDim.x) {
            const int i = o / q2, k = o % q2;
            const T *sc = slot + (size_t)4 * i * q2 + k;
            T v = zero<T>();
            v += sc[0];
            v += sc[q2];
            v += sc[2 * q2];
            v += sc[3 * q2];
            Xh[tree_cluster(A, patch, r2, r1, lv, i / w, i % w) * q2 + k] = 0.25 * v;
        }
    }
}

template <class T>
__global__ void __launch_bounds__(1024) k_down_tree(TreeArgs A, int SL, T *__restrict__ Yh, T *__restrict__ ys)
{
    extern __shared__ double sh[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    const int q = A.q, q2 = q * q, n1 = A.n1;
    T *W0 = (T *)sh + (size_t)wave * SL;
    double *M1 = (double *)((T *)sh + (size_t)nwv * SL + (size_t)16 * q2), *E2 = M1 + n1 * q;  // staged operators
    tree_stage_ops(A, M1, E2);
    const int nr = 1 << A.ls, root = blockIdx.x;
    const int patch = root / (nr * nr), r2 = (root % (nr * nr)) / nr, r1 = root % nr;
    // Y^_c += 1/4 (E_c1 (x) E_c2) Y^_P
    for (int lv = A.ls + 1; lv <= A.lb; ++lv) {
        const int w = 1 << (lv - A.ls);
        T *Yp = W0, *Z = W0 + q2;
        for (int i = wave; i < w * w; i += nwv) {
            const int a2 = i / w, a1 = i % w, c1 = a1 & 1, c2 = a2 & 1;
            const int64_t gc = tree_cluster(A, patch, r2, r1, lv, a2, a1);
            const int64_t gp = tree_cluster(A, patch, r2, r1, lv - 1, a2 >> 1, a1 >> 1);
            for (int o = lane; o < q2; o += 64) Yp[o] = Yh[gp * q2 + o];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const double *Ec1 = E2 + c1 * q2, *Ec2 = E2 + c2 * q2;
            for (int o = lane; o < q2; o += 64) {
                int mu2 = o / q, nu1 = o % q;
                T s = zero<T>();
                for (int mu1 = 0; mu1 < q; ++mu1) s += Ec1[nu1 * q + mu1] * Yp[mu2 * q + mu1];
                Z[o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int o = lane; o < q2; o += 64) {
                int nu2 = o / q, nu1 = o % q;
                T s = zero<T>();
                for (int mu2 = 0; mu2 < q; ++mu2) s += Ec2[nu2 * q + mu2] * Z[mu2 * q + nu1];
                Yh[gc * q2 + o] += 0.25 * s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
        __syncthreads();
    }
    if (A.lb == A.L) {
        const int w = 1 << (A.L - A.ls);
        const int64_t leaf0 = A.cl_off[A.L];
        T *Y = W0, *Z = W0 + q2;
        for (int i = wave; i < w * w; i += nwv) {
            const int64_t g = tree_cluster(A, patch, r2, r1, A.L, i / w, i % w), leaf = g - leaf0;
            for (int o = lane; o < q2; o += 64) Y[o] = Yh[g * q2 + o];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int o = lane; o < q * n1; o += 64) {
                int mu2 = o / n1, i1 = o % n1;
                T s = zero<T>();
                for (int mu1 = 0; mu1 < q; ++mu1) s += M1[i1 * q + mu1] * Y[mu2 * q + mu1];
                Z[o] = s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            for (int f = lane; f < A.nl; f += 64) {
                int el = f / A.nloc, r = f % A.nloc;
                int i1 = (el % A.side) * A.P1 + r % A.P1, i2 = (el / A.side) * A.P1 + r / A.P1;
                T s = zero<T>();
                for (int mu2 = 0; mu2 < q; ++mu2) s += M1[i2 * q + mu2] * Z[mu2 * n1 + i1];
                ys[leaf * A.nl + f] += s;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
    }
}

// Block-sparse matrix-vector product y_t = sum_k B_k x_src(k) over a CSR of
// column-major nb x nb blocks (near field: leaf blocks; far field: coupling
// blocks over all levels).  One workgroup per target row, waves split the
// row's blocks, lanes own block rows; the block stream is read once,
// coalesced.  ROLE only names the instantiation (0 near field, 1 coupling)
// so that profiles tell the two launches apart.
template <class T, int ROLE>
__global__ void __launch_bounds__(256) k_bsr_gemv(int nb, const int64_t *__restrict__ ptr, const int32_t *__restrict__ src,
                                                  const T *__restrict__ blocks, const T *__restrict__ x, T *__restrict__ y,
                                                  int64_t row0)
{
    extern __shared__ double sh[];
    T *part = (T *)sh;  // nw * nb
    int64_t t = row0 + blockIdx.x;
    int64_t k0 = ptr[t], k1 = ptr[t + 1];
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int nw = blockDim.x >> 6;
    for (int a0 = 0; a0 < nb; a0 += 64) {
        int a = a0 + lane;
        T acc = zero<T>();
        if (a < nb) {
            for (int64_t k = k0 + wave; k < k1; k += nw) {
                const T *B = blocks + k * (int64_t)nb * nb + a;
                const T *xs = x + (int64_t)src[k] * nb;
                int b = 0;
                for (; b + 4 <= nb; b += 4) {
                    T v0 = B[(int64_t)b * nb], v1 = B[(int64_t)(b + 1) * nb], v2 = B[(int64_t)(b + 2) * nb],
                      v3 = B[(int64_t)(b + 3) * nb];
                    acc += v0 * xs[b];
                    acc += v1 * xs[b + 1];
                    acc += v2 * xs[b + 2];
                    acc += v3 * xs[b + 3];
                }
                for (; b < nb; ++b) acc += B[(int64_t)b * nb] * xs[b];
            }
            part[wave * nb + a] = acc;
        }
    }
    __syncthreads();
    for (int a = threadIdx.x; a < nb; a += blockDim.x) {
        T s = part[a];
        for (int w = 1; w < nw; ++w) s += part[w * nb + a];
        y[t * nb + a] = s;
    }
}

// Near-field product with symmetric block storage (Sec. 4 item 4 blocks, one
// stored block per mirrored pair): one wave per stored block k = (t, s),
// t <= s, column-major with column stride ld (a multiple of 8, padding rows
// zero).  The lanes form an 8 x 8 grid; lane (li, lj) reads 8 consecutive
// rows (64 contiguous bytes) of the columns lj, lj + 8, ... of each 64-row
// tile and accumulates both B x_s (rows) and B^T x_t (columns).  Writes the
// partial rows part[2k] = B x_s (for leaf t) and, when t != s,
// part[2k+1] = B^T x_t (for leaf s); k_gather sums them per leaf.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Complex near-field blocks rounded to single precision, (re, im) float pairs: the
// near field of the inner operator of the single-precision Helmholtz solve.
struct cf {
    float re, im;
};

// 8 consecutive single-precision complex entries (64 bytes), widened to double
__device__ inline void load8(const cf *p, cd v[8])
{
    const v4f *q = (const v4f *)p;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const v4f w = q[r];
        v[2 * r] = cd{(double)w.x, (double)w.y};
        v[2 * r + 1] = cd{(double)w.z, (double)w.w};
    }
}

template <class T>
__device__ inline void load8(const T *p, T v[8])
{
    const v2d *q = (const v2d *)p;
    if constexpr (NComp<T>::value == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v2d w = q[r];
            v[2 * r] = w.x;
            v[2 * r + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            v2d w = q[r];
            v[r] = T{w.x, w.y};
        }
    }
}

// Sum over the 8 adjacent lanes of a lane group (lanes 8g .. 8g+7), every lane
// receiving the total: quad_perm exchanges within quads (lane ^ 1, lane ^ 2),
// then row_half_mirror (lane 7 - i within the group) joins the two quads.
template <int CTRL>
__device__ inline float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <class R>
__device__ inline R group8_sum(R v)
{
    v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    return v;
}

__device__ inline cd group8_sum(cd v) { return cd{group8_sum(v.re), group8_sum(v.im)}; }
__device__ inline double shfl_xor_(double v, int o) { return __shfl_xor(v, o); }
__device__ inline cd shfl_xor_(cd v, int o) { return cd{__shfl_xor(v.re, o), __shfl_xor(v.im, o)}; }

struct NearSymArgs {
    int64_t nsb;
    const int32_t *sb_t, *sb_s;
    int nl, ld;
};

// One stored near block k, executed by one whole wave; cacc is the wave's LDS
// slice of 8 ld + 520 elements.
template <class T>
__device__ inline void near_sym_wave(const NearSymArgs &N, int64_t k, const T *__restrict__ blocks,
                                     const T *__restrict__ x, T *__restrict__ part, T *cacc)
{
    const int nl = N.nl, ld = N.ld;
    const int lane = threadIdx.x & 63;
    const int li = lane >> 3, lj = lane & 7;
    const int64_t t = N.sb_t[k], sc = N.sb_s[k];
    T *rbuf = cacc + 8 * ld;  // [lj][row of the tile], row stride 65; cacc: [li][column]
    const T *B = blocks + k * (int64_t)nl * ld;
    const T *xt = x + t * nl, *xsrc = x + sc * nl;
    T *prow = part + (size_t)(2 * k) * ld;
    for (int rt = 0; rt < nl; rt += 64) {
        const int r0 = rt + 8 * li;
        T xr[8], ra[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            xr[r] = r0 + r < nl ? xt[r0 + r] : zero<T>();
            ra[r] = zero<T>();
        }
        for (int c = lj; c < nl; c += 8) {
            T cs = zero<T>();
            if (r0 < ld) {
                T v[8];
                load8(B + (int64_t)c * ld + r0, v);
                const T xc = xsrc[c];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    ra[r] += v[r] * xc;
                    cs += v[r] * xr[r];
                }
            }
            cacc[li * ld + c] = rt == 0 ? cs : cacc[li * ld + c] + cs;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) rbuf[lj * 65 + 8 * li + r] = ra[r];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (rt + lane < nl) {
            T v = rbuf[lane];
#pragma unroll
            for (int q = 1; q < 8; ++q) v += rbuf[q * 65 + lane];
            prow[rt + lane] = v;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    if (t != sc) {
        T *pcol = part + (size_t)(2 * k + 1) * ld;
        for (int c = lane; c < nl; c += 64) {
            T v = cacc[c];
#pragma unroll
            for (int q = 1; q < 8; ++q) v += cacc[q * ld + c];
            pcol[c] = v;
        }
    }
}

// one block entry, widened to the type of the sums
__device__ inline cd load1(const cd *p)
{
    const v2d w = *(const v2d *)p;
    return cd{w.x, w.y};
}
__device__ inline cd load1(const cf *p)
{
    const cf w = *p;
    return cd{(double)w.re, (double)w.im};
}
__device__ inline double load1(const double *p) { return *p; }

// One stored near block k by one whole wave, without LDS (nl <= 64 S): lane
// l = 8 lj + li owns rows rt + RPL li .. rt + RPL li + RPL - 1 of every 8 RPL-row
// tile and the columns c = lj + 8 kc.  A lane's RPL rows are consecutive in the
// column-major block, so the 8 lanes of a group read 8 RPL consecutive rows of one
// column.  Row sums (B x_s) are reduced over the 8 lanes lj at the end of a tile
// (shuffles); column sums (B^T x_t, the mirrored block's product) over the 8
// adjacent lanes li after every column step (DPP) and kept by the lane
// li == kc % 8 in slot kc / 8.  Writes the same partial rows as near_sym_wave.
// RPL = 8 (whole 64-row tiles) fits blocks of 64 and 256 functions; 144 (p = 2,
// 16 elements per leaf) takes RPL = 9, two full tiles instead of 64 + 64 + 16
// rows, and 36 takes RPL = 5.  U columns go per step, their loads issued
// together (the single-precision copy of the 144 blocks: RPL = 6, U = 2).
template <class T, int S, class BT = T, int RPL = 8, int U = 1>
__device__ inline void near_sym_wave_reg(const NearSymArgs &N, int64_t k, const BT *__restrict__ blocks,
                                         const T *__restrict__ x, T *__restrict__ part)
{
    const int nl = N.nl, ld = N.ld;
    const int lane = threadIdx.x & 63;
    const int li = lane & 7, lj = lane >> 3;
    const int64_t t = N.sb_t[k], sc = N.sb_s[k];
    const BT *B = blocks + k * (int64_t)nl * ld;
    const T *xt = x + t * nl, *xsrc = x + sc * nl;
    T *prow = part + (size_t)(2 * k) * ld;
    T own[S];
#pragma unroll
    for (int q = 0; q < S; ++q) own[q] = zero<T>();
    const int ncs = lj < nl ? (nl - lj + 7) / 8 : 0;  // columns lj + 8 kc < nl (the same for a whole group)
    for (int rt = 0; rt < nl; rt += 8 * RPL) {
        const int r0 = rt + RPL * li;
        const bool rows = r0 < nl;
        T xr[RPL], ra[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            xr[r] = r0 + r < nl ? xt[r0 + r] : zero<T>();
            ra[r] = zero<T>();
        }
        for (int kc = 0; kc < ncs; kc += U) {
            // U columns per step: all their loads are issued before the products
            T v[U][RPL], xc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lj + 8 * (kc + u);
                if (rows && kc + u < ncs) {
                    if constexpr (RPL == 8) {
                        load8(B + (int64_t)c * ld + r0, v[u]);
                    } else {
                        // rows past nl of the last tile read padding inside the column (ld >= 8 RPL tiles is
                        // not guaranteed, so those loads are skipped)
#pragma unroll
                        for (int r = 0; r < RPL; ++r)
                            v[u][r] = r0 + r < nl ? load1(B + (int64_t)c * ld + r0 + r) : zero<T>();
                    }
                    xc[u] = xsrc[c];
                } else {
#pragma unroll
                    for (int r = 0; r < RPL; ++r) v[u][r] = zero<T>();
                    xc[u] = zero<T>();
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T cs = zero<T>();
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    ra[r] += v[u][r] * xc[u];
                    cs += v[u][r] * xr[r];
                }
                cs = group8_sum(cs);
#pragma unroll
                for (int q = 0; q < S; ++q)
                    if (li == ((kc + u) & 7) && ((kc + u) >> 3) == q) own[q] += cs;
            }
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            T a = ra[r];
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) a += shfl_xor_(a, o);
            if (lj == (r & 7) && r0 + r < nl) prow[r0 + r] = a;
        }
    }
    if (t != sc) {
        T *pcol = part + (size_t)(2 * k + 1) * ld;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int kc = 8 * q + li;
            if (kc < ncs) pcol[lj + 8 * kc] = own[q];
        }
    }
}

// A stored near block by one wave: without LDS when nl <= 256, else with the
// wave's LDS slice cacc (8 ld + 520 elements).
template <class T>
__device__ inline void near_sym_block(const NearSymArgs &N, int64_t k, const T *__restrict__ blocks,
                                      const T *__restrict__ x, T *__restrict__ part, T *cacc)
{
    if (N.nl == 36) near_sym_wave_reg<T, 1, T, 5>(N, k, blocks, x, part);
    else if (N.nl <= 64) near_sym_wave_reg<T, 1>(N, k, blocks, x, part);
    else if (N.nl <= 128) near_sym_wave_reg<T, 2>(N, k, blocks, x, part);
    else if (N.nl == 144) near_sym_wave_reg<T, 3, T, 9>(N, k, blocks, x, part);
    else if (N.nl <= 192) near_sym_wave_reg<T, 3>(N, k, blocks, x, part);
    else if (N.nl <= 256) near_sym_wave_reg<T, 4>(N, k, blocks, x, part);
    else near_sym_wave<T>(N, k, blocks, x, part, cacc);
}

// LDS elements per wave of near_sym_block
__host__ __device__ inline int near_sym_lds(int nl, int ld) { return nl <= 256 ? 0 : 8 * ld + 520; }

template <class T>
__global__ void __launch_bounds__(256) k_near_sym(NearSymArgs N, const T *__restrict__ blocks, const T *__restrict__ x,
                                                  T *__restrict__ part)
{
    extern __shared__ double sh[];
    const int wave = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (k >= N.nsb) return;  // whole waves only; no block-wide barrier follows
    near_sym_block<T>(N, k, blocks, x, part, (T *)sh + (size_t)wave * near_sym_lds(N.nl, N.ld));
}

// A stored near block with single-precision complex entries (nl <= 256, products and sums in FP64)
__device__ inline void near_sym_block_c32(const NearSymArgs &N, int64_t k, const cf *__restrict__ blocks,
                                          const cd *__restrict__ x, cd *__restrict__ part)
{
    if (N.nl == 36) near_sym_wave_reg<cd, 1, cf, 5>(N, k, blocks, x, part);
    else if (N.nl <= 64) near_sym_wave_reg<cd, 1, cf>(N, k, blocks, x, part);
    else if (N.nl <= 128) near_sym_wave_reg<cd, 2, cf>(N, k, blocks, x, part);
    else if (N.nl == 144) near_sym_wave_reg<cd, 3, cf, 6, 2>(N, k, blocks, x, part);  // two columns in flight
    else if (N.nl <= 192) near_sym_wave_reg<cd, 3, cf>(N, k, blocks, x, part);
    else near_sym_wave_reg<cd, 4, cf>(N, k, blocks, x, part);
}

__global__ void __launch_bounds__(256) k_near_sym32(NearSymArgs N, const cf *__restrict__ blocks,
                                                    const cd *__restrict__ x, cd *__restrict__ part)
{
    const int wave = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (k >= N.nsb) return;
    near_sym_block_c32(N, k, blocks, x, part);
}

// blocks rounded to single precision, n complex values
__global__ void k_round_c32(int64_t n, const cd *__restrict__ in, cf *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = cf{(float)in[i].re, (float)in[i].im};
}


// Sum of partial rows: out[t*n + a] (t = row0 + r, r < rows) = sum over the CSR
// entries e of row t, in order, of part[pidx[e]*ld + a], times
// scale * w[(t*n + a)*4] when w is given (node weights of the far field).
struct GatherArgs {
    int n, ld;
    const int64_t *ptr;
    const int32_t *pidx;
    const void *part;
    const double *w;
    double scale;
    void *out;
    int64_t row0;
};

// Workgroups [0, nb_a) gather the rows of A, the rest those of B (one launch for
// the far-field and the near-field partial rows).  Four waves per row take every
// fourth entry; the four partial sums are added in wave order.
template <class T>
__global__ void __launch_bounds__(256) k_gather(GatherArgs A, GatherArgs B, int64_t nb_a)
{
    extern __shared__ double sh[];
    T *red = (T *)sh;  // [4][n]
    const bool first = (int64_t)blockIdx.x < nb_a;
    const GatherArgs &G = first ? A : B;
    const int n = G.n, ld = G.ld;
    const T *part = (const T *)G.part;
    T *out = (T *)G.out;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t t = G.row0 + (first ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - nb_a);
    const int64_t k0 = G.ptr[t], k1 = G.ptr[t + 1];
    for (int a = lane; a < n; a += 64) {
        T acc = zero<T>();
        int64_t e = k0 + wave;
        // four entries per step, all loads issued before the sums (same summation order)
        for (; e + 12 < k1; e += 16) {
            const int32_t i0 = G.pidx[e], i1 = G.pidx[e + 4], i2 = G.pidx[e + 8], i3 = G.pidx[e + 12];
            const T v0 = part[(size_t)i0 * ld + a], v1 = part[(size_t)i1 * ld + a];
            const T v2 = part[(size_t)i2 * ld + a], v3 = part[(size_t)i3 * ld + a];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; e < k1; e += 4) acc += part[(size_t)G.pidx[e] * ld + a];
        red[wave * n + a] = acc;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        T v = red[a] + red[n + a] + red[2 * n + a] + red[3 * n + a];
        if (G.w) v = v * (G.scale * G.w[((size_t)t * n + a) * 4]);
        out[(size_t)t * n + a] = v;
    }
}

// Far field with coupling blocks generated on the fly (Sec. 4.2): for target
// cluster t, Y^_t[mu] = kappa_t[mu] sum_{s far} sum_nu G(x_mu, y_nu) kappa_s[nu] X^_s[nu].
// One workgroup per target row; each wave takes every 4th far block of the
// row, stages the source nodes and kappa-weighted moments in its own LDS
// slice, and its lanes own target nodes (up to 4 per lane for q^2 <= 256).
template <class T>
__global__ void __launch_bounds__(256) k_far_onthefly(int q2, const int64_t *__restrict__ ptr, const int32_t *__restrict__ src,
                                                      const double *__restrict__ nodes, const T *__restrict__ Xh,
                                                      double kappa, T *__restrict__ Yh, int64_t row0)
{
    constexpr int NC = NComp<T>::value;
    constexpr int ST = 3 + NC;  // staged doubles per source node: x, y, z, weight (re, im)
    extern __shared__ double sh[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    double *S = sh + (size_t)wave * q2 * ST;
    T *part = (T *)(sh + (size_t)nw * q2 * ST);  // nw * q2
    const int64_t t = row0 + blockIdx.x;
    const int64_t k0 = ptr[t], k1 = ptr[t + 1];
    const int nch = (q2 + 63) >> 6;
    double tx[4], ty[4], tz[4];
    T acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int mu = lane + 64 * c;
        acc[c] = zero<T>();
        tx[c] = ty[c] = tz[c] = 0.0;
        if (c < nch && mu < q2) {
            const double *nd = nodes + ((size_t)t * q2 + mu) * 4;
            tx[c] = nd[0];
            ty[c] = nd[1];
            tz[c] = nd[2];
        }
    }
    for (int64_t k = k0 + wave; k < k1; k += nw) {
        const int64_t sc = src[k];
        for (int nu = lane; nu < q2; nu += 64) {
            const double *nd = nodes + ((size_t)sc * q2 + nu) * 4;
            T w = Xh[(size_t)sc * q2 + nu] * nd[3];
            S[nu * ST + 0] = nd[0];
            S[nu * ST + 1] = nd[1];
            S[nu * ST + 2] = nd[2];
            S[nu * ST + 3] = re_(w);
            if constexpr (NC == 2) S[nu * ST + 4] = im_(w);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int nu = 0; nu < q2; ++nu) {
            const double sx = S[nu * ST], sy = S[nu * ST + 1], sz = S[nu * ST + 2], swr = S[nu * ST + 3];
            double swi = 0.0;
            if constexpr (NC == 2) swi = S[nu * ST + 4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c < nch) {
                    double d0 = tx[c] - sx, d1 = ty[c] - sy, d2 = tz[c] - sz;
                    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    if constexpr (NC == 1) {
                        acc[c] += rsqrt(r2) * swr;
                    } else {
                        double ir = rsqrt(r2), sn, cs;
                        sincos_red(kappa * (r2 * ir), &sn, &cs);
                        double gr = cs * ir, gi = sn * ir;
                        acc[c] += T{gr * swr - gi * swi, gr * swi + gi * swr};
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int mu = lane + 64 * c;
        if (c < nch && mu < q2) part[wave * q2 + mu] = acc[c];
    }
    __syncthreads();
    for (int mu = threadIdx.x; mu < q2; mu += blockDim.x) {
        T sum = part[mu];
        for (int w = 1; w < nw; ++w) sum += part[w * q2 + mu];
        Yh[(size_t)t * q2 + mu] = sum * (0.07957747154594767 * nodes[((size_t)t * q2 + mu) * 4 + 3]);
    }
}

// Far field generated on the fly, once per mirrored pair of coupling blocks
// (Sec. 4.2): G is symmetric, so the block of (s, t) is the transpose of the
// block of (t, s) and one evaluation of G(x_i, y_j) serves both products.
// One wave per pair k (t < s, same level); its 64 lanes form an 8 x 8 grid and
// lane (li, lj) owns targets li*TT .. li*TT+TT-1 and sources lj*TT .. lj*TT+TT-1
// (q^2 <= 8 TT).  The unscaled products are written as partial rows:
// part[2k] = sum_j G_ij w_j X_s[j] (for cluster t), part[2k+1] = sum_i G_ij w_i X_t[i]
// (for cluster s); k_far_gather sums them per cluster and applies the weights.
struct FarSymArgs {
    int64_t nup;
    const int32_t *up_t, *up_s;
    int q2;
    const double *nodes;
    double kappa;
    const double *sctab;  // sin, cos (j pi/128), j < 256 (complex kernel, see sincos_tab)
};

// Mirrored far-field pairs handled by one wave in a row (node data of the next
// pair is loaded while the current one is evaluated).  Two rather than four:
// the shorter far workgroups interleave better with the near ones of the
// single launch (sphere 0.146 -> 0.133 ms; the torus unchanged).
constexpr int kFarChunk = 2;

// LDS doubles per wave of far_mfma_chunk (W = 16 NTI padded nodes): the
// staged nodes and |x'|^2 (9 W), reused after the products for the row sums
// (W rows of 17) and the column sums (4 rows of W + 1).
template <int NTI>
constexpr int far_mfma_lds() { return 21 * 16 * NTI + 4; }

// LDS doubles per wave for the far-field pairs: the matrix-core path for the
// real kernel; for the complex one (far_sym_chunk) the pair's target and
// source nodes (x, y, z, weighted moment re, im) and its column sums (re,
// im), 8 TT each.
template <class T, int TT>
constexpr int far_sym_lds()
{
    if constexpr (NComp<T>::value == 1) return far_mfma_lds<(TT + 1) / 2>();
    else return 12 * 8 * TT;
}


// Node data of one cluster's node j for the far field: position and the
// weighted moment kappa_j X^[j] (padding nodes j >= q2: far from every node,
// zero weight; targets and sources are pushed to opposite sides).
template <class T>
struct FarNode {
    double x, y, z;
    T w;
};
template <class T>
__device__ inline FarNode<T> far_node(const FarSymArgs &F, const T *__restrict__ Xh, int64_t c, int j, double pad)
{
    FarNode<T> n{pad, 0.0, 0.0, zero<T>()};
    if (j < F.q2) {
        const double *nd = F.nodes + ((size_t)c * F.q2 + j) * 4;
        n.x = nd[0];
        n.y = nd[1];
        n.z = nd[2];
        n.w = Xh[(size_t)c * F.q2 + j] * nd[3];
    }
    return n;
}

// Kernel value G(x, y) 4 pi = exp(i kappa r) / r of the complex far field from r^2.  Double precision:
// refined reciprocal square root, the phase clamped into the range of sincos_red (padding nodes sit 1e100
// away; their weight is zero on one side and their value below 1e-100 on the other); with the table
// (TAB) the caller places the padding nodes so that no clamp is needed.  Single precision
// (RAW): the hardware reciprocal square root, the phase kappa r / (2 pi) in turns reduced to one turn
// (v_fract) for the hardware sine and cosine, which take turns.  TAB (double precision): sine and cosine
// from the table in LDS (sincos_tab) instead of sincos_red.
template <bool RAW, bool TAB = false>
__device__ inline void helm_far_value(typename std::conditional<RAW, float, double>::type r2,
                                      typename std::conditional<RAW, float, double>::type kap,
                                      typename std::conditional<RAW, float, double>::type &gr,
                                      typename std::conditional<RAW, float, double>::type &gi,
                                      const double *tab = nullptr)
{
    if constexpr (RAW) {
        const float ir = __builtin_amdgcn_rsqf(r2);
        const float ph = __builtin_amdgcn_fractf(r2 * ir * kap);
        gr = __builtin_amdgcn_cosf(ph) * ir;
        gi = __builtin_amdgcn_sinf(ph) * ir;
    } else {
        const double ir = rsqrt_pos(r2);
        double sn, cs;
        if constexpr (TAB) sincos_tab(kap * (r2 * ir), tab, &sn, &cs);  // phases bounded by the padding
        else sincos_red(fmin(kap * (r2 * ir), 0x1p19), &sn, &cs);
        gr = cs * ir;
        gi = sn * ir;
    }
}

// Add v into an LDS word (no return value).
template <class R>
__device__ inline void lds_add(R *p, R v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Complex kernel: pairs k0 .. k1-1 of the far field, executed by one whole wave;
// lds is the wave's slice of far_sym_lds<cd, TT>() doubles (the two clusters'
// nodes, then the pair's column sums).  Lane (li, lj) owns targets li*TT + ii
// and sources jj*8 + lj (ii, jj < TT).  The targets go in NP passes of at most
// five (seven in single precision), so that few of them are held in registers
// at a time.  For each source
// the lane's targets are summed in registers, reduced over the 8 lanes li
// (DPP) and added by lane li = 0 into the source's LDS column sum (eight
// distinct words per instruction); rows are reduced over the 8 lanes lj by
// lane shuffles at the end of the pass and written by the owner lanes.  The
// column sums are written after the last pass.  Positions are taken relative
// to the pair's first target node.  RAW: kernel values and the sums inside the
// pair in FP32 (positions rounded after the shift, so the rounding is relative
// to the cluster separation).
template <int TT, bool RAW, bool TAB = false>
__device__ inline void far_sym_chunk(const FarSymArgs &F, int64_t k0, int64_t k1, const cd *__restrict__ Xh,
                                     cd *__restrict__ part, double *lds, const double *tab = nullptr)
{
    using R = typename std::conditional<RAW, float, double>::type;
    constexpr int W = 8 * TT;  // padded nodes per cluster
    // passes of at most five targets per lane (single precision with more than 64 nodes: seven, whose
    // registers the FP32 values leave room for: far field 1.73 -> 1.59 ms on the torus)
    constexpr int NP = RAW && TT > 8 ? (TT + 6) / 7 : (TT + 4) / 5;
    constexpr int THL = TT / NP, NH = TT - THL * NP;  // NH passes of THL + 1 targets, NP - NH of THL
    constexpr int THH = NH > 0 ? THL + 1 : THL;
    double *tg = lds, *sr = lds + 5 * W;  // [x | y | z | w.re | w.im] x W each
    R *csum = (R *)(lds + 10 * W);        // (re, im) x W
    const int q2 = F.q2;
    const R kap = RAW ? (R)(F.kappa * 0.15915494309189535) : (R)F.kappa;  // RAW: turns per unit length
    const double pad = RAW ? 1e4 : 1e100;
    const int lane = threadIdx.x & 63;
    const int li = lane & 7, lj = lane >> 3;
    auto stage = [&](double *d, int j, const FarNode<cd> &n) {
        d[j] = n.x;
        d[W + j] = n.y;
        d[2 * W + j] = n.z;
        d[3 * W + j] = n.w.re;
        d[4 * W + j] = n.w.im;
    };
    for (int64_t k = k0; k < k1; ++k) {
        // the pair's nodes into LDS (the other waves of the SIMD cover the load latency), sums cleared
        for (int j = lane; j < W; j += 64) {
            stage(tg, j, far_node<cd>(F, Xh, F.up_t[k], j, pad));
            stage(sr, j, far_node<cd>(F, Xh, F.up_s[k], j, -pad));
            csum[2 * j] = csum[2 * j + 1] = (R)0;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        {
            // positions relative to the pair's first target node, in FP64, once per pair
            const double cx = tg[0], cy = tg[W], cz = tg[2 * W];
            double ext = 0.0;  // largest relative coordinate of a real node
            for (int j = lane; j < W; j += 64) {
                const double a0 = tg[j] - cx, a1 = tg[W + j] - cy, a2 = tg[2 * W + j] - cz;
                const double b0 = sr[j] - cx, b1 = sr[W + j] - cy, b2 = sr[2 * W + j] - cz;
                if (j < q2)
                    ext = fmax(ext, fmax(fmax(fmax(fabs(a0), fabs(a1)), fmax(fabs(a2), fabs(b0))),
                                         fmax(fabs(b1), fabs(b2))));
                tg[j] = a0;
                tg[W + j] = a1;
                tg[2 * W + j] = a2;
                sr[j] = b0;
                sr[W + j] = b1;
                sr[2 * W + j] = b2;
            }
            if constexpr (TAB) {
                // padding targets to (P, 0, 0), sources to (-P, 0, 0), P four times the pair's extent:
                // every distance from a padding node stays positive and every phase finite (the table
                // sine/cosine takes no clamp), and their zero weights cancel them exactly
                for (int o = 32; o > 0; o >>= 1) ext = fmax(ext, __shfl_xor(ext, o, 64));
                const double P = fmax(4.0 * ext, 1e-30);
                for (int j = q2 + lane; j < W; j += 64) {
                    tg[j] = P;
                    sr[j] = -P;
                    tg[W + j] = tg[2 * W + j] = sr[W + j] = sr[2 * W + j] = 0.0;
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
        cd *pr = part + (size_t)(2 * k) * q2, *pc = part + (size_t)(2 * k + 1) * q2;
        // one pass over all sources for THP targets per lane starting at t0
        auto pass = [&](auto thp, int t0) {
            constexpr int THP = decltype(thp)::value;
            R tx[THP], ty[THP], tz[THP], wr[THP], wi[THP], ar[THP], ai[THP];
#pragma unroll
            for (int ii = 0; ii < THP; ++ii) {
                const int i = li * TT + t0 + ii;
                tx[ii] = (R)tg[i];
                ty[ii] = (R)tg[W + i];
                tz[ii] = (R)tg[2 * W + i];
                wr[ii] = (R)tg[3 * W + i];
                wi[ii] = (R)tg[4 * W + i];
                ar[ii] = ai[ii] = (R)0;
            }
#pragma unroll 1
            for (int jj = 0; jj < TT; ++jj) {
                const int j = jj * 8 + lj;
                const R sx = (R)sr[j], sy = (R)sr[W + j], sz = (R)sr[2 * W + j];
                const R swr = (R)sr[3 * W + j], swi = (R)sr[4 * W + j];
                R pr_ = (R)0, pi_ = (R)0;
#pragma unroll
                for (int ii = 0; ii < THP; ++ii) {
                    const R d0 = tx[ii] - sx, d1 = ty[ii] - sy, d2 = tz[ii] - sz;
                    R gr, gi;
                    helm_far_value<RAW, TAB>(d0 * d0 + d1 * d1 + d2 * d2, kap, gr, gi, tab);
                    // two fused multiply-adds per real accumulation
                    ar[ii] = fma(gr, swr, ar[ii]);
                    ar[ii] = fma(-gi, swi, ar[ii]);
                    ai[ii] = fma(gr, swi, ai[ii]);
                    ai[ii] = fma(gi, swr, ai[ii]);
                    pr_ = fma(gr, wr[ii], pr_);
                    pr_ = fma(-gi, wi[ii], pr_);
                    pi_ = fma(gr, wi[ii], pi_);
                    pi_ = fma(gi, wr[ii], pi_);
                }
                pr_ = group8_sum(pr_);
                pi_ = group8_sum(pi_);
                if (li == 0) {
                    lds_add(csum + 2 * j, pr_);
                    lds_add(csum + 2 * j + 1, pi_);
                }
            }
            // rows of this pass: reduce over the 8 lanes lj; lane lj == ii writes target ii
#pragma unroll
            for (int ii = 0; ii < THP; ++ii) {
                R a = ar[ii], b = ai[ii];
#pragma unroll
                for (int o = 8; o < 64; o <<= 1) {
                    a += __shfl_xor(a, o);
                    b += __shfl_xor(b, o);
                }
                const int i = li * TT + t0 + ii;
                if (lj == ii && i < q2) pr[i] = cd{(double)a, (double)b};
            }
        };
        // TT targets per lane in NP passes: NH of THH targets, the rest of THL = THH - 1 (no padding)
#pragma unroll 1
        for (int h = 0; h < NH; ++h) pass(std::integral_constant<int, THH>{}, h * THH);
        if constexpr (THL > 0) {
#pragma unroll 1
            for (int h = NH; h < NP; ++h) pass(std::integral_constant<int, THL>{}, NH * THH + (h - NH) * THL);
        }
        __builtin_amdgcn_wave_barrier();  // every lane's additions are in before the sums are read
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        for (int j = lane; j < q2; j += 64) pc[j] = cd{(double)csum[2 * j], (double)csum[2 * j + 1]};
        __builtin_amdgcn_wave_barrier();  // every lane has read the nodes and sums before the next staging
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
}


// Real kernel: pairs k0 .. k1-1 with the squared distances on the matrix
// cores.  For a 16 x 16 tile of target nodes x and source nodes y, one
// v_mfma_f64_16x16x4f64 forms a . b + c with a = (x', 1), b = (-2 y', |y'|^2)
// and c = |x'|^2, i.e. |x - y|^2, where ' is relative to the pair's first
// target node (small operands: no cancellation for admissible pairs).  The
// vector units then take 1/|x - y| and the two weighted sums.  W = 16 NTI
// nodes per cluster (padding as in far_node).  Result layout of the product:
// lane l, element e holds row 4e + l/16 (target), column l%16 (source).
typedef double v4d_far __attribute__((ext_vector_type(4)));
template <int NTI, bool RAW>
__device__ inline void far_mfma_chunk(const FarSymArgs &F, int64_t k0, int64_t k1, const double *__restrict__ Xh,
                                      double *__restrict__ part, double *lds)
{
    constexpr int W = 16 * NTI;
    double *tg = lds, *sr = lds + 4 * W, *nx2 = lds + 8 * W;  // [x | y | z | w] x W each, |x'|^2
    double *rs = lds, *cs = lds + 17 * W;                     // after the products: row and column sums
    const int q2 = F.q2;
    const int lane = threadIdx.x & 63, col = lane & 15, sub = lane >> 4;
    FarNode<double> nt{}, ns{};
    if (lane < W) {
        nt = far_node<double>(F, Xh, F.up_t[k0], lane, 1e100);
        ns = far_node<double>(F, Xh, F.up_s[k0], lane, -1e100);
    }
    for (int64_t k = k0; k < k1; ++k) {
        if (lane < W) {
            tg[lane] = nt.x;
            tg[W + lane] = nt.y;
            tg[2 * W + lane] = nt.z;
            tg[3 * W + lane] = nt.w;
            sr[lane] = ns.x;
            sr[W + lane] = ns.y;
            sr[2 * W + lane] = ns.z;
            sr[3 * W + lane] = ns.w;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const double cx = tg[0], cy = tg[W], cz = tg[2 * W];
        if (lane < W) {
            const double a0 = nt.x - cx, a1 = nt.y - cy, a2 = nt.z - cz;
            nx2[lane] = a0 * a0 + a1 * a1 + a2 * a2;
        }
        if (k + 1 < k1 && lane < W) {  // prefetch the next pair
            nt = far_node<double>(F, Xh, F.up_t[k + 1], lane, 1e100);
            ns = far_node<double>(F, Xh, F.up_s[k + 1], lane, -1e100);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // every LDS value of the pair into registers first: the staging space
        // then takes the row and column sums
        const double ck = sub == 0 ? cx : (sub == 1 ? cy : cz);
        double bop[NTI], ws[NTI], csum[NTI], aop[NTI], wt[NTI][4];
        v4d_far cin[NTI];
#pragma unroll
        for (int tj = 0; tj < NTI; ++tj) {
            const int j = 16 * tj + col;
            const double y0 = sr[j] - cx, y1 = sr[W + j] - cy, y2 = sr[2 * W + j] - cz;
            bop[tj] = sub == 3 ? y0 * y0 + y1 * y1 + y2 * y2 : -2.0 * (sub == 0 ? y0 : (sub == 1 ? y1 : y2));
            ws[tj] = sr[3 * W + j];
            csum[tj] = 0.0;
        }
#pragma unroll
        for (int ti = 0; ti < NTI; ++ti) {
            aop[ti] = sub == 3 ? 1.0 : tg[sub * W + 16 * ti + col] - ck;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * ti + 4 * e + sub;
                cin[ti][e] = nx2[r];
                wt[ti][e] = tg[3 * W + r];
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
        for (int ti = 0; ti < NTI; ++ti) {
            double racc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int tj = 0; tj < NTI; ++tj) {
                const v4d_far d = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[ti], bop[tj], cin[ti], 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // RAW: the hardware estimate alone (relative error below 6e-8, single-precision
                    // far field); else refined to full double precision
                    const double ir = RAW ? __builtin_amdgcn_rsq(d[e]) : rsqrt_pos(d[e]);
                    racc[e] += ir * ws[tj];
                    csum[tj] += ir * wt[ti][e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) rs[(16 * ti + 4 * e + sub) * 17 + col] = racc[e];
        }
#pragma unroll
        for (int tj = 0; tj < NTI; ++tj) cs[sub * (W + 1) + 16 * tj + col] = csum[tj];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        double *pr = part + (size_t)(2 * k) * q2, *pc = part + (size_t)(2 * k + 1) * q2;
        for (int i = lane; i < q2; i += 64) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) v += rs[i * 17 + c];
            pr[i] = v;
            double u = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) u += cs[t * (W + 1) + i];
            pc[i] = u;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
}

// Far-field pairs k0 .. k1-1 of one wave: matrix-core path for the real
// kernel (RAW: single-precision kernel values), far_sym_chunk for the complex
// one (full precision only).
template <class T, int TT, bool RAW>
__device__ inline void far_chunk(const FarSymArgs &F, int64_t k0, int64_t k1, const T *__restrict__ Xh,
                                 T *__restrict__ part, double *lds, const double *tab = nullptr)
{
    if constexpr (NComp<T>::value == 1) {
        far_mfma_chunk<(TT + 1) / 2, RAW>(F, k0, k1, Xh, part, lds);
    } else if constexpr (TT > 8 && !RAW) {
        far_sym_chunk<TT, RAW, true>(F, k0, k1, Xh, part, lds, tab);  // sine and cosine from the LDS table
    } else {
        far_sym_chunk<TT, RAW>(F, k0, k1, Xh, part, lds);
    }
}

// three waves per SIMD for the real kernel: the far-field pairs need the
// occupancy more than the deeper product pipeline the compiler would build
template <class T, int TT, bool RAW>
__global__ void __launch_bounds__(256, NComp<T>::value == 1 ? 3 : 1) k_far_sym(FarSymArgs F, const T *__restrict__ Xh,
                                                                             T *__restrict__ part)
{
    __shared__ double buf[4][far_sym_lds<T, TT>()];
    const int wave = threadIdx.x >> 6;
    const int64_t k0 = ((int64_t)blockIdx.x * 4 + wave) * kFarChunk;
    if (k0 >= F.nup) return;  // whole waves only; no block-wide barrier follows
    far_chunk<T, TT, RAW>(F, k0, min(k0 + kFarChunk, F.nup), Xh, part, buf[wave]);
}

// The far-field pairs and the stored near blocks in one launch (ALU-bound and
// HBM-bound work on the same CUs): nf far workgroups (four waves of kFarChunk
// pairs) and nn near workgroups (four waves of one block), the near ones spread
// evenly through the grid (workgroup b is near iff
// floor((b+1) nn / (nf+nn)) > floor(b nn / (nf+nn))); nn = 0 gives the far
// pairs alone.  The complex kernel with more than 64 nodes per cluster (double
// precision) takes its sine and cosine from a table staged in LDS per
// workgroup and is held to three waves per SIMD.
// BT = cf: the near blocks of the single-precision complex product (FP32 copy, FP64 sums).
template <class T, int TT, bool RAW, class BT = T>
__global__ void __launch_bounds__(256, NComp<T>::value == 1 || TT > 8 ? 3 : 1) k_sym_products(FarSymArgs F, NearSymArgs N,
                                                                                  int64_t nf, int64_t nn,
                                                      const T *__restrict__ Xh, T *__restrict__ fpart,
                                                      const BT *__restrict__ blocks, const T *__restrict__ x,
                                                      T *__restrict__ npart)
{
    extern __shared__ double sh[];
    constexpr bool TAB = NComp<T>::value == 2 && TT > 8 && !RAW;
    __shared__ __attribute__((aligned(16))) double tabs[TAB ? 2 * kSinCosTab : 1];
    if constexpr (TAB) {  // before any wave leaves
        for (int i = threadIdx.x; i < 2 * kSinCosTab; i += blockDim.x) tabs[i] = F.sctab[i];
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6;
    const int64_t b = blockIdx.x, tot = nf + nn;
    const int64_t before = b * nn / tot, upto = (b + 1) * nn / tot;
    // per-wave LDS slice (doubles): the larger of the two kinds
    const int slice = max(far_sym_lds<T, TT>(), near_sym_lds(N.nl, N.ld) * NComp<T>::value);
    if (upto > before) {
        const int64_t k = before * 4 + wave;
        if (k >= N.nsb) return;
        if constexpr (std::is_same<BT, T>::value) near_sym_block<T>(N, k, blocks, x, npart, (T *)(sh + (size_t)wave * slice));
        else near_sym_block_c32(N, k, blocks, x, npart);
    } else {
        const int64_t k0 = ((b - before) * 4 + wave) * kFarChunk;
        if (k0 >= F.nup) return;
        far_chunk<T, TT, RAW>(F, k0, min(k0 + kFarChunk, F.nup), Xh, fpart, sh + (size_t)wave * slice, tabs);
    }
}

// ===========================================================================
// kernels: S <-> S* (Sec. 4.3) and order permutations
// ===========================================================================

struct Layout {
    int p, P1, nloc, nl, side, L, ne, ns1;
};

// internal S* index -> (patch, e1, e2, r1, r2)
__device__ inline void decode_internal(const Layout &lo, int64_t a, int &patch, int &e1, int &e2, int &r1, int &r2)
{
    int64_t leaf = a / lo.nl;
    int f = (int)(a % lo.nl);
    int el = f / lo.nloc, r = f % lo.nloc;
    int nL = 1 << lo.L;
    patch = (int)(leaf / (nL * nL));
    int rl = (int)(leaf % (nL * nL));
    int k2 = rl / nL, k1 = rl % nL;
    e1 = k1 * lo.side + el % lo.side;
    e2 = k2 * lo.side + el / lo.side;
    r1 = r % lo.P1;
    r2 = r / lo.P1;
}

__device__ inline int64_t encode_internal(const Layout &lo, int patch, int e1, int e2, int r1, int r2)
{
    int nL = 1 << lo.L;
    int64_t leaf = (int64_t)patch * nL * nL + (e2 / lo.side) * nL + e1 / lo.side;
    int el = (e2 % lo.side) * lo.side + e1 % lo.side;
    return leaf * lo.nl + el * lo.nloc + r2 * lo.P1 + r1;
}

// The three kernels below take the degree as a template parameter (P1 = P + 1
// terms per direction, loops fully unrolled so that every load of a thread is
// in flight at once) and 32-bit index arithmetic (the host checks that the
// superspace size fits).
template <int P>
__device__ inline void decode_internal32(const Layout &lo, int a, int &patch, int &e1, int &e2, int &r1, int &r2)
{
    constexpr int P1 = P + 1;
    const int leaf = a / lo.nl, f = a - leaf * lo.nl;
    const int el = f / (P1 * P1), r = f - el * (P1 * P1);
    const int nL = 1 << lo.L, l2 = leaf >> (2 * lo.L), rl = leaf & (nL * nL - 1);
    patch = l2;
    const int k2 = rl >> lo.L, k1 = rl & (nL - 1);
    e1 = k1 * lo.side + el % lo.side;
    e2 = k2 * lo.side + el / lo.side;
    r1 = r % P1;
    r2 = r / P1;
}

// xs = T^T w: superspace coefficient a (patch, e1, e2, r1, r2) gathers the
// P1 x P1 B-spline coefficients whose support covers element (e1, e2).
template <class T, int P>
__global__ void k_Tt(Layout lo, int nsup, const double *__restrict__ Tb, const T *__restrict__ w, T *__restrict__ xs)
{
    constexpr int P1 = P + 1;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nsup) return;
    int patch, e1, e2, r1, r2;
    decode_internal32<P>(lo, a, patch, e1, e2, r1, r2);
    const double *t1 = Tb + (e1 * P1 + r1) * P1, *t2 = Tb + (e2 * P1 + r2) * P1;
    const T *wp = w + patch * lo.ns1 * lo.ns1 + e2 * lo.ns1 + e1;
    T s = zero<T>();
#pragma unroll
    for (int j2 = 0; j2 < P1; ++j2)
#pragma unroll
        for (int j1 = 0; j1 < P1; ++j1) s += (t1[j1] * t2[j2]) * wp[j2 * lo.ns1 + j1];
    xs[a] = s;
}

// y = T ys applied as (T1 (x) T1) per patch in two separable passes.
// Pass 1: Z[patch][e2][r2][j1] = sum_{e1, r1} T1[j1, (e1, r1)] ys[patch, e1, e2, r1, r2]
// (element e1 = j1 - P + d, d < P1, inside the patch)
template <class T, int P>
__global__ void k_T_pass1(Layout lo, int npatch, const double *__restrict__ Tb, const T *__restrict__ ys, T *__restrict__ Z)
{
    constexpr int P1 = P + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = npatch * lo.ne * P1 * lo.ns1;
    if (i >= n) return;
    const int j1 = i % lo.ns1, rest = i / lo.ns1;
    const int r2 = rest % P1, rest2 = rest / P1;
    const int e2 = rest2 % lo.ne, patch = rest2 / lo.ne;
    const int nL = 1 << lo.L;
    const int leafrow = (patch * nL + e2 / lo.side) * nL, elrow = (e2 % lo.side) * lo.side;
    T s = zero<T>();
#pragma unroll
    for (int d = 0; d < P1; ++d) {
        const int e1 = j1 - P + d;
        if (e1 < 0 || e1 >= lo.ne) continue;
        const int leaf = leafrow + e1 / lo.side, el = elrow + e1 % lo.side;
        const T *y0 = ys + leaf * lo.nl + el * (P1 * P1) + r2 * P1;
        const double *tb = Tb + e1 * P1 * P1 + (P - d);
#pragma unroll
        for (int r1 = 0; r1 < P1; ++r1) s += tb[r1 * P1] * y0[r1];
    }
    Z[i] = s;
}

// Pass 2: y[patch][j2][j1] = sum_{e2, r2} T1[j2, (e2, r2)] Z[patch][e2][r2][j1];
// with dx given, part[block] = sum over the block's i of conj(dx[i]) y[i].
template <class T, int P>
__global__ void __launch_bounds__(256) k_T_pass2(Layout lo, int ndof, const double *__restrict__ Tb,
                                                 const T *__restrict__ Z, T *__restrict__ y, const T *__restrict__ dx,
                                                 T *__restrict__ part)
{
    constexpr int P1 = P + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    T s = zero<T>();
    if (i < ndof) {
        const int nn = lo.ns1 * lo.ns1;
        const int patch = i / nn, r = i % nn, j2 = r / lo.ns1, j1 = r % lo.ns1;
        const T *Zp = Z + patch * lo.ne * P1 * lo.ns1 + j1;
#pragma unroll
        for (int d = 0; d < P1; ++d) {
            const int e2 = j2 - P + d;
            if (e2 < 0 || e2 >= lo.ne) continue;
            const double *tb = Tb + e2 * P1 * P1 + (P - d);
#pragma unroll
            for (int r2 = 0; r2 < P1; ++r2) s += tb[r2 * P1] * Zp[(e2 * P1 + r2) * lo.ns1];
        }
        y[i] = s;
    }
    if (dx) {
        __shared__ T red[256];
        red[threadIdx.x] = i < ndof ? conj_(dx[i]) * s : zero<T>();
        __syncthreads();
        for (int k = blockDim.x / 2; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = red[0];
    }
}

// external S* order (element-major) <-> internal (leaf-major)
template <class T>
__global__ void k_perm(Layout lo, int64_t nsup, const T *__restrict__ in, T *__restrict__ out, int to_internal)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nsup) return;
    int patch, e1, e2, r1, r2;
    decode_internal(lo, a, patch, e1, e2, r1, r2);
    int64_t ext = ((int64_t)patch * lo.ne * lo.ne + (int64_t)e2 * lo.ne + e1) * lo.nloc + r2 * lo.P1 + r1;
    if (to_internal) out[a] = in[ext];
    else out[ext] = in[a];
}

// ===========================================================================
// kernels: right-hand side and potential
// ===========================================================================

__global__ void k_rhs_points(int64_t n, const double *__restrict__ rp, double *__restrict__ xyz)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xyz[3 * i] = rp[4 * i];
    xyz[3 * i + 1] = rp[4 * i + 1];
    xyz[3 * i + 2] = rp[4 * i + 2];
}

// g*_a = sum_q g(x_q) kappa w_q phi_a(x_q) on the element of a (internal order)
template <class T>
__global__ void k_rhs_super(Layout lo, int64_t nsup, int g, const double *__restrict__ gxr, const double *__restrict__ rp,
                            const T *__restrict__ gv, T *__restrict__ gs)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nsup) return;
    int patch, e1, e2, r1, r2;
    decode_internal(lo, a, patch, e1, e2, r1, r2);
    int64_t E = (int64_t)patch * lo.ne * lo.ne + (int64_t)e2 * lo.ne + e1;
    T s = zero<T>();
    double B[9];
    for (int j = 0; j < g; ++j) {
        bernstein(lo.p, gxr[j], B);
        double b2 = B[r2];
        for (int i = 0; i < g; ++i) {
            bernstein(lo.p, gxr[i], B);
            int64_t k = E * g * g + j * g + i;
            s += gv[k] * (rp[4 * k + 3] * B[r1] * b2);
        }
    }
    gs[a] = s;
}

// per quadrature point of the potential: c_q = mu_h(y_q) kappa w_q
template <class T>
__global__ void k_pot_prep(Layout lo, int nelem, int g, const double *__restrict__ gxr, const double *__restrict__ rp,
                           const T *__restrict__ xs, T *__restrict__ c)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int gg = g * g;
    if (k >= (int64_t)nelem * gg) return;
    int E = (int)(k / gg), ij = (int)(k % gg), j = ij / g, i = ij % g;
    int patch = E / (lo.ne * lo.ne), r = E % (lo.ne * lo.ne), e2 = r / lo.ne, e1 = r % lo.ne;
    double Bi[9], Bj[9];
    bernstein(lo.p, gxr[i], Bi);
    bernstein(lo.p, gxr[j], Bj);
    T s = zero<T>();
    for (int r2 = 0; r2 < lo.P1; ++r2)
        for (int r1 = 0; r1 < lo.P1; ++r1) s += (Bi[r1] * Bj[r2]) * xs[encode_internal(lo, patch, e1, e2, r1, r2)];
    c[k] = s * rp[4 * k + 3];
}

// direct sum over source chunks: part[chunk * npts + x] = sum_q c_q G(x, y_q)
template <class T>
__global__ void __launch_bounds__(256) k_pot_eval(int64_t npts, const double *__restrict__ X, int64_t nsrc,
                                                  const double *__restrict__ rp, const T *__restrict__ c, double kappa,
                                                  int64_t chunk, T *__restrict__ part, const double *__restrict__ tab,
                                                  double hx, double hy, double hz, double hr)
{
    constexpr bool CPLX = NComp<T>::value == 2;
    __shared__ double sy[256 * 3];
    __shared__ T sc[256];
    __shared__ __attribute__((aligned(16))) double stab[CPLX ? 2 * kSinCosTab : 1];
    if constexpr (CPLX)
        for (int i = threadIdx.x; i < 2 * kSinCosTab; i += blockDim.x) stab[i] = tab[i];
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s0 = (int64_t)blockIdx.y * chunk, s1 = s0 + chunk < nsrc ? s0 + chunk : nsrc;
    double px = 0, py = 0, pz = 0;
    if (x < npts) { px = X[3 * x]; py = X[3 * x + 1]; pz = X[3 * x + 2]; }
    // a point within 2^19 / kappa of the ball (hx, hy, hz; hr) around the surface has every phase
    // kappa |x - y| below 2^19: refined reciprocal square root and table sine and cosine; farther
    // points take the library's square root, sine and cosine
    const double hd = sqrt((px - hx) * (px - hx) + (py - hy) * (py - hy) + (pz - hz) * (pz - hz));
    const bool fast = kappa * (hd + hr) < 0x1p19;
    T acc = zero<T>();
    for (int64_t b = s0; b < s1; b += 256) {
        int64_t q = b + threadIdx.x;
        if (q < s1) {
            sy[3 * threadIdx.x] = rp[4 * q];
            sy[3 * threadIdx.x + 1] = rp[4 * q + 1];
            sy[3 * threadIdx.x + 2] = rp[4 * q + 2];
            sc[threadIdx.x] = c[q];
        }
        __syncthreads();
        int nb = (int)((s1 - b) < 256 ? (s1 - b) : 256);
        if (fast) {
            for (int k = 0; k < nb; ++k) {
                double d0 = px - sy[3 * k], d1 = py - sy[3 * k + 1], d2 = pz - sy[3 * k + 2];
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double ir = r2 > 0.0 ? rsqrt_pos(r2) : __builtin_inf();
                const double f = 0.07957747154594767 * ir;
                if constexpr (CPLX) {
                    double sn, cs;
                    sincos_tab(kappa * (r2 * ir), stab, &sn, &cs);
                    acc += T{cs * f, sn * f} * sc[k];
                } else {
                    acc += f * sc[k];
                }
            }
        } else {
            for (int k = 0; k < nb; ++k) {
                double d0 = px - sy[3 * k], d1 = py - sy[3 * k + 1], d2 = pz - sy[3 * k + 2];
                acc += green_any<T>(sqrt(d0 * d0 + d1 * d1 + d2 * d2), kappa) * sc[k];
            }
        }
        __syncthreads();
    }
    if (x < npts) part[(int64_t)blockIdx.y * npts + x] = acc;
}

// Sum over the 64 lanes of a wave (every lane gets it).
__device__ inline double wave_sum64(double s)
{
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}
__device__ inline cd wave_sum64(cd s) { return {wave_sum64(s.re), wave_sum64(s.im)}; }

// The potential with the far field interpolated (the H2 approximation of Sec. 4.2 applied to the point
// evaluation of Sec. 3.1, eq. eq::repform): from the clusters of the coarsest far-field level down, a
// cluster s is admissible for the point x when diam(s) < eta (|x - c_s| - r_s) (centre c_s and radius r_s
// of its surface grid) and kappa diam(s) <= kappa_diam (kPotKappaDiam, or the operator's smaller
// wavenumber option: the interpolation of exp(i kappa r) over the cluster then stays accurate); it then
// contributes sum_nu G(x, F(xi_nu)) kappa(xi_nu) X^_nu at its Chebyshev nodes
// (moments X^ of the density from the upward pass), else its children are visited; leaves that are never
// admissible contribute the direct sum over their quadrature points.  One wave per point: the lanes test
// 64 candidate clusters at a time, then evaluate the admissible clusters' nodes and the near leaves'
// points together.  A level with more than kH2Cap candidates sets *flag and leaves the point unwritten.
constexpr int kH2Cap = 1024;
// kappa diam(s) of the clusters the Helmholtz potential interpolates: Chebyshev interpolation of the phase
// over a cluster of kappa diam = 4 errs by about (kappa diam / 2)^q / (2^(q-1) q!), 5e-7 at q = 10
constexpr double kPotKappaDiam = 4.0;
constexpr int kH2MaxLevel = 15;
struct PotH2Args {
    int lmin, L, npatch, q2, ne, side, gg;
    int64_t cl_off[kH2MaxLevel + 2];
    const double *clg;    // per global cluster: centre (3), radius, diameter
    const double *nodes;  // per global cluster: q2 x (x, y, z, surface measure)
    const void *Xh;       // moments, q2 per global cluster
    const double *rp;     // quadrature points of the potential rule (x, y, z, weight)
    const void *c;        // weighted density at them
    double eta, kappa, kappa_diam, hx, hy, hz, hr;
    const double *tab;
    int *flag;
};

template <class T>
__global__ void __launch_bounds__(256) k_pot_h2(int64_t npts, const double *__restrict__ X, PotH2Args A,
                                                T *__restrict__ u)
{
    constexpr bool CPLX = NComp<T>::value == 2;
    __shared__ int32_t lists[4][2][kH2Cap];
    __shared__ __attribute__((aligned(16))) double stab[CPLX ? 2 * kSinCosTab : 1];
    if constexpr (CPLX)
        for (int i = threadIdx.x; i < 2 * kSinCosTab; i += blockDim.x) stab[i] = A.tab[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t x = (int64_t)blockIdx.x * 4 + wave;
    if (x >= npts) return;  // whole waves; no barrier follows
    const double px = X[3 * x], py = X[3 * x + 1], pz = X[3 * x + 2];
    const double hd = sqrt((px - A.hx) * (px - A.hx) + (py - A.hy) * (py - A.hy) + (pz - A.hz) * (pz - A.hz));
    const bool fast = A.kappa * (hd + A.hr) < 0x1p19;  // every phase in the range of the table sine/cosine
    const T *Xh = (const T *)A.Xh, *cq = (const T *)A.c;
    auto gval = [&](double y0, double y1, double y2) -> T {
        const double d0 = px - y0, d1 = py - y1, d2 = pz - y2;
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (fast) {
            const double ir = r2 > 0.0 ? rsqrt_pos(r2) : __builtin_inf();
            const double f = 0.07957747154594767 * ir;
            if constexpr (CPLX) {
                double sn, cs;
                sincos_tab(A.kappa * (r2 * ir), stab, &sn, &cs);
                return T{cs * f, sn * f};
            } else {
                return f;
            }
        }
        return green_any<T>(sqrt(r2), A.kappa);
    };
    T acc = zero<T>();
    int32_t *cur = lists[wave][0], *nxt = lists[wave][1];
    int ncur = A.npatch << (2 * A.lmin);  // the coarsest level: every cluster, by index
    bool all = true;
    for (int l = A.lmin; l <= A.L && ncur > 0; ++l) {
        const int n = 1 << l;
        int nnext = 0;
        for (int base = 0; base < ncur; base += 64) {
            const int k = base + lane;
            const bool valid = k < ncur;
            const int c = valid ? (all ? k : cur[k]) : 0;
            bool adm = false;
            if (valid) {
                const double *cg = A.clg + (A.cl_off[l] + c) * 5;
                const double dc = sqrt((px - cg[0]) * (px - cg[0]) + (py - cg[1]) * (py - cg[1]) +
                                       (pz - cg[2]) * (pz - cg[2]));
                adm = dc - cg[3] > 0.0 && cg[4] < A.eta * (dc - cg[3]) && A.kappa * cg[4] <= A.kappa_diam;
            }
            const unsigned long long mfar = __ballot(valid && adm);
            const unsigned long long mnear = __ballot(valid && !adm && l == A.L);
            const unsigned long long msplit = __ballot(valid && !adm && l < A.L);
            if (valid && !adm && l < A.L) {  // the four children, in lane order
                const int pos = nnext + 4 * __popcll(msplit & ((1ull << lane) - 1ull));
                const int patch = c / (n * n), r = c % (n * n), k2 = r / n, k1 = r % n, nn = 2 * n;
                for (int a = 0; a < 4; ++a)
                    if (pos + a < kH2Cap) nxt[pos + a] = patch * nn * nn + (2 * k2 + (a >> 1)) * nn + 2 * k1 + (a & 1);
            }
            nnext += 4 * __popcll(msplit);
            for (unsigned long long m = mfar; m; m &= m - 1) {  // admissible: the cluster's nodes
                const int64_t g = A.cl_off[l] + __shfl(c, __ffsll((long long)m) - 1);
                for (int nu = lane; nu < A.q2; nu += 64) {
                    const double *nd = A.nodes + (g * A.q2 + nu) * 4;
                    acc += gval(nd[0], nd[1], nd[2]) * (Xh[g * A.q2 + nu] * nd[3]);
                }
            }
            for (unsigned long long m = mnear; m; m &= m - 1) {  // near leaf: its quadrature points
                const int cl = __shfl(c, __ffsll((long long)m) - 1);
                const int patch = cl / (n * n), r = cl % (n * n), k2 = r / n, k1 = r % n;
                const int row = A.side * A.gg, npl = A.side * row;
                for (int t = lane; t < npl; t += 64) {
                    const int64_t kq = ((int64_t)patch * A.ne * A.ne + (int64_t)(k2 * A.side + t / row) * A.ne +
                                        (int64_t)k1 * A.side) * A.gg + t % row;
                    const double *y = A.rp + kq * 4;
                    acc += gval(y[0], y[1], y[2]) * cq[kq];
                }
            }
        }
        if (nnext > kH2Cap) {  // uniform: the host evaluates these points by the direct sum instead
            if (lane == 0) *A.flag = 1;
            return;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
        ncur = nnext;
        all = false;
    }
    acc = wave_sum64(acc);
    if (lane == 0) u[x] = acc;
}

template <class T>
__global__ void k_pot_reduce(int64_t npts, int nchunk, const T *__restrict__ part, T *__restrict__ u)
{
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= npts) return;
    T s = zero<T>();
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * npts + x];
    u[x] = s;
}

// ===========================================================================
// kernels: Jacobi diagonal D_i = t_i^T A t_i
// ===========================================================================

__device__ inline int64_t csr_find(const int64_t *ptr, const int32_t *idx, int64_t row, int32_t key)
{
    int64_t lo = ptr[row], hi = ptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t v = idx[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

struct DiagArgs {
    Layout lo;
    int m, q, lmin;
    const double *Tb;
    const double *Mlev;
    const int64_t *Mlev_off;
    const int64_t *cl_off;
    const int64_t *near_ptr;
    const int32_t *near_src;
    const int32_t *sb;  // stored near block of each CSR entry (-1: read the mirror transposed)
    int ld;             // column stride of the stored near blocks
    const void *cbuf;   // per stored block, the near-field terms of k_diag_blocks (or null)
    const int64_t *far_ptr;
    const int32_t *far_src;
    const double *nodes;
    double kappa;
};

// Kernel value from |d|^2 and 1/|d| (Sec. 3.1 fundamental solutions).
template <class T> __device__ inline T green_ir(double r2, double ir, double kappa);
template <> __device__ inline double green_ir<double>(double, double ir, double) { return 0.07957747154594767 * ir; }
template <> __device__ inline cd green_ir<cd>(double r2, double ir, double kappa)
{
    double sn, cs;
    sincos_red(kappa * (r2 * ir), &sn, &cs);
    const double f = 0.07957747154594767 * ir;
    return {cs * f, sn * f};
}

// Near-field terms of the Jacobi diagonal, block by block (symmetric storage):
// for the stored leaf block B of (t, s) (t <= s) and every B-spline j whose
// support meets both leaves, c = u^T B v with u, v the restrictions of
// t_j = T^T e_j to the superspace functions of t and of s (tensor products of
// the 1D weights of Sec. 4.3, zero where the support does not reach).  One
// workgroup per stored block; c goes to slot (j2 - j2lo) W + (j1 - j1lo) of
// the block's W^2 (W = side + p), (j1lo, j2lo) the first B-spline of the
// window both leaves share.  Leaves of different patches share no B-spline.
// LDS: V (nl x nj), the four 1D weight tables, the row terms (nj x nl).
template <class T>
__global__ void __launch_bounds__(256) k_diag_blocks(Layout lo, const int32_t *__restrict__ sb_t,
                                                     const int32_t *__restrict__ sb_s, int ld,
                                                     const double *__restrict__ Tb, const T *__restrict__ nearb,
                                                     T *__restrict__ cbuf)
{
    extern __shared__ double sh[];
    const int64_t k = blockIdx.x;
    const int P1 = lo.P1, p = lo.p, side = lo.side, nl = lo.nl, nloc = lo.nloc, W = side + p, SP = side * P1;
    const int n = 1 << lo.L;
    const int t = sb_t[k], s = sb_s[k];
    if (t / (n * n) != s / (n * n)) return;
    const int rt = t % (n * n), rs = s % (n * n);
    const int t2 = rt / n, t1 = rt % n, s2 = rs / n, s1 = rs % n;
    const int j1lo = max(t1, s1) * side, j1hi = min(t1, s1) * side + side - 1 + p;
    const int j2lo = max(t2, s2) * side, j2hi = min(t2, s2) * side + side - 1 + p;
    if (j1lo > j1hi || j2lo > j2hi) return;
    const int w1 = j1hi - j1lo + 1, w2 = j2hi - j2lo + 1, nj = w1 * w2;
    double *V = sh;                                   // [nl][nj]
    double *Tt1 = V + (size_t)nl * nj, *Tt2 = Tt1 + SP * w1, *Ts1 = Tt2 + SP * w2, *Ts2 = Ts1 + SP * w1;
    T *red = (T *)(sh + (((size_t)nl * nj + 2 * (size_t)SP * (w1 + w2) + 1) & ~(size_t)1));  // [nj][nl], 16-byte aligned
    // 1D weights: leaf-local index i = el*P1 + r along one direction, B-spline j = jlo + jj
    auto w1d = [&](int leafk, int i, int jj, int jlo) -> double {
        const int e = leafk * side + i / P1, r = i % P1, j = jlo + jj, d = j - e;
        return (d >= 0 && d <= p) ? Tb[(e * P1 + r) * P1 + d] : 0.0;
    };
    for (int x = threadIdx.x; x < SP * w1; x += blockDim.x) {
        Tt1[x] = w1d(t1, x / w1, x % w1, j1lo);
        Ts1[x] = w1d(s1, x / w1, x % w1, j1lo);
    }
    for (int x = threadIdx.x; x < SP * w2; x += blockDim.x) {
        Tt2[x] = w1d(t2, x / w2, x % w2, j2lo);
        Ts2[x] = w1d(s2, x / w2, x % w2, j2lo);
    }
    __syncthreads();
    // superspace function f of a leaf: element el = el2*side + el1, r = r2*P1 + r1
    auto i1of = [&](int f) { const int el = f / nloc, r = f % nloc; return (el % side) * P1 + r % P1; };
    auto i2of = [&](int f) { const int el = f / nloc, r = f % nloc; return (el / side) * P1 + r / P1; };
    for (int x = threadIdx.x; x < nl * nj; x += blockDim.x) {
        const int b = x / nj, jj = x % nj;
        V[x] = Ts1[i1of(b) * w1 + jj % w1] * Ts2[i2of(b) * w2 + jj / w1];
    }
    __syncthreads();
    // 256 threads: lane = row a (mod 64), group g of four takes the window columns
    // jj = g, g+4, ...; y = B v for those columns, then the row's share of u^T y
    // 256 threads: lane = row a (mod 64), group g of four takes the window columns
    // jj = g, g+4, ...; y = B v for those columns, the row's share of u^T y into
    // red[jj][a], then one fixed-order sum per column
    const T *B = nearb + k * (int64_t)nl * ld;  // column b: rows a of leaf t, stride ld
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    constexpr int YC = 16;  // columns per thread, nj <= 64
    for (int a = lane; a < nl; a += 64) {
        T y[YC];
#pragma unroll
        for (int c = 0; c < YC; ++c) y[c] = zero<T>();
        for (int b = 0; b < nl; ++b) {
            const T Bab = B[(int64_t)b * ld + a];
            const double *vb = V + (size_t)b * nj;
#pragma unroll
            for (int c = 0; c < YC; ++c)
                if (g + 4 * c < nj) y[c] += Bab * vb[g + 4 * c];
        }
        const int ia1 = i1of(a), ia2 = i2of(a);
#pragma unroll
        for (int c = 0; c < YC; ++c) {
            const int jj = g + 4 * c;
            if (jj < nj) red[(size_t)jj * nl + a] = y[c] * (Tt1[ia1 * w1 + jj % w1] * Tt2[ia2 * w2 + jj / w1]);
        }
    }
    __syncthreads();
    for (int jj = threadIdx.x; jj < nj; jj += blockDim.x) {
        T v = zero<T>();
        for (int a = 0; a < nl; ++a) v += red[(size_t)jj * nl + a];
        cbuf[k * W * W + (int64_t)(jj / w1) * W + jj % w1] = v;
    }
}

// One workgroup per B-spline function i (patch, j1, j2); its support is the
// element window [lo1, hi1] x [lo2, hi2].  Far field: at every level, the
// moments of t_i on the clusters meeting the support, then for every
// admissible pair of those clusters (each unordered pair once: the coupling
// kernel is symmetric) the q^2 x q^2 coupling product, one (pair, column)
// work item per thread.  Near field: the superspace functions of the support
// elements with their weights in t_i (zero weights included, in a fixed
// order), and for every pair of them the stored near-field entry (blocks read
// through the symmetric storage map).  Fixed summation order throughout.
template <class T>
__global__ void __launch_bounds__(256) k_diag(DiagArgs A, int64_t ndof, const T *__restrict__ nearb,
                                              const T *__restrict__ coup, T *__restrict__ D)
{
    extern __shared__ double sh[];
    __shared__ T red[256];
    __shared__ unsigned char ff[4096];
    const Layout &lo = A.lo;
    const int q = A.q, q2 = q * q, P1 = lo.P1;
    const int64_t i = blockIdx.x;
    const int nn = lo.ns1 * lo.ns1;
    const int patch = (int)(i / nn), rr = (int)(i % nn), j2 = rr / lo.ns1, j1 = rr % lo.ns1;
    const int lo1 = j1 - lo.p < 0 ? 0 : j1 - lo.p, hi1 = j1 < lo.ne - 1 ? j1 : lo.ne - 1;
    const int lo2 = j2 - lo.p < 0 ? 0 : j2 - lo.p, hi2 = j2 < lo.ne - 1 ? j2 : lo.ne - 1;
    T acc = zero<T>();
    double *mv = sh;  // up to (p+2)^2 clusters x q2
    // far field, level by level
    for (int l = A.lmin; l <= lo.L; ++l) {
        const int nsub = lo.ne >> l, n = 1 << l;
        const int c1lo = lo1 / nsub, c1hi = hi1 / nsub, c2lo = lo2 / nsub, c2hi = hi2 / nsub;
        const int nc1 = c1hi - c1lo + 1, nc = nc1 * (c2hi - c2lo + 1);
        const double *Ml = A.Mlev + A.Mlev_off[l];
        // the moments of t_i on a cluster are tensor products: one 1D sum per
        // cluster column and node (s1) and per cluster row and node (s2)
        const int nc2 = nc / nc1;
        double *s1 = mv + (size_t)nc * q2, *s2 = s1 + (size_t)nc1 * q;
        for (int o = threadIdx.x; o < (nc1 + nc2) * q; o += blockDim.x) {
            const bool first = o < nc1 * q;
            const int oo = first ? o : o - nc1 * q, c = oo / q, mu = oo % q;
            const int cc = (first ? c1lo : c2lo) + c, jj = first ? j1 : j2;
            const int elo = first ? lo1 : lo2, ehi = first ? hi1 : hi2;
            double sum = 0.0;
            for (int e = (elo > cc * nsub ? elo : cc * nsub); e <= ehi && e < (cc + 1) * nsub; ++e)
                for (int r = 0; r < P1; ++r)
                    sum += A.Tb[(e * P1 + r) * P1 + (jj - e)] * Ml[((e - cc * nsub) * P1 + r) * q + mu];
            (first ? s1 : s2)[oo] = sum;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < nc * q2; o += blockDim.x) {
            const int c = o / q2, mu = o % q2, mu2 = mu / q, mu1 = mu % q;
            mv[o] = s1[(c % nc1) * q + mu1] * s2[(c / nc1) * q + mu2];
        }
        // admissible pairs ca < cb
        for (int c = threadIdx.x; c < nc * nc; c += blockDim.x) {
            const int ca = c / nc, cb = c % nc;
            unsigned char f = 0;
            if (ca < cb) {
                const int ida = patch * n * n + (c2lo + ca / nc1) * n + c1lo + ca % nc1;
                const int idb = patch * n * n + (c2lo + cb / nc1) * n + c1lo + cb % nc1;
                f = csr_find(A.far_ptr, A.far_src, A.cl_off[l] + ida, (int32_t)(A.cl_off[l] + idb)) >= 0;
            }
            ff[c] = f;
        }
        __syncthreads();
        for (int w = threadIdx.x; w < nc * nc * q2; w += blockDim.x) {
            const int c = w / q2, nu = w % q2;
            if (!ff[c]) continue;
            const int ca = c / nc, cb = c % nc;
            const int ida = patch * n * n + (c2lo + ca / nc1) * n + c1lo + ca % nc1;
            const int idb = patch * n * n + (c2lo + cb / nc1) * n + c1lo + cb % nc1;
            // coupling entries K[mu][nu] = G(x_mu, y_nu) kappa_mu kappa_nu from the node geometry
            const double *na = A.nodes + (size_t)(A.cl_off[l] + ida) * q2 * 4;
            const double *y = A.nodes + ((size_t)(A.cl_off[l] + idb) * q2 + nu) * 4;
            const double y0 = y[0], y1 = y[1], y2 = y[2];
            T s = zero<T>();
            for (int mu = 0; mu < q2; ++mu) {
                const double *x = na + 4 * mu;
                const double d0 = x[0] - y0, d1 = x[1] - y1, d2 = x[2] - y2;
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                s += green_ir<T>(r2, rsqrt_pos(r2), A.kappa) * (x[3] * mv[ca * q2 + mu]);
            }
            // the pair (cb, ca) contributes the same amount
            acc += s * (2.0 * y[3] * mv[cb * q2 + nu]);
        }
        __syncthreads();
    }
    // near field at the leaf level: from the per-block terms of k_diag_blocks
    // (each unordered pair of support leaves once, twice when they differ) ...
    if (A.cbuf) {
        const int nsub = lo.side, n = 1 << lo.L, W = lo.side + lo.p;
        const int c1lo = lo1 / nsub, c1hi = hi1 / nsub, c2lo = lo2 / nsub, c2hi = hi2 / nsub;
        const int nc1 = c1hi - c1lo + 1, nc = nc1 * (c2hi - c2lo + 1);
        const T *cb = (const T *)A.cbuf;
        for (int w = threadIdx.x; w < nc * nc; w += blockDim.x) {
            const int ca = w / nc, cbb = w % nc;
            if (cbb < ca) continue;
            const int a1 = c1lo + ca % nc1, a2 = c2lo + ca / nc1, b1 = c1lo + cbb % nc1, b2 = c2lo + cbb / nc1;
            const int ia = patch * n * n + a2 * n + a1, ib = patch * n * n + b2 * n + b1;
            const bool fwd = ia <= ib;
            const int64_t e = csr_find(A.near_ptr, A.near_src, fwd ? ia : ib, fwd ? ib : ia);
            if (e < 0) continue;
            const int64_t kb = A.sb[e];
            const int j1lo = max(a1, b1) * nsub, j2lo = max(a2, b2) * nsub;
            const T v = cb[kb * W * W + (int64_t)(j2 - j2lo) * W + (j1 - j1lo)];
            acc += ca == cbb ? v : 2.0 * v;
        }
    } else {
    // ... or, for non-symmetric storage, entry by entry
    {
        const int nsub = lo.side, n = 1 << lo.L;
        const int c1lo = lo1 / nsub, c1hi = hi1 / nsub, c2lo = lo2 / nsub, c2hi = hi2 / nsub;
        const int nc1 = c1hi - c1lo + 1, nc = nc1 * (c2hi - c2lo + 1);
        const int w1 = hi1 - lo1 + 1, w2 = hi2 - lo2 + 1, ns = w1 * w2 * lo.nloc;
        // support functions: weight, leaf slot, index within the leaf
        double *lt = sh;
        int *lc = (int *)(lt + ns), *lf = lc + ns;
        int *bt = lf + ns;  // per leaf-slot pair: stored block, -2 - block when transposed, -1 when not near
        for (int k = threadIdx.x; k < ns; k += blockDim.x) {
            const int r = k % lo.nloc, e = k / lo.nloc;
            const int e1 = lo1 + e % w1, e2 = lo2 + e / w1, ra = r % P1, rb = r / P1;
            lt[k] = A.Tb[(e1 * P1 + ra) * P1 + (j1 - e1)] * A.Tb[(e2 * P1 + rb) * P1 + (j2 - e2)];
            lc[k] = (e2 / nsub - c2lo) * nc1 + (e1 / nsub - c1lo);
            lf[k] = ((e2 % nsub) * nsub + e1 % nsub) * lo.nloc + r;
        }
        for (int c = threadIdx.x; c < nc * nc; c += blockDim.x) {
            const int ca = c / nc, cb = c % nc;
            const int ida = patch * n * n + (c2lo + ca / nc1) * n + c1lo + ca % nc1;
            const int idb = patch * n * n + (c2lo + cb / nc1) * n + c1lo + cb % nc1;
            int code = -1;
            const int64_t k = csr_find(A.near_ptr, A.near_src, ida, idb);
            if (k >= 0) {
                const int64_t kb = A.sb[k];
                if (kb >= 0) {
                    code = (int)kb;
                } else {
                    const int64_t km = csr_find(A.near_ptr, A.near_src, idb, ida);
                    if (km >= 0 && A.sb[km] >= 0) code = -2 - (int)A.sb[km];
                }
            }
            bt[c] = code;
        }
        __syncthreads();
        for (int w = threadIdx.x; w < ns * ns; w += blockDim.x) {
            const int ia = w % ns, ib = w / ns;
            const double t = lt[ia] * lt[ib];
            const int code = bt[lc[ia] * nc + lc[ib]];
            if (t == 0.0 || code == -1) continue;
            const int fa = lf[ia], fb = lf[ib];
            if (code >= 0) acc += nearb[(int64_t)code * lo.nl * A.ld + (int64_t)fb * A.ld + fa] * t;
            else acc += nearb[(int64_t)(-2 - code) * lo.nl * A.ld + (int64_t)fa * A.ld + fb] * t;
        }
    }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) D[i] = red[0];
}

// ===========================================================================
// kernels: Krylov helpers
// ===========================================================================

// partial sums of conj(a) . b per block
template <class T>
__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                                                     T *__restrict__ part)
{
    __shared__ T red[256];
    T s = zero<T>();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += conj_(a[i]) * b[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <class T>
__global__ void k_reduce_to(int nparts, const T *__restrict__ part, T *__restrict__ out)
{
    __shared__ T red[256];
    T s = zero<T>();
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// CG (real), Jacobi preconditioned: scal = [rz (even steps), -, rz (odd steps),
// rr, done, threshold]; done (1.0) is set by the direction kernel once rr <=
// threshold and turns every later step into a no-op, so the host may test
// convergence one step behind the device.

// Sum of the first np entries of part, in a fixed order (every block that
// calls it gets the same value).  Needs a __syncthreads-safe call site.
__device__ inline double block_sum_parts(const double *__restrict__ part, int np, double *red)
{
    double v0 = 0.0;
    for (int k = threadIdx.x; k < np; k += blockDim.x) v0 += part[k];
    red[threadIdx.x] = v0;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double v = red[0];
    __syncthreads();
    return v;
}

// CG step (real, Jacobi): alpha = rz / (p . Ap) with p . Ap summed from the np
// partials of the product; w += alpha p, r -= alpha Ap, z = r / D; per-block
// partials of r . z and r . r into part2[blockIdx] and part2[256 + blockIdx].
// Nothing happens once *done is set.  256 threads, at most 256 blocks.
__global__ void __launch_bounds__(256) k_cg_step(int64_t n, const double *__restrict__ rz_old,
                                                 const double *__restrict__ pap_part, int np, double *__restrict__ w,
                                                 double *__restrict__ r, const double *__restrict__ p,
                                                 const double *__restrict__ Ap, const double *__restrict__ D,
                                                 double *__restrict__ z, double *__restrict__ part2,
                                                 const double *__restrict__ done)
{
    __shared__ double red[256];
    if (*done != 0.0) return;  // uniform: the whole grid returns
    const double alpha = *rz_old / block_sum_parts(pap_part, np, red);
    double rzs = 0.0, rrs = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        w[i] += alpha * p[i];
        const double ri = r[i] - alpha * Ap[i];
        r[i] = ri;
        const double zi = ri / D[i];
        z[i] = zi;
        rzs += ri * zi;
        rrs += ri * ri;
    }
    red[threadIdx.x] = rzs;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part2[blockIdx.x] = red[0];
    __syncthreads();
    red[threadIdx.x] = rrs;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part2[256 + blockIdx.x] = red[0];
}

// CG direction: rz_new, rr from the np partials of k_cg_step; p = z + (rz_new /
// rz_old) p; block 0 stores rz_new, rr and done = (rr <= *thr) (the next step
// reads rz_new as its rz_old), and (rr, done) also into host_out (device view
// of pinned host memory) when given.  After a skipped step the partials are
// those of the last real one, so the stored values do not change.
__global__ void __launch_bounds__(256) k_cg_dir(int64_t n, const double *__restrict__ part2, int np,
                                                const double *__restrict__ rz_old, double *__restrict__ rz_new,
                                                double *__restrict__ rr, double *__restrict__ p,
                                                const double *__restrict__ z, const double *__restrict__ thr,
                                                double *__restrict__ done, double *__restrict__ host_out)
{
    __shared__ double red[256];
    const double rzn = block_sum_parts(part2, np, red);
    const double rrn = block_sum_parts(part2 + 256, np, red);
    const double beta = rzn / *rz_old;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double dn = rrn <= *thr ? 1.0 : 0.0;
        *rz_new = rzn;
        *rr = rrn;
        *done = dn;
        if (host_out) {  // pinned host memory: (rr, done) of this step
            host_out[0] = rrn;
            host_out[1] = dn;
        }
    }
}

__global__ void k_set2(double *a, double va, double *b, double vb)
{
    *a = va;
    *b = vb;
}

template <class T>
__global__ void k_axpby(int64_t n, T alpha, const T *__restrict__ x, T beta, T *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = alpha * x[i] + beta * y[i];
}

template <class T>
__global__ void k_div(int64_t n, const T *__restrict__ x, const T *__restrict__ D, T *__restrict__ y);

template <>
__global__ void k_div<double>(int64_t n, const double *__restrict__ x, const double *__restrict__ D, double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] / D[i];
}

template <>
__global__ void k_div<cd>(int64_t n, const cd *__restrict__ x, const cd *__restrict__ D, cd *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cd d = D[i];
        double den = d.re * d.re + d.im * d.im;
        cd a = x[i];
        y[i] = {(a.re * d.re + a.im * d.im) / den, (a.im * d.re - a.re * d.im) / den};
    }
}

// GMRES: h[j] = <v_j, w> for j < k (classical Gram-Schmidt pass), partial per
// block: block (b, c) takes rows b*256 + u + m*nblk*256 (u < 256), its wave q
// the vectors j = 4c + q, 4c + q + 4 gridDim.y, ..., reduced with cross-lane
// shuffles, so no barrier is needed; part[j*nblk + b].

template <class T>
__global__ void __launch_bounds__(256) k_multidot_partial(int64_t n, int k, const T *__restrict__ V, int64_t ldv,
                                                          const T *__restrict__ w, T *__restrict__ part, int nblk)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t stride = (int64_t)nblk * 256;
    T wl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t i = (int64_t)blockIdx.x * 256 + lane + 64 * t;
        wl[t] = i < n ? w[i] : zero<T>();
    }
    for (int j = (int)blockIdx.y * 4 + wave; j < k; j += 4 * (int)gridDim.y) {
        const T *v = V + (int64_t)j * ldv;
        T s = zero<T>();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t i = (int64_t)blockIdx.x * 256 + lane + 64 * t;
            if (i < n) s += conj_(v[i]) * wl[t];
        }
        for (int64_t r0 = (int64_t)blockIdx.x * 256 + stride; r0 < n; r0 += stride)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = r0 + lane + 64 * t;
                if (i < n) s += conj_(v[i]) * w[i];
            }
        s = wave_sum64(s);
        if (lane == 0) part[(int64_t)j * nblk + blockIdx.x] = s;
    }
}

static int multidot_blocks(int64_t n) { return (int)std::min<int64_t>(64, (n + 255) / 256); }

// w -= V h for the first k columns, with h[j] = sum_b part[j*nblk + b] (b in
// order) formed by every block in LDS (block 0 also stores h to hout); with
// nrm, each block also writes its partial sum of |w_new|^2 to nrm[block].
template <class T>
__global__ void __launch_bounds__(256) k_sub_Vh_red(int64_t n, int k, const T *__restrict__ V, int64_t ldv,
                                                    const T *__restrict__ part, int nblk, T *__restrict__ hout,
                                                    T *__restrict__ w, double *__restrict__ nrm)
{
    extern __shared__ double shd[];
    __shared__ double wred[4];
    T *h = (T *)shd;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        T s = zero<T>();
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)j * nblk + b];
        h[j] = s;
        if (blockIdx.x == 0) hout[j] = s;
    }
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        T s = w[i];
        int j = 0;
        for (; j + 8 <= k; j += 8) {  // eight independent loads in flight
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(j + u) * ldv + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s -= h[j + u] * v[u];
        }
        for (; j < k; ++j) s -= h[j] * V[(int64_t)j * ldv + i];
        w[i] = s;
        acc += abs2(s);
    }
    if (nrm) {
        acc = wave_sum64(acc);
        if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) nrm[blockIdx.x] = (wred[0] + wred[1]) + (wred[2] + wred[3]);
    }
}

template <class T>
__global__ void k_multireduce(int k, int nblk, const T *__restrict__ part, T *__restrict__ h)
{
    int j = blockIdx.x;
    __shared__ T red[256];
    T s = zero<T>();
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[(int64_t)j * nblk + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int q = blockDim.x / 2; q > 0; q >>= 1) {
        if ((int)threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[j] = red[0];
}

// w -= V h (first k columns), eight columns' loads in flight per thread
template <class T>
__global__ void k_sub_Vh(int64_t n, int k, const T *__restrict__ V, int64_t ldv, const T *__restrict__ h, T *__restrict__ w)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        T s = w[i];
        int j = 0;
        for (; j + 8 <= k; j += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(j + u) * ldv + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s -= h[j + u] * v[u];
        }
        for (; j < k; ++j) s -= h[j] * V[(int64_t)j * ldv + i];
        w[i] = s;
    }
}

// ===========================================================================
// operator object
// ===========================================================================

// ---------------------------------------------------------------------------
// device memory pool
// ---------------------------------------------------------------------------
// Process-wide, per device: buffers given back by destroyed operators (and the
// scratch of potentials and exports) stay in free lists by size class and go
// to later requests of the same class, so an application that creates
// operators again and again calls hipMalloc / hipFree only the first time.
// igb_release_cached_memory frees what is cached; an allocation that fails for
// lack of memory releases the cache and tries once more.  A buffer is given
// back only after its operator's stream has drained.
struct DevBlock {
    void *p = nullptr;
    size_t bytes = 0;  // size class actually allocated
    int dev = 0;
};

namespace {
struct DevPool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> lists;
};
DevPool &dev_pool()
{
    static DevPool *p = new DevPool();  // lives until the process ends
    return *p;
}
size_t pool_class(size_t b)
{
    const size_t big = (size_t)2 << 20;
    return b <= big ? (b + 4095) / 4096 * 4096 : (b + big - 1) / big * big;
}
}  // namespace

static hipError_t pool_release_all()
{
    DevPool &P = dev_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    bool any = false;
    for (auto &kv : P.lists) any = any || !kv.second.empty();
    if (!any) return hipSuccess;
    int cur = 0;
    const hipError_t ecur = hipGetDevice(&cur);
    hipError_t res = hipSuccess;
    for (auto &kv : P.lists) {
        if (kv.second.empty()) continue;
        hipError_t e = hipSetDevice(kv.first.first);
        for (void *q : kv.second)
            if (e == hipSuccess) e = hipFree(q);
        if (e != hipSuccess) res = e;
        kv.second.clear();
    }
    if (ecur == hipSuccess) (void)hipSetDevice(cur);
    return res;
}

static hipError_t pool_alloc(DevBlock &b, size_t bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t c = pool_class(bytes == 0 ? 8 : bytes);
    {
        DevPool &P = dev_pool();
        std::lock_guard<std::mutex> lk(P.mu);
        auto it = P.lists.find({dev, c});
        if (it != P.lists.end() && !it->second.empty()) {
            b.p = it->second.back();
            b.bytes = c;
            b.dev = dev;
            it->second.pop_back();
            return hipSuccess;
        }
    }
    void *q = nullptr;
    e = hipMalloc(&q, c);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        (void)pool_release_all();
        e = hipMalloc(&q, c);
    }
    if (e != hipSuccess) return e;
    b.p = q;
    b.bytes = c;
    b.dev = dev;
    return hipSuccess;
}

static void pool_free(DevBlock &b)
{
    if (!b.p) return;
    DevPool &P = dev_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    P.lists[{b.dev, b.bytes}].push_back(b.p);
    b = DevBlock{};
}

struct igb_operator {
    Setup s;
    hipStream_t st = nullptr;
    bool cplx = false;
    size_t esz = 8;
    int ncu = 256;  // compute units of the device (grid size of the persistent far-field launches)
    Layout lo{};
    int lmin = 0;  // coarsest level with far blocks (L+1 if none)
    // device data
    double *tiles = nullptr;
    double *tline = nullptr;   // line-contraction tiles: [0] tile, [1] transpose (see tile_fix)
    int32_t *tdeg = nullptr;
    double *gx = nullptr, *gw = nullptr;
    double *btab = nullptr;        // per order n: n*(p+1) Bernstein values, offset goff[n]*(p+1)
    double *gpts[3] = {nullptr, nullptr, nullptr};
    int gord[3] = {0, 0, 0};
    double *rpts = nullptr;        // rhs/potential order geometry
    double *nodes = nullptr;
    double *sctab = nullptr;       // sin, cos (j pi/128), j < 256, for the complex far field
    hipEvent_t qev[6] = {};        // around the identical, adjacent and regular pair quadrature
    double quad_ms[2] = {0.0, 0.0};  // regular, touching (identical + adjacent) pair quadrature
    double *zdev = nullptr;        // Chebyshev nodes
    int64_t *cl_off = nullptr;
    double *M1 = nullptr, *E2 = nullptr, *Mlev = nullptr, *Tb = nullptr;
    int64_t *Mlev_off = nullptr;
    int64_t *near_ptr = nullptr;
    int32_t *near_src = nullptr;
    void *nearb = nullptr;
    // near-field storage (see near_layout): stored block of every CSR entry,
    // (t, s) of every stored block, partial-row index of every entry, partial rows
    bool near_sym = false;
    int near_ld = 0;
    int64_t nsb = 0;
    int32_t *sb = nullptr, *sb_t = nullptr, *sb_s = nullptr, *near_pidx = nullptr;
    void *npart = nullptr;
    std::vector<int32_t> sb_host;
    int64_t *far_ptr = nullptr;
    int32_t *far_src = nullptr, *far_tgt = nullptr;
    void *coup = nullptr;
    // on-the-fly far field by mirrored block pairs (q^2 <= 64): the pairs t < s,
    // the partial-row index of every CSR far entry, the partial rows
    int64_t nup = 0;
    int32_t *up_t = nullptr, *up_s = nullptr, *far_pidx = nullptr;
    void *fpart = nullptr;
    void *xs = nullptr, *ys = nullptr, *Xh = nullptr, *Yh = nullptr, *ext = nullptr;
    void *diag = nullptr;
    // solver work
    void *r = nullptr, *z = nullptr, *pv = nullptr, *Ap = nullptr, *tmp = nullptr;
    void *part = nullptr;
    void *dpart = nullptr;     // CG: per-block partials of p . Ap (one per block of the last T pass)
    double *scal = nullptr;
    double *h_scal = nullptr;  // pinned
    void *V = nullptr;         // GMRES basis (Vcols columns of ndof)
    int Vcols = 0;
    void *hdev = nullptr;      // GMRES projection coefficients
    void *mpart = nullptr;     // GMRES multi-dot partial sums
    void *potc = nullptr;      // potential: weighted density at the quadrature points
    double *clgeo = nullptr;   // H2 potential: cluster bounds (5 per global cluster) and a flag word
    void *tz = nullptr;        // intermediate of the separable T application
    // staged touching-pair blocks (nloc^2 per pair, row-major): identical pairs (E, E) in
    // element order, and the common-edge / common-vertex pairs in (E, F) order
    void *pairbuf_id = nullptr, *pairbuf = nullptr;
    std::vector<PairRec> touch_id, touch;  // host copies of the staged pairs
    int64_t near_bytes = 0, coup_bytes = 0;
    double assembly_seconds = 0.0;
    std::vector<DevBlock> owned;
    DevBlock Vblk{}, hblk{}, mblk{};  // GMRES basis, projections, multi-dot partials
    DevBlock Zblk{};                  // flexible GMRES: preconditioned directions
    DevBlock Gblk{};                  // flexible GMRES: Hessenberg matrix, rotations, state
    int Zcols = 0;
    // far_precision IGB_FP32: products use single-precision far-field kernel values;
    // force_fp64 is set while the solver forms its double-precision residuals
    bool far_single = false, force_fp64 = false;
    void *rr = nullptr, *dw = nullptr;  // refinement: residual and correction (IGB_FP32)
    // side stream of the product: the near-field block GEMV (HBM-bound) runs there, overlapping the tree
    // passes and the on-the-fly far field (ALU-bound) on st; forked and joined with the two events
    hipStream_t st2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // single-precision Helmholtz far field: the stored near blocks rounded to FP32 as well, for the
    // products of the inner solves (the FP64 residual products use nearb)
    void *nearb32 = nullptr;
    int dev = 0;  // the device current at igb_operator_create
};

static igb_status dalloc(igb_operator *op, void **p, size_t bytes)
{
    DevBlock b{};
    hipError_t e = pool_alloc(b, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? IGB_ENOMEM : IGB_EHIP,
                    "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    }
    *p = b.p;
    op->owned.push_back(b);
    return IGB_OK;
}

template <class P>
static igb_status upload(igb_operator *op, P **dst, const void *src, size_t bytes)
{
    igb_status s = dalloc(op, (void **)dst, bytes);
    if (s) return s;
    if (bytes) HIPCHK(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, op->st));
    return IGB_OK;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Near-field storage: symmetric (blocks t <= s only, column stride nl rounded up
// to 8) when a wave's staging of k_near_sym fits 48 KB of LDS, else every
// block (t, s) of the CSR list with column stride nl.
struct NearLayout {
    bool sym;
    int ld;
    int64_t nsb;
};
static NearLayout near_layout(const Setup &s, size_t esz)
{
    NearLayout L;
    int ld8 = (s.nl + 7) & ~7;
    L.sym = (size_t)(8 * ld8 + 520) * esz <= 48 * 1024;
    L.ld = L.sym ? ld8 : s.nl;
    L.nsb = 0;
    if (L.sym) {
        for (int64_t t = 0; t < (int64_t)s.near_ptr.size() - 1; ++t)
            for (int64_t e = s.near_ptr[t]; e < s.near_ptr[t + 1]; ++e) L.nsb += s.near_src[e] >= t;
    } else {
        L.nsb = (int64_t)s.near_src.size();
    }
    return L;
}

// With both products symmetric, the near blocks ride along in the far-field
// launch (and both gathers share one launch) when four waves' near staging fits
// 64 KB of LDS.
static bool fused_products(bool near_sym, int nl, int near_ld, size_t esz, int q2)
{
    return near_sym && (q2 <= 64 || (esz == sizeof(cd) && q2 <= 104)) &&
           4 * (size_t)near_sym_lds(nl, near_ld) * esz <= 64 * 1024;
}

// Far field evaluated once per mirrored pair of blocks (on the fly; q^2 <= 64 for
// the real kernel, q^2 <= 104 for the complex one).
static bool far_mirrored(const Setup &s)
{
    // real kernel up to 64 nodes per cluster, complex up to 104 (13 per lane)
    return s.mode == IGB_H2_ONTHEFLY && !s.far_src.empty() &&
           (s.q * s.q <= 64 || (s.kernel == IGB_HELMHOLTZ && s.q * s.q <= 104));
}

static int64_t csr_find_host(const Setup &s, int t, int src)
{
    auto b = s.near_src.begin() + s.near_ptr[t], e = s.near_src.begin() + s.near_ptr[t + 1];
    auto it = std::lower_bound(b, e, src);
    return (it == e || *it != src) ? -1 : (int64_t)(it - s.near_src.begin());
}

// ---------------------------------------------------------------------------
// template launchers
// ---------------------------------------------------------------------------
template <class T, int P>
static igb_status launch_regular_p(igb_operator *op, const PairRec *d_pairs, int64_t n, int g, const double *gp)
{
    int gg = g * g, NLOC = (P + 1) * (P + 1);
    size_t shm =
        (size_t)gg * 8 * sizeof(double) + (size_t)gg * NLOC * sizeof(double) + (size_t)gg * (NLOC + 1) * sizeof(T);
    if (shm > 160 * 1024) return fail(IGB_EUNSUPPORTED, "regular quadrature order too large for LDS");
    (void)hipFuncSetAttribute((const void *)k_near_regular<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    const int threads = gg <= 64 ? 64 : 128;  // one quadrature point of E per thread in the first phase
    for (int64_t off = 0; off < n; off += 1 << 20) {
        int64_t cnt = std::min<int64_t>(n - off, 1 << 20);
        hipLaunchKernelGGL((k_near_regular<T, P>), dim3((unsigned)cnt), dim3(threads), shm, op->st, d_pairs + off, (int)cnt, g,
                           gp, op->btab + (size_t)op->s.goff[g] * (P + 1), op->s.kappa, op->s.nl, op->near_ld, op->sb,
                           (T *)op->nearb, (const double *)op->sctab);
        LAUNCHCHK();
    }
    return IGB_OK;
}

template <class T, int P, int PG>
static igb_status launch_singular_pg(igb_operator *op, const PairRec *d_pairs, int64_t n, void *outbuf, bool vertex)
{
    constexpr int NLOC = (P + 1) * (P + 1), NPAD = 16 * ((NLOC + 15) / 16), NC = NComp<T>::value;
    constexpr int STAGE_BYTES = (32 * (NC + 1) * (NPAD + 1) + 8) * 8;
    constexpr int WAVES = 4;
    // the final reduction reuses the stage: it needs WAVES * NC * NPAD^2 doubles
    constexpr size_t RED_BYTES = (size_t)WAVES * NC * NPAD * NPAD * 8;
    size_t stage = std::max<size_t>((size_t)WAVES * STAGE_BYTES, RED_BYTES);
    size_t shm = (size_t)128 * sizeof(double) + stage;
    if (shm > 160 * 1024) return fail(IGB_EUNSUPPORTED, "touching-pair quadrature: LDS too small for this degree");
    const int gs = op->s.gs;
    // identical and common-edge pairs, then (vertex) the common-vertex pairs of the same list
    auto go = [&](auto vtx) -> igb_status {
        constexpr bool V = decltype(vtx)::value;
        (void)hipFuncSetAttribute((const void *)k_near_singular<T, P, PG, WAVES, V>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        for (int64_t off = 0; off < n; off += 1 << 20) {
            int64_t cnt = std::min<int64_t>(n - off, 1 << 20);
            hipLaunchKernelGGL((k_near_singular<T, P, PG, WAVES, V>), dim3((unsigned)cnt), dim3(64 * WAVES), shm,
                               op->st, d_pairs + off, gs, op->gx + op->s.goff[gs], op->gw + op->s.goff[gs], op->tline,
                               op->tline + (size_t)op->s.nelem * op->s.tile_stride, op->s.kappa,
                               (T *)outbuf + off * NLOC * NLOC, (const double *)op->sctab);
            LAUNCHCHK();
        }
        return IGB_OK;
    };
    igb_status rc = go(std::false_type{});
    if (rc == IGB_OK && vertex) rc = go(std::true_type{});
    return rc;
}

template <class T, int P>
static igb_status launch_singular_p(igb_operator *op, const PairRec *d_pairs, int64_t n, void *outbuf, bool vertex)
{
    switch (op->s.tile_degree) {
    case 1: return launch_singular_pg<T, P, 1>(op, d_pairs, n, outbuf, vertex);
    case 2: return launch_singular_pg<T, P, 2>(op, d_pairs, n, outbuf, vertex);
    case 4: return launch_singular_pg<T, P, 4>(op, d_pairs, n, outbuf, vertex);
    case 8: return launch_singular_pg<T, P, 8>(op, d_pairs, n, outbuf, vertex);
    }
    return fail(IGB_EUNSUPPORTED, "tile degree");
}

template <class T>
static igb_status launch_regular(igb_operator *op, const PairRec *d, int64_t n, int g, const double *gp)
{
    switch (op->s.p) {
    case 0: return launch_regular_p<T, 0>(op, d, n, g, gp);
    case 1: return launch_regular_p<T, 1>(op, d, n, g, gp);
    case 2: return launch_regular_p<T, 2>(op, d, n, g, gp);
    case 3: return launch_regular_p<T, 3>(op, d, n, g, gp);
    case 4: return launch_regular_p<T, 4>(op, d, n, g, gp);
    case 5: return launch_regular_p<T, 5>(op, d, n, g, gp);
    case 6: return launch_regular_p<T, 6>(op, d, n, g, gp);
    }
    return fail(IGB_EUNSUPPORTED, "p > 6");
}

template <class T>
static igb_status launch_singular(igb_operator *op, const PairRec *d, int64_t n, void *outbuf, bool vertex)
{
    switch (op->s.p) {
    case 0: return launch_singular_p<T, 0>(op, d, n, outbuf, vertex);
    case 1: return launch_singular_p<T, 1>(op, d, n, outbuf, vertex);
    case 2: return launch_singular_p<T, 2>(op, d, n, outbuf, vertex);
    case 3: return launch_singular_p<T, 3>(op, d, n, outbuf, vertex);
    case 4: return launch_singular_p<T, 4>(op, d, n, outbuf, vertex);
    case 5: return launch_singular_p<T, 5>(op, d, n, outbuf, vertex);
    case 6: return launch_singular_p<T, 6>(op, d, n, outbuf, vertex);
    }
    return fail(IGB_EUNSUPPORTED, "p > 6");
}

// superspace matvec on internal vectors: ys = A xs.  When ev is given, ev[k]
// is recorded on the operator's stream before stage k and ev[6] at the end:
// stages 0 upward (leaf moments and transfers), 1 coupling blocks, 2 coupling
// gather (on the fly by mirrored pairs only), 3 near GEMV, 4 near gather
// (symmetric near storage only), 5 downward (transfers and leaf back-moments).
static FarSymArgs far_args(const igb_operator *op)
{
    return FarSymArgs{op->nup, op->up_t, op->up_s, op->s.q * op->s.q, op->nodes, op->s.kappa, op->sctab};
}
static NearSymArgs near_args(const igb_operator *op)
{
    return NearSymArgs{op->nsb, op->sb_t, op->sb_s, op->s.nl, op->near_ld};
}

// far pairs alone, or (fuse) far pairs and stored near blocks in one launch;
// RAW: single-precision kernel values (far_precision IGB_FP32)
template <class T, int TT, bool RAW>
static void launch_far_sym_p(igb_operator *op, const T *Xh, const T *xs, bool fuse)
{
    // far pairs and near blocks in one launch (with_near false: the far pairs alone); the single-precision
    // complex product reads the FP32 copy of the near blocks when there is one
    auto fused = [&](bool with_near) {
        const int64_t nf = (op->nup + 4 * kFarChunk - 1) / (4 * kFarChunk), nn = with_near ? (op->nsb + 3) / 4 : 0;
        const size_t shm = 4 *
                           std::max<size_t>((size_t)near_sym_lds(op->s.nl, op->near_ld) * NComp<T>::value,
                                            (size_t)far_sym_lds<T, TT>()) * 8;
        if constexpr (NComp<T>::value == 2 && RAW) {
            if (op->nearb32) {
                hipLaunchKernelGGL((k_sym_products<T, TT, RAW, cf>), dim3((unsigned)(nf + nn)), dim3(256), shm, op->st,
                                   far_args(op), near_args(op), nf, nn, Xh, (T *)op->fpart, (const cf *)op->nearb32, xs,
                                   (T *)op->npart);
                return;
            }
        }
        hipLaunchKernelGGL((k_sym_products<T, TT, RAW>), dim3((unsigned)(nf + nn)), dim3(256), shm, op->st, far_args(op),
                           near_args(op), nf, nn, Xh, (T *)op->fpart, (const T *)op->nearb, xs, (T *)op->npart);
    };
    if (TT > 8 || fuse) {
        fused(fuse);
        return;
    }
    hipLaunchKernelGGL((k_far_sym<T, TT, RAW>), dim3((unsigned)((op->nup + 4 * kFarChunk - 1) / (4 * kFarChunk))),
                       dim3(256), 0, op->st, far_args(op), Xh, (T *)op->fpart);
}

template <class T, int TT>
static void launch_far_sym(igb_operator *op, const T *Xh, const T *xs, bool fuse)
{
    static_assert(TT <= 8 || NComp<T>::value == 2, "more than 64 nodes per cluster: complex kernel only");
    if (op->far_single && !op->force_fp64) {
        launch_far_sym_p<T, TT, true>(op, Xh, xs, fuse);
        return;
    }
    launch_far_sym_p<T, TT, false>(op, Xh, xs, fuse);
}

// Slices of the cluster tree for k_up_tree / k_down_tree: (ls, lb) pairs from
// the leaves up, lb - ls <= 2, ending at the coarsest far-field level.
struct TreeLaunch {
    TreeArgs A;
    int SL, waves;
    unsigned roots;
    size_t shm;
};
static std::vector<TreeLaunch> tree_slices(const igb_operator *op, size_t esz)
{
    const Setup &s = op->s;
    std::vector<TreeLaunch> v;
    const int q2 = s.q * s.q;
    const int SL = std::max({s.n1 * s.n1 + s.n1 * s.q, 2 * q2, q2 + s.q * s.n1});
    const int waves = (int)std::max<size_t>(1, std::min<size_t>(16, (48 * 1024) / ((size_t)SL * esz)));
    int lb = s.L;
    do {
        TreeLaunch t;
        const int ls = std::max(op->lmin, lb - 2);
        t.A = TreeArgs{ls, lb, s.L, s.q, s.n1, s.side, s.p + 1, s.nloc, s.nl, op->M1, op->E2, op->cl_off};
        t.SL = SL;
        t.waves = waves;
        t.roots = (unsigned)(s.npatch << (2 * ls));
        // slices + child slots of <= 4 parents + the staged M1 and E2
        t.shm = ((size_t)waves * SL + (size_t)16 * q2) * esz + (size_t)(s.n1 * s.q + 2 * q2) * sizeof(double);
        v.push_back(t);
        lb = ls;
    } while (lb > op->lmin);
    return v;
}

// symmetric near storage: one wave per stored block (t, s), partial rows for both sides
template <class T>
static void launch_near_sym(igb_operator *op, const T *xs, hipStream_t st)
{
    if constexpr (NComp<T>::value == 2) {
        if (op->nearb32 && op->far_single && !op->force_fp64) {
            hipLaunchKernelGGL(k_near_sym32, dim3((unsigned)((op->nsb + 3) / 4)), dim3(256), 0, st, near_args(op),
                               (const cf *)op->nearb32, (const cd *)xs, (cd *)op->npart);
            return;
        }
    }
    const size_t wave_lds = (size_t)near_sym_lds(op->s.nl, op->near_ld) * sizeof(T);
    const int wpb = wave_lds ? (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / wave_lds)) : 4;
    hipLaunchKernelGGL((k_near_sym<T>), dim3((unsigned)((op->nsb + wpb - 1) / wpb)), dim3(64 * wpb), wpb * wave_lds,
                       st, near_args(op), (const T *)op->nearb, xs, (T *)op->npart);
}

// ev (optional): IGB_NUM_MATVEC_STAGES + 1 events recorded on st between the stages; evn (optional): two
// events recorded on the side stream around the forked near-field GEMV, forked (optional) tells whether
// the GEMV was forked.
template <class T>
static igb_status matvec_internal(igb_operator *op, const T *xs, T *ys, hipEvent_t *ev = nullptr,
                                  bool separate = false, hipEvent_t *evn = nullptr, bool *forked = nullptr)
{
    const Setup &s = op->s;
    int q = s.q, q2 = q * q;
    T *Xh = (T *)op->Xh, *Yh = (T *)op->Yh;
    bool has_far = op->lmin <= s.L;
    auto mark = [&](int k) -> igb_status {
        if (ev) HIPCHK(hipEventRecord(ev[k], op->st));
        return IGB_OK;
    };
    igb_status rc;
    const std::vector<TreeLaunch> TS = has_far ? tree_slices(op, sizeof(T)) : std::vector<TreeLaunch>();
    if ((rc = mark(0))) return rc;
    for (const TreeLaunch &t : TS) {
        if (t.shm > 64 * 1024) {
            if (t.shm > 160 * 1024) return fail(IGB_EUNSUPPORTED, "cluster-tree transfers: q too large for LDS");
            (void)hipFuncSetAttribute((const void *)k_up_tree<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)t.shm);
            (void)hipFuncSetAttribute((const void *)k_down_tree<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)t.shm);
        }
        hipLaunchKernelGGL((k_up_tree<T>), dim3(t.roots), dim3(64 * t.waves), t.shm, op->st, t.A, t.SL, xs, Xh);
        LAUNCHCHK();
    }
    if ((rc = mark(1))) return rc;
    int64_t row0 = s.cl_off[op->lmin], nrows = s.cl_off[s.L + 1] - row0;
    const bool sym = has_far && op->fpart != nullptr;
    const bool fuse = sym && !separate && fused_products(op->near_sym, s.nl, op->near_ld, sizeof(T), q2);
    // near blocks not fused into the far-field launch: their GEMV reads only xs, so it runs on the side
    // stream from the start of the product and is joined before its gather
    const bool fork = has_far && op->near_sym && !fuse && !separate;
    if (forked) *forked = fork;
    if (fork) {
        if (!op->st2) {
            HIPCHK(hipStreamCreateWithFlags(&op->st2, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(op->ev_fork, op->st));
        HIPCHK(hipStreamWaitEvent(op->st2, op->ev_fork, 0));
        if (evn) HIPCHK(hipEventRecord(evn[0], op->st2));
        launch_near_sym<T>(op, xs, op->st2);
        if (evn) HIPCHK(hipEventRecord(evn[1], op->st2));
        HIPCHK(hipEventRecord(op->ev_join, op->st2));
    }
    if (has_far) {
        if (sym) {
            switch ((q2 + 7) / 8) {
            case 1: launch_far_sym<T, 1>(op, Xh, xs, fuse); break;
            case 2: launch_far_sym<T, 2>(op, Xh, xs, fuse); break;
            case 3: launch_far_sym<T, 3>(op, Xh, xs, fuse); break;
            case 4: launch_far_sym<T, 4>(op, Xh, xs, fuse); break;
            case 5: launch_far_sym<T, 5>(op, Xh, xs, fuse); break;
            case 6: launch_far_sym<T, 6>(op, Xh, xs, fuse); break;
            case 7: launch_far_sym<T, 7>(op, Xh, xs, fuse); break;
            case 8: launch_far_sym<T, 8>(op, Xh, xs, fuse); break;
            default:  // complex kernel, 65 .. 104 nodes per cluster
                if constexpr (NComp<T>::value == 2) {
                    switch ((q2 + 7) / 8) {
                    case 9: launch_far_sym<T, 9>(op, Xh, xs, fuse); break;
                    case 10: launch_far_sym<T, 10>(op, Xh, xs, fuse); break;
                    case 11: launch_far_sym<T, 11>(op, Xh, xs, fuse); break;
                    case 12: launch_far_sym<T, 12>(op, Xh, xs, fuse); break;
                    default: launch_far_sym<T, 13>(op, Xh, xs, fuse); break;
                    }
                } else {
                    return fail(IGB_EINVAL, "mirrored far field: more than 64 nodes per cluster");
                }
            }
        } else if (s.mode == IGB_H2_ONTHEFLY) {
            size_t shm = (size_t)4 * q2 * (3 + NComp<T>::value) * sizeof(double) + (size_t)4 * q2 * sizeof(T);
            hipLaunchKernelGGL((k_far_onthefly<T>), dim3((unsigned)nrows), dim3(256), shm, op->st, q2, op->far_ptr,
                               op->far_src, op->nodes, (const T *)Xh, s.kappa, Yh, row0);
        } else {
            hipLaunchKernelGGL((k_bsr_gemv<T, 1>), dim3((unsigned)nrows), dim3(256), 4 * q2 * sizeof(T), op->st, q2,
                               op->far_ptr, op->far_src, (const T *)op->coup, (const T *)Xh, Yh, row0);
        }
        LAUNCHCHK();
    }
    if ((rc = mark(2))) return rc;
    const GatherArgs GF{q2, q2, op->far_ptr, op->far_pidx, op->fpart, op->nodes + 3, 0.07957747154594767, Yh, row0};
    const GatherArgs GN{s.nl, op->near_ld, op->near_ptr, op->near_pidx, op->npart, nullptr, 1.0, ys, 0};
    if (fuse) {  // both gathers in one launch
        hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)(nrows + s.nleaf)), dim3(256),
                           4 * std::max(q2, s.nl) * sizeof(T), op->st, GF, GN, nrows);
        LAUNCHCHK();
    } else if (sym) {
        hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)nrows), dim3(256), 4 * q2 * sizeof(T), op->st, GF, GF, nrows);
        LAUNCHCHK();
    }
    if ((rc = mark(3))) return rc;
    if (fuse) {
        // done inside the far-field launch
    } else if (fork) {
        HIPCHK(hipStreamWaitEvent(op->st, op->ev_join, 0));
    } else if (op->near_sym) {
        launch_near_sym<T>(op, xs, op->st);
        LAUNCHCHK();
    } else {
        hipLaunchKernelGGL((k_bsr_gemv<T, 0>), dim3(s.nleaf), dim3(256), 4 * s.nl * sizeof(T), op->st, s.nl,
                           op->near_ptr, op->near_src, (const T *)op->nearb, xs, ys, (int64_t)0);
        LAUNCHCHK();
    }
    if ((rc = mark(4))) return rc;
    if (op->near_sym && !fuse) {
        hipLaunchKernelGGL((k_gather<T>), dim3(s.nleaf), dim3(256), 4 * s.nl * sizeof(T), op->st, GN, GN,
                           (int64_t)s.nleaf);
        LAUNCHCHK();
    }
    if ((rc = mark(5))) return rc;
    for (auto t = TS.rbegin(); t != TS.rend(); ++t) {
        hipLaunchKernelGGL((k_down_tree<T>), dim3(t->roots), dim3(64 * t->waves), t->shm, op->st, t->A, t->SL, Yh, ys);
        LAUNCHCHK();
    }
    return mark(6);
}

template <class T, int P>
static void launch_Tt_p(igb_operator *op, const T *w, T *xs)
{
    hipLaunchKernelGGL((k_Tt<T, P>), dim3(nblk(op->s.nsup, 256)), dim3(256), 0, op->st, op->lo, (int)op->s.nsup, op->Tb,
                       w, xs);
}

template <class T, int P>
static void launch_T_p(igb_operator *op, const T *ys, T *y, const T *dx, T *part)
{
    const int64_t nz = (int64_t)op->s.npatch * op->s.ne * (P + 1) * op->s.ns1;
    hipLaunchKernelGGL((k_T_pass1<T, P>), dim3(nblk(nz, 256)), dim3(256), 0, op->st, op->lo, op->s.npatch, op->Tb, ys,
                       (T *)op->tz);
    hipLaunchKernelGGL((k_T_pass2<T, P>), dim3(nblk(op->s.ndof, 256)), dim3(256), 0, op->st, op->lo, (int)op->s.ndof,
                       op->Tb, (const T *)op->tz, y, dx, part);
}

// The T kernels index with 32-bit integers: every superspace index must fit.
static igb_status t_sizes_ok(const igb_operator *op)
{
    if (op->s.nsup >= ((int64_t)1 << 31) ||
        (int64_t)op->s.npatch * op->s.ne * (op->s.p + 1) * op->s.ns1 >= ((int64_t)1 << 31))
        return fail(IGB_EUNSUPPORTED, "superspace dimension >= 2^31");
    return IGB_OK;
}

template <class T>
static igb_status apply_Tt(igb_operator *op, const T *w, T *xs)
{
    igb_status rc;
    if ((rc = t_sizes_ok(op))) return rc;
    switch (op->s.p) {
    case 0: launch_Tt_p<T, 0>(op, w, xs); break;
    case 1: launch_Tt_p<T, 1>(op, w, xs); break;
    case 2: launch_Tt_p<T, 2>(op, w, xs); break;
    case 3: launch_Tt_p<T, 3>(op, w, xs); break;
    case 4: launch_Tt_p<T, 4>(op, w, xs); break;
    case 5: launch_Tt_p<T, 5>(op, w, xs); break;
    case 6: launch_Tt_p<T, 6>(op, w, xs); break;
    default: return fail(IGB_EUNSUPPORTED, "p > 6");
    }
    LAUNCHCHK();
    return IGB_OK;
}

// y = T ys; with dx given, also the per-block partial sums of conj(dx) . y
// into part (nblk(ndof, 256) entries).
template <class T>
static igb_status apply_T(igb_operator *op, const T *ys, T *y, const T *dx = nullptr, T *part = nullptr)
{
    igb_status rc;
    if ((rc = t_sizes_ok(op))) return rc;
    switch (op->s.p) {
    case 0: launch_T_p<T, 0>(op, ys, y, dx, part); break;
    case 1: launch_T_p<T, 1>(op, ys, y, dx, part); break;
    case 2: launch_T_p<T, 2>(op, ys, y, dx, part); break;
    case 3: launch_T_p<T, 3>(op, ys, y, dx, part); break;
    case 4: launch_T_p<T, 4>(op, ys, y, dx, part); break;
    case 5: launch_T_p<T, 5>(op, ys, y, dx, part); break;
    case 6: launch_T_p<T, 6>(op, ys, y, dx, part); break;
    default: return fail(IGB_EUNSUPPORTED, "p > 6");
    }
    LAUNCHCHK();
    return IGB_OK;
}

// y = A x in the spline space; with part given, also the per-block partial
// sums of conj(x) . y (nblk(ndof, 256) entries).
template <class T>
static igb_status matvec_S(igb_operator *op, const T *x, T *y, T *part = nullptr)
{
    igb_status rc;
    if ((rc = apply_Tt<T>(op, x, (T *)op->xs))) return rc;
    if ((rc = matvec_internal<T>(op, (const T *)op->xs, (T *)op->ys))) return rc;
    return apply_T<T>(op, (const T *)op->ys, y, part ? x : nullptr, part);
}

static const int kRedBlocks = 256;

template <class T>
static igb_status dot_dev(igb_operator *op, int64_t n, const T *a, const T *b, T *out)
{
    hipLaunchKernelGGL((k_dot_partial<T>), dim3(kRedBlocks), dim3(256), 0, op->st, n, a, b, (T *)op->part);
    LAUNCHCHK();
    hipLaunchKernelGGL((k_reduce_to<T>), dim3(1), dim3(256), 0, op->st, kRedBlocks, (const T *)op->part, out);
    LAUNCHCHK();
    return IGB_OK;
}

// Assembly, first part (needs only the element tiles): Gauss-node geometry and
// the quadrature of the identical pairs (E, E), which are known without any
// search, into a staging buffer.  Runs on the GPU while the host computes the
// element geometry and looks for the other touching pairs.
template <class T>
static igb_status assemble_identical(igb_operator *op)
{
    Setup &s = op->s;
    igb_status rc;
    if (op->cplx) {
        // one period of sine and cosine at multiples of pi/128, from extended-precision host values (the
        // touching-pair quadrature, the far field and the potential read it)
        std::vector<double> tab(2 * kSinCosTab);
        for (int j = 0; j < kSinCosTab; ++j) {
            const long double a = (long double)j * 3.141592653589793238462643383279502884L / 128.0L;
            tab[2 * j] = (double)sinl(a);
            tab[2 * j + 1] = (double)cosl(a);
        }
        if ((rc = upload(op, &op->sctab, tab.data(), tab.size() * sizeof(double)))) return rc;
        HIPCHK(hipStreamSynchronize(op->st));  // the host table goes out of scope
    }
    int ords[3] = {s.g0, std::min(40, s.g0 + 2), std::min(40, s.g0 + 4)};
    for (int k = 0; k < 3; ++k) {
        op->gord[k] = ords[k];
        int g = ords[k];
        if ((rc = dalloc(op, (void **)&op->gpts[k], (size_t)s.nelem * g * g * 4 * sizeof(double)))) return rc;
        hipLaunchKernelGGL(k_gauss_geom, dim3(nblk((int64_t)s.nelem * g * g, 256)), dim3(256), 0, op->st, s.nelem,
                           s.tile_stride, op->tiles, op->tdeg, g, op->gx + s.goff[g], op->gw + s.goff[g], op->gpts[k]);
        LAUNCHCHK();
    }
    {
        int g = s.grhs;
        if ((rc = dalloc(op, (void **)&op->rpts, (size_t)s.nelem * g * g * 4 * sizeof(double)))) return rc;
        hipLaunchKernelGGL(k_gauss_geom, dim3(nblk((int64_t)s.nelem * g * g, 256)), dim3(256), 0, op->st, s.nelem,
                           s.tile_stride, op->tiles, op->tdeg, g, op->gx + s.goff[g], op->gw + s.goff[g], op->rpts);
        LAUNCHCHK();
    }
    std::vector<PairRec> &tid = op->touch_id;
    tid.assign(s.nelem, PairRec{});
    for (int E = 0; E < s.nelem; ++E) {  // same record as the plan's classification of (E, E)
        PairRec &R = tid[E];
        std::memset(&R, 0, sizeof R);
        R.E = R.F = E;
        R.cls = kIdentical;
        R.order = s.gs;
        R.oE = 0; R.aE = 1; R.bE = 3; R.oF = 0; R.aF = 1; R.bF = 3;
    }
    PairRec *d = nullptr;
    if ((rc = upload(op, &d, tid.data(), tid.size() * sizeof(PairRec)))) return rc;
    if ((rc = dalloc(op, &op->pairbuf_id, (size_t)s.nelem * s.nloc * s.nloc * sizeof(T)))) return rc;
    HIPCHK(hipEventRecord(op->qev[0], op->st));
    rc = launch_singular<T>(op, d, (int64_t)s.nelem, op->pairbuf_id, false);
    HIPCHK(hipEventRecord(op->qev[1], op->st));
    return rc;
}

// The common-edge and common-vertex pairs, found from corner coincidence of the
// element geometry (no partition needed), into their staging buffer.
template <class T>
static igb_status assemble_adjacent(igb_operator *op)
{
    Setup &s = op->s;
    igb_status rc;
    std::vector<PairRec> &touch = op->touch;
    std::string err = enumerate_touching(s, touch, false);
    if (!err.empty()) return fail(IGB_EINVAL, err);
    const int64_t n = (int64_t)touch.size();
    PairRec *d = nullptr;
    if ((rc = upload(op, &d, touch.data(), touch.size() * sizeof(PairRec)))) return rc;
    if ((rc = dalloc(op, &op->pairbuf, (size_t)n * s.nloc * s.nloc * sizeof(T)))) return rc;
    HIPCHK(hipEventRecord(op->qev[2], op->st));
    if (n > 0) rc = launch_singular<T>(op, d, n, op->pairbuf, true);
    HIPCHK(hipEventRecord(op->qev[3], op->st));
    return rc;
}

// Assembly, second part (needs the plan): near-field blocks (regular pairs by
// quadrature, touching pairs scattered from the staging buffer), cluster-node
// geometry, stored coupling blocks, Jacobi diagonal.
template <class T>
static igb_status assemble(igb_operator *op)
{
    Setup &s = op->s;
    igb_status rc;
    int q2 = s.q * s.q;
    const int *ords = op->gord;
    // the touching pairs of the plan must be exactly the ones quadrature already ran on
    // (and, sorted like them, they carry the near-block indices for the scatter)
    std::vector<PairRec> staged(op->touch_id.size() + op->touch.size()), touch, touch_id, touch_adj;
    auto by_ef = [](const PairRec &a, const PairRec &b) { return a.E < b.E || (a.E == b.E && a.F < b.F); };
    std::merge(op->touch_id.begin(), op->touch_id.end(), op->touch.begin(), op->touch.end(), staged.begin(), by_ef);
    std::string terr = check_touching(s, staged, &touch);
    if (!terr.empty()) return fail(IGB_EINVAL, terr);
    for (const PairRec &R : touch) (R.E == R.F ? touch_id : touch_adj).push_back(R);  // staging orders
    // near-field blocks: storage map, partial-row indices, zeroed storage
    {
        NearLayout NL = near_layout(s, sizeof(T));
        op->near_sym = NL.sym;
        op->near_ld = NL.ld;
        op->nsb = NL.nsb;
        int64_t nnear = (int64_t)s.near_src.size();
        std::vector<int32_t> &sbh = op->sb_host;
        sbh.assign(nnear, -1);
        if (NL.sym) {
            std::vector<int32_t> st, ss, pidx(nnear);
            for (int t = 0; t < s.nleaf; ++t)
                for (int64_t e = s.near_ptr[t]; e < s.near_ptr[t + 1]; ++e)
                    if (s.near_src[e] >= t) {
                        sbh[e] = (int32_t)st.size();
                        st.push_back(t);
                        ss.push_back(s.near_src[e]);
                    }
            for (int t = 0; t < s.nleaf; ++t)
                for (int64_t e = s.near_ptr[t]; e < s.near_ptr[t + 1]; ++e) {
                    int src = s.near_src[e];
                    if (src >= t) {
                        pidx[e] = 2 * sbh[e];
                        continue;
                    }
                    int64_t m = csr_find_host(s, src, t);
                    if (m < 0) return fail(IGB_EINVAL, "near-field partition is not symmetric");
                    pidx[e] = 2 * sbh[m] + 1;
                }
            if ((rc = upload(op, &op->sb_t, st.data(), st.size() * sizeof(int32_t)))) return rc;
            if ((rc = upload(op, &op->sb_s, ss.data(), ss.size() * sizeof(int32_t)))) return rc;
            if ((rc = upload(op, &op->near_pidx, pidx.data(), pidx.size() * sizeof(int32_t)))) return rc;
            if ((rc = dalloc(op, &op->npart, (size_t)2 * op->nsb * op->near_ld * sizeof(T)))) return rc;
        } else {
            for (int64_t e = 0; e < nnear; ++e) sbh[e] = (int32_t)e;
        }
        if ((rc = upload(op, &op->sb, sbh.data(), sbh.size() * sizeof(int32_t)))) return rc;
    }
    op->near_bytes = op->nsb * s.nl * op->near_ld * (int64_t)sizeof(T);
    if ((rc = dalloc(op, &op->nearb, op->near_bytes))) return rc;
    HIPCHK(hipMemsetAsync(op->nearb, 0, op->near_bytes, op->st));
    {
        // the plan keeps the regular pairs grouped by Gauss order (ords[k] is group k): one upload, one launch
        // per group
        const int64_t nreg = s.pair_off[3];
        PairRec *d = nullptr;
        if (nreg > 0 && (rc = upload(op, &d, s.pairs.data(), (size_t)nreg * sizeof(PairRec)))) return rc;
        HIPCHK(hipEventRecord(op->qev[4], op->st));
        for (int k = 0; k < 3; ++k) {
            const int64_t n = s.pair_off[k + 1] - s.pair_off[k];
            if (n == 0) continue;
            if ((rc = launch_regular<T>(op, d + s.pair_off[k], n, ords[k], op->gpts[k]))) return rc;
        }
        HIPCHK(hipEventRecord(op->qev[5], op->st));
        for (int part = 0; part < 2; ++part) {
            const std::vector<PairRec> &lst = part == 0 ? touch_id : touch_adj;
            const T *buf = (const T *)(part == 0 ? op->pairbuf_id : op->pairbuf);
            if (lst.empty()) continue;
            PairRec *d = nullptr;
            if ((rc = upload(op, &d, lst.data(), lst.size() * sizeof(PairRec)))) return rc;
            for (int64_t off = 0; off < (int64_t)lst.size(); off += 1 << 20) {
                int64_t cnt = std::min<int64_t>((int64_t)lst.size() - off, 1 << 20);
                hipLaunchKernelGGL((k_scatter_pairs<T>), dim3((unsigned)cnt), dim3(256), 0, op->st, d + off, s.nloc, s.nl,
                                   op->near_ld, op->sb, buf + off * s.nloc * s.nloc, (T *)op->nearb);
                LAUNCHCHK();
            }
        }
    }
    // far field: Chebyshev-node geometry of every cluster, coupling blocks
    int64_t ncl_all = s.cl_off[s.L + 1];
    int64_t nfar = (int64_t)s.far_src.size();
    op->coup_bytes = nfar * q2 * q2 * (int64_t)sizeof(T);
    if ((rc = dalloc(op, (void **)&op->nodes, (size_t)ncl_all * q2 * 4 * sizeof(double)))) return rc;
    hipLaunchKernelGGL(k_cluster_nodes, dim3(nblk(ncl_all * q2, 256)), dim3(256), 0, op->st, ncl_all, s.L, op->cl_off,
                       s.q, s.m, s.ne, op->zdev, s.tile_stride, op->tiles, op->tdeg, op->nodes);
    LAUNCHCHK();
    if (s.mode != IGB_H2_STORED) op->coup_bytes = 0;
    if ((rc = dalloc(op, &op->coup, op->coup_bytes))) return rc;
    if (nfar > 0 && s.mode == IGB_H2_STORED) {
        hipLaunchKernelGGL((k_coupling<T>), dim3((unsigned)nfar), dim3(256), 0, op->st, nfar, op->far_tgt, op->far_src, q2,
                           op->nodes, s.kappa, (T *)op->coup);
        LAUNCHCHK();
    }
    // Jacobi diagonal
    if ((rc = dalloc(op, &op->diag, (size_t)s.ndof * sizeof(T)))) return rc;
    {
        DiagArgs A;
        A.lo = op->lo;
        A.m = s.m;
        A.q = s.q;
        A.lmin = op->lmin;
        A.Tb = op->Tb;
        A.Mlev = op->Mlev;
        A.Mlev_off = op->Mlev_off;
        A.cl_off = op->cl_off;
        A.near_ptr = op->near_ptr;
        A.near_src = op->near_src;
        A.sb = op->sb;
        A.ld = op->near_ld;
        A.cbuf = nullptr;
        {
            // near-field terms block by block (symmetric storage, windows that fit LDS)
            const int W = s.side + s.p, SP = s.side * (s.p + 1), nj = W * W;
            const size_t shm_b =
                ((size_t)s.nl * nj + 2 * (size_t)SP * 2 * W + 1) * sizeof(double) + (size_t)nj * s.nl * sizeof(T);
            if (op->near_sym && op->nsb > 0 && nj <= 64 && shm_b <= 64 * 1024) {
                void *cb = nullptr;
                if ((rc = dalloc(op, &cb, (size_t)op->nsb * nj * sizeof(T)))) return rc;
                HIPCHK(hipMemsetAsync(cb, 0, (size_t)op->nsb * nj * sizeof(T), op->st));
                (void)hipFuncSetAttribute((const void *)k_diag_blocks<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)shm_b);
                hipLaunchKernelGGL((k_diag_blocks<T>), dim3((unsigned)op->nsb), dim3(256), shm_b, op->st, op->lo,
                                   op->sb_t, op->sb_s, op->near_ld, op->Tb, (const T *)op->nearb, (T *)cb);
                LAUNCHCHK();
                A.cbuf = cb;
            }
        }
        A.far_ptr = op->far_ptr;
        A.far_src = op->far_src;
        A.nodes = op->nodes;
        A.kappa = s.kappa;
        // far: moments of up to (p+2)^2 clusters; near: (p+1)^2 nloc support functions
        // (weight, slot, index) and the (p+2)^4 leaf-pair table
        const size_t ns = (size_t)(s.p + 1) * (s.p + 1) * s.nloc, ncm = (size_t)(s.p + 2) * (s.p + 2);
        size_t shm = std::max(((size_t)(s.p + 2) * (s.p + 2) * q2 + (size_t)2 * (s.p + 2) * s.q) * sizeof(double),
                              ns * (sizeof(double) + 2 * sizeof(int)) + ncm * ncm * sizeof(int));
        if (shm > 140 * 1024 || ncm * ncm > 4096) return fail(IGB_EUNSUPPORTED, "Jacobi diagonal: p or q too large");
        (void)hipFuncSetAttribute((const void *)k_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((k_diag<T>), dim3((unsigned)s.ndof), dim3(256), shm, op->st, A, s.ndof, (const T *)op->nearb,
                           (const T *)op->coup, (T *)op->diag);
        LAUNCHCHK();
    }
    return IGB_OK;
}

static igb_status create_device_geometry(igb_operator *op)
{
    Setup &s = op->s;
    igb_status rc;
    size_t esz = op->esz;
    int q2 = s.q * s.q;
    if ((rc = upload(op, &op->tiles, s.tiles.data(), s.tiles.size() * sizeof(double)))) return rc;
    {
        // line-contraction tiles of the touching-pair quadrature (see tile_fix), built on
        // the device from the element tiles: cm[l*G1 + k] = coefficient of t^l in the
        // Bernstein polynomial B_k of degree PG (identity when PG > 4: Bernstein form kept)
        const int PG = s.tile_degree, G1 = PG + 1;
        std::vector<double> cm((size_t)G1 * G1, 0.0);
        if (PG <= 4) {
            auto binom = [](int n, int k) {
                double c = 1.0;
                for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
                return c;
            };
            for (int l = 0; l <= PG; ++l)
                for (int k = 0; k <= l; ++k) cm[(size_t)l * G1 + k] = ((l - k) & 1 ? -1.0 : 1.0) * binom(PG, l) * binom(l, k);
        } else {
            for (int k = 0; k <= PG; ++k) cm[(size_t)k * G1 + k] = 1.0;
        }
        double *dcm = nullptr;
        if ((rc = upload(op, &dcm, cm.data(), cm.size() * sizeof(double)))) return rc;
        if ((rc = dalloc(op, (void **)&op->tline, (size_t)2 * s.nelem * s.tile_stride * sizeof(double)))) return rc;
        const int64_t n = (int64_t)s.nelem * G1 * G1 * 4;
        hipLaunchKernelGGL(k_tline, dim3(nblk(n, 256)), dim3(256), 0, op->st, s.nelem, G1, dcm, op->tiles, op->tline);
        LAUNCHCHK();
    }
    if ((rc = upload(op, &op->tdeg, s.tile_deg.data(), s.tile_deg.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(op, &op->gx, s.gx.data(), s.gx.size() * sizeof(double)))) return rc;
    if ((rc = upload(op, &op->gw, s.gw.data(), s.gw.size() * sizeof(double)))) return rc;
    {
        std::vector<double> bt(s.gx.size() * (s.p + 1));
        for (size_t k = 0; k < s.gx.size(); ++k) {
            double t = s.gx[k];
            for (int r = 0; r <= s.p; ++r) {
                double c = 1.0;
                for (int i = 1; i <= r; ++i) c = c * (s.p - r + i) / i;
                bt[k * (s.p + 1) + r] = c * std::pow(t, r) * std::pow(1.0 - t, s.p - r);
            }
        }
        if ((rc = upload(op, &op->btab, bt.data(), bt.size() * sizeof(double)))) return rc;
    }
    if ((rc = upload(op, &op->cl_off, s.cl_off.data(), s.cl_off.size() * sizeof(int64_t)))) return rc;
    if ((rc = upload(op, &op->zdev, s.z.data(), s.z.size() * sizeof(double)))) return rc;
    if ((rc = upload(op, &op->M1, s.M1.data(), s.M1.size() * sizeof(double)))) return rc;
    if ((rc = upload(op, &op->E2, s.E2.data(), s.E2.size() * sizeof(double)))) return rc;
    if ((rc = upload(op, &op->Mlev, s.Mlev.data(), s.Mlev.size() * sizeof(double)))) return rc;
    if ((rc = upload(op, &op->Mlev_off, s.Mlev_off.data(), s.Mlev_off.size() * sizeof(int64_t)))) return rc;
    if ((rc = upload(op, &op->Tb, s.Tb.data(), s.Tb.size() * sizeof(double)))) return rc;
    int64_t ncl_all = s.cl_off[s.L + 1];
    if ((rc = dalloc(op, &op->xs, s.nsup * esz))) return rc;
    if ((rc = dalloc(op, &op->ys, s.nsup * esz))) return rc;
    if ((rc = dalloc(op, &op->Xh, ncl_all * q2 * esz))) return rc;
    if ((rc = dalloc(op, &op->Yh, ncl_all * q2 * esz))) return rc;
    HIPCHK(hipMemsetAsync(op->Xh, 0, ncl_all * q2 * esz, op->st));
    HIPCHK(hipMemsetAsync(op->Yh, 0, ncl_all * q2 * esz, op->st));
    for (void **v : {&op->r, &op->z, &op->pv, &op->Ap, &op->tmp, &op->rr, &op->dw})
        if ((rc = dalloc(op, v, s.ndof * esz))) return rc;
    if ((rc = dalloc(op, &op->part, 3 * kRedBlocks * esz))) return rc;  // dot partials; CG: 3 sets
    if ((rc = dalloc(op, &op->dpart, nblk(s.ndof, 256) * esz))) return rc;  // p . Ap partials of the T pass
    if ((rc = dalloc(op, &op->tz, (size_t)s.npatch * s.ne * (s.p + 1) * s.ns1 * esz))) return rc;
    if ((rc = dalloc(op, (void **)&op->scal, 16 * sizeof(double)))) return rc;
    // mapped and coherent: the CG direction kernel writes residuals into it directly
    HIPCHK(hipHostMalloc((void **)&op->h_scal, 16 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    if ((rc = dalloc(op, &op->potc, (size_t)s.nelem * s.grhs * s.grhs * esz))) return rc;
    return op->cplx ? assemble_identical<cd>(op) : assemble_identical<double>(op);
}

static igb_status create_device_plan(igb_operator *op)
{
    Setup &s = op->s;
    igb_status rc;
    if ((rc = upload(op, &op->near_ptr, s.near_ptr.data(), s.near_ptr.size() * sizeof(int64_t)))) return rc;
    if ((rc = upload(op, &op->near_src, s.near_src.data(), s.near_src.size() * sizeof(int32_t)))) return rc;
    if ((rc = upload(op, &op->far_ptr, s.far_ptr.data(), s.far_ptr.size() * sizeof(int64_t)))) return rc;
    if ((rc = upload(op, &op->far_src, s.far_src.data(), s.far_src.size() * sizeof(int32_t)))) return rc;
    {
        std::vector<int32_t> tg(s.far_src.size());
        for (int64_t c = 0; c + 1 < (int64_t)s.far_ptr.size(); ++c)
            for (int64_t k = s.far_ptr[c]; k < s.far_ptr[c + 1]; ++k) tg[k] = (int32_t)c;
        if ((rc = upload(op, &op->far_tgt, tg.data(), tg.size() * sizeof(int32_t)))) return rc;
    }
    if (far_mirrored(s)) {
        // mirrored pairs: entry e = (c, src) with src > c owns pair k; its mirror
        // (src, c) reads the column part of k
        int64_t nfar = (int64_t)s.far_src.size(), ncl = (int64_t)s.far_ptr.size() - 1;
        std::vector<int64_t> upk(nfar, -1);
        std::vector<int32_t> ut, us, pidx(nfar);
        for (int64_t c = 0; c < ncl; ++c)
            for (int64_t e = s.far_ptr[c]; e < s.far_ptr[c + 1]; ++e)
                if (s.far_src[e] > c) {
                    upk[e] = (int64_t)ut.size();
                    ut.push_back((int32_t)c);
                    us.push_back(s.far_src[e]);
                }
        if ((int64_t)ut.size() * 2 >= ((int64_t)1 << 31)) return fail(IGB_EUNSUPPORTED, "too many far blocks");
        for (int64_t c = 0; c < ncl; ++c)
            for (int64_t e = s.far_ptr[c]; e < s.far_ptr[c + 1]; ++e) {
                int32_t src = s.far_src[e];
                if (src > c) {
                    pidx[e] = (int32_t)(2 * upk[e]);
                    continue;
                }
                auto b = s.far_src.begin() + s.far_ptr[src], en = s.far_src.begin() + s.far_ptr[src + 1];
                auto it = std::lower_bound(b, en, (int32_t)c);
                if (src == c || it == en || *it != (int32_t)c)
                    return fail(IGB_EINVAL, "far-field partition is not symmetric");
                pidx[e] = (int32_t)(2 * upk[it - s.far_src.begin()] + 1);
            }
        op->nup = (int64_t)ut.size();
        if ((rc = upload(op, &op->up_t, ut.data(), ut.size() * sizeof(int32_t)))) return rc;
        if ((rc = upload(op, &op->up_s, us.data(), us.size() * sizeof(int32_t)))) return rc;
        if ((rc = upload(op, &op->far_pidx, pidx.data(), pidx.size() * sizeof(int32_t)))) return rc;
        if ((rc = dalloc(op, &op->fpart, (size_t)2 * op->nup * s.q * s.q * op->esz))) return rc;
    }
    return op->cplx ? assemble<cd>(op) : assemble<double>(op);
}

// ---------------------------------------------------------------------------
// Krylov solvers
// ---------------------------------------------------------------------------
static igb_status read_scalar(igb_operator *op, int idx, double *out)
{
    HIPCHK(hipMemcpyAsync(op->h_scal + idx, op->scal + idx, sizeof(double), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
    *out = op->h_scal[idx];
    return IGB_OK;
}

// far_precision IGB_FP32: the steps use the single-precision far field; every
// kReplaceEvery steps the recursive residual is replaced by the FP64 one
// ("reliable updates"), and convergence is always judged on the FP64 residual.
static const int kReplaceEvery = 20;

static igb_status solve_cg(igb_operator *op, const double *b, double *w, double tol, int maxit, igb_solve_info *info)
{
    int64_t n = op->s.ndof;
    double *r = (double *)op->r, *z = (double *)op->z, *p = (double *)op->pv, *Ap = (double *)op->Ap;
    const double *D = (const double *)op->diag;
    double *sc = op->scal;
    igb_status rc;
    unsigned gb = std::min<unsigned>(nblk(n, 256), 1024);
    double bn2, rr;
    if ((rc = dot_dev<double>(op, n, b, b, sc + 3))) return rc;
    if ((rc = read_scalar(op, 3, &bn2))) return rc;
    double bn = std::sqrt(bn2);
    if (bn == 0.0) bn = 1.0;
    int it = 0;
    double rel = 0.0;
    for (;;) {
        // the true residual, always with the full-precision far field
        op->force_fp64 = true;
        rc = matvec_S<double>(op, w, Ap);
        op->force_fp64 = false;
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, op->st));
        hipLaunchKernelGGL((k_axpby<double>), dim3(gb), dim3(256), 0, op->st, n, -1.0, Ap, 1.0, r);
        LAUNCHCHK();
        if ((rc = dot_dev<double>(op, n, r, r, sc + 3))) return rc;
        if ((rc = read_scalar(op, 3, &rr))) return rc;
        rel = std::sqrt(rr) / bn;
        if (rel <= tol || it >= maxit) break;
        hipLaunchKernelGGL((k_div<double>), dim3(gb), dim3(256), 0, op->st, n, r, D, z);
        LAUNCHCHK();
        HIPCHK(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, op->st));
        if ((rc = dot_dev<double>(op, n, r, z, sc + 0))) return rc;
        // rz alternates between sc[0] and sc[2] (the step reads the old value while the
        // direction kernel writes the new one); r.z and r.r partials live in op->part.
        // Step k writes (rr, done) to pinned slot k & 1 and records ev[k & 1]; the host
        // reads step k while step k + 1 runs, and a step after convergence does nothing.
        double *pp = (double *)op->dpart, *p2 = (double *)op->part + 256;
        const int np = (int)nblk(n, 256);
        const unsigned gs = std::min<unsigned>(gb, 256);
        hipLaunchKernelGGL(k_set2, dim3(1), dim3(1), 0, op->st, sc + 4, 0.0, sc + 5, (tol * bn) * (tol * bn));
        LAUNCHCHK();
        hipEvent_t ev[2];
        HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(ev[0]);
            return fail(IGB_EHIP, "hipEventCreate");
        }
        // the direction kernel writes (rr, done) of step k straight into pinned slot k & 1
        double *hres = nullptr;
        if (hipHostGetDevicePointer((void **)&hres, op->h_scal + 8, 0) != hipSuccess) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            return fail(IGB_EHIP, "hipHostGetDevicePointer");
        }
        int slot = 0, launched = 0, examined = 0;
        bool conv = false;
        rc = IGB_OK;
        while (true) {
            if (it + launched < maxit && launched - examined < 2) {
                if (op->far_single && launched > 0 && launched % kReplaceEvery == 0) {
                    // reliable update: the recursive residual is replaced by b - A w with the
                    // full-precision far field (and z, r.z with it); the direction p is kept
                    op->force_fp64 = true;
                    rc = matvec_S<double>(op, w, Ap);
                    op->force_fp64 = false;
                    if (rc) break;
                    if (hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, op->st) != hipSuccess) {
                        rc = fail(IGB_EHIP, "CG residual replacement");
                        break;
                    }
                    hipLaunchKernelGGL((k_axpby<double>), dim3(gb), dim3(256), 0, op->st, n, -1.0, Ap, 1.0, r);
                    hipLaunchKernelGGL((k_div<double>), dim3(gb), dim3(256), 0, op->st, n, r, D, z);
                    if ((rc = dot_dev<double>(op, n, r, z, sc + slot))) break;
                }
                if ((rc = matvec_S<double>(op, p, Ap, pp))) break;
                hipLaunchKernelGGL(k_cg_step, dim3(gs), dim3(256), 0, op->st, n, sc + slot, pp, np, w, r, p, Ap, D, z,
                                   p2, sc + 4);
                hipLaunchKernelGGL(k_cg_dir, dim3(gs), dim3(256), 0, op->st, n, p2, (int)gs, sc + slot, sc + (2 - slot),
                                   sc + 3, p, z, sc + 5, sc + 4, hres + 2 * (launched & 1));
                if (hipGetLastError() != hipSuccess || hipEventRecord(ev[launched & 1], op->st) != hipSuccess) {
                    rc = fail(IGB_EHIP, "CG kernel launch");
                    break;
                }
                slot = 2 - slot;
                ++launched;
                continue;
            }
            if (examined == launched) break;  // max_iter reached and every step read
            if (hipEventSynchronize(ev[examined & 1]) != hipSuccess) { rc = fail(IGB_EHIP, "hipEventSynchronize"); break; }
            const double *h = op->h_scal + 8 + 2 * (examined & 1);
            rr = h[0];
            ++examined;
            if (h[1] != 0.0) { conv = true; break; }
        }
        (void)hipStreamSynchronize(op->st);  // the pinned slots stay valid until the last copy lands
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (rc) return rc;
        it += examined;
        (void)conv;  // the true residual b - A w decides, at the top of the loop
    }
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->converged = rel <= tol;
        info->fallback = 0;
    }
    return rel <= tol ? IGB_OK : fail(IGB_ENOT_CONVERGED, "CG stopped at max_iter with relative residual " + std::to_string(rel));
}

// One Arnoldi step's bookkeeping of (flexible) GMRES, on the device: the new
// Hessenberg column h = hA + hB (two classical Gram-Schmidt passes) with
// h[k+1] = |v_{k+1}| (from the nvv partial sums of its squared norm), the
// earlier Givens rotations applied to it, a new rotation that zeroes h[k+1],
// the rotated right-hand side g, and the residual estimate |g[k+1]| / |b|.
// G holds H ((R+1) x R, row j, column k at j*R + k), cs, sn (R each), g (R+1),
// then the state st (doubles): |b|, 1/|v_{k+1}|, the first step count that
// reached tol (or -1), tol.  The estimate and a converged flag go to the
// host-mapped pair `out`.  Steps after convergence leave G as it is.  One
// wave: the column, the rotations and the norm partials are staged in LDS by
// all lanes, the rotations run serially on lane 0, and the lanes write back.
template <class T> __host__ __device__ inline T from_real(double a);
template <> __host__ __device__ inline double from_real<double>(double a) { return a; }
template <> __host__ __device__ inline cd from_real<cd>(double a) { return {a, 0.0}; }
__host__ __device__ inline double div_(double a, double b) { return a / b; }
__host__ __device__ inline cd div_(cd a, cd b)
{
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

template <class T>
__global__ void __launch_bounds__(64) k_arnoldi(int k, int R, const T *__restrict__ hA, const T *__restrict__ hB,
                                                 const double *__restrict__ vv, int nvv, T *__restrict__ G,
                                                 double *__restrict__ out)
{
    extern __shared__ double sm[];
    T *col = (T *)sm, *c = col + k + 2, *sv = c + k + 1;
    T *H = G, *cs = G + (size_t)(R + 1) * R, *sn = cs + R, *g = sn + R;
    double *st = (double *)(g + R + 1);
    const int lane = threadIdx.x;
    if (st[2] >= 0.0) {  // converged at an earlier step
        if (lane == 0) {
            out[0] = 0.0;
            out[1] = 1.0;
        }
        return;
    }
    for (int j = lane; j <= k; j += 64) {
        col[j] = hA[j] + hB[j];
        c[j] = cs[j];
        sv[j] = sn[j];
    }
    double v2 = 0.0;
    for (int b = lane; b < nvv; b += 64) v2 += vv[b];
    v2 = wave_sum64(v2);
    __syncthreads();
    if (lane == 0) {
        const double hn = sqrt(v2);
        st[1] = hn > 0.0 ? 1.0 / hn : 0.0;
        for (int j = 0; j < k; ++j) {
            const T a = col[j], b = col[j + 1];
            col[j] = conj_(c[j]) * a + conj_(sv[j]) * b;
            col[j + 1] = c[j] * b - sv[j] * a;
        }
        const T a = col[k];
        const double den = sqrt(abs2(a) + hn * hn);
        const T ck = den > 0.0 ? a * (1.0 / den) : from_real<T>(1.0);
        const T sk = from_real<T>(den > 0.0 ? hn / den : 0.0);
        cs[k] = ck;
        sn[k] = sk;
        col[k] = from_real<T>(den);
        const T gk = g[k];
        g[k + 1] = zero<T>() - sk * gk;
        g[k] = conj_(ck) * gk;
        const double res = sqrt(abs2(g[k + 1])) / st[0];
        const bool conv = res <= st[3];
        if (conv) st[2] = k + 1;
        out[0] = res;
        out[1] = conv ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = lane; j <= k; j += 64) H[(size_t)j * R + k] = col[j];
}

// x *= *alpha (alpha real, on the device); with z, also z = x / D (the next
// Jacobi direction)
template <class T>
__global__ void k_scale_dev(int64_t n, const double *__restrict__ alpha, T *__restrict__ x, const T *__restrict__ D,
                            T *__restrict__ z)
{
    const double a = *alpha;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = x[i] * a;
        x[i] = v;
        if (z) z[i] = div_(v, D[i]);
    }
}

// GMRES, right preconditioned in the flexible form (the preconditioned
// directions z_k are kept, since a network is not a fixed linear map; with
// Jacobi it is plain right-preconditioned GMRES), classical Gram-Schmidt applied
// twice, Givens rotations on the device.  The host keeps at most two steps in
// flight and reads each step's residual estimate from mapped memory, so the
// device never waits for it; the small triangular solve runs on the host once
// per restart cycle.  Real (Laplace, optionally with a network) and complex
// (Helmholtz, Jacobi) systems; the operator runs in FP64 throughout.
// fp64 = false (single-precision far field only): the products use that far field; the
// refinement of solve_refined keeps the FP64 residuals outside.
template <class T>
static igb_status solve_gmres_dev(igb_operator *op, const igb_cnn *net, const T *b, T *w, double tol, int maxit,
                                  int restart, igb_solve_info *info, bool fp64 = true)
{
    const Setup &s = op->s;
    const int64_t n = s.ndof;
    const int R = std::max(1, std::min(restart, std::max(1, maxit)));
    igb_status rc;
    struct Restore {
        igb_operator *o;
        bool v;
        ~Restore() { o->force_fp64 = v; }
    } restore{op, op->force_fp64};
    op->force_fp64 = fp64;
    const size_t gT = (size_t)(R + 1) * R + 3 * (size_t)R + 1;  // H, cs, sn, g
    if (op->Vcols < R + 1 || op->Zcols < R) {
        HIPCHK(hipStreamSynchronize(op->st));
        pool_free(op->Vblk);
        pool_free(op->Zblk);
        pool_free(op->Gblk);
        pool_free(op->hblk);
        pool_free(op->mblk);
        op->V = op->hdev = op->mpart = nullptr;
        op->Vcols = op->Zcols = 0;
        HIPCHK(pool_alloc(op->Vblk, (size_t)(R + 1) * n * sizeof(T)));
        HIPCHK(pool_alloc(op->Zblk, (size_t)R * n * sizeof(T)));
        HIPCHK(pool_alloc(op->Gblk, gT * sizeof(T) + 8 * sizeof(double)));
        HIPCHK(pool_alloc(op->hblk, 2 * (size_t)(R + 1) * sizeof(T)));
        HIPCHK(pool_alloc(op->mblk, (size_t)(R + 1) * kRedBlocks * sizeof(T)));
        op->V = op->Vblk.p;
        op->hdev = op->hblk.p;
        op->mpart = op->mblk.p;
        op->Vcols = R + 1;
        op->Zcols = R;
    }
    T *V = (T *)op->V, *Z = (T *)op->Zblk.p, *G = (T *)op->Gblk.p, *t = (T *)op->tmp, *r = (T *)op->r;
    T *hA = (T *)op->hdev, *hB = hA + R + 1, *gdev = G + (size_t)(R + 1) * R + 2 * (size_t)R;
    double *st = (double *)(gdev + R + 1);
    const T *D = (const T *)op->diag;
    const unsigned gb = std::min<unsigned>(nblk(n, 256), 1024);
    const int mdb = multidot_blocks(n);
    const unsigned gsub = std::min<unsigned>(nblk(n, 256), 256);  // k_sub_Vh_red blocks (norm partials)
    double *nrm = (double *)op->part;                             // 3 kRedBlocks >= gsub doubles
    // the Givens step stages 3 k + 4 values in LDS: above 64 KB (complex cycles longer than 1365) the
    // launch needs the larger limit of gfx950 (160 KB per workgroup) granted explicitly
    if (sizeof(T) * (3 * (size_t)R + 4) > 64 * 1024 &&
        hipFuncSetAttribute((const void *)k_arnoldi<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(T) * (3 * (size_t)R + 4))) != hipSuccess)
        return fail(IGB_EHIP, "hipFuncSetAttribute: GMRES restart " + std::to_string(R) + " needs " +
                                  std::to_string(sizeof(T) * (3 * (size_t)R + 4)) + " bytes of LDS");
    double *hout = nullptr;  // two (estimate, converged) slots of mapped host memory, device view
    HIPCHK(hipHostGetDevicePointer((void **)&hout, op->h_scal + 12, 0));
    auto norm2 = [&](const T *x, double *out) -> igb_status {
        igb_status c;
        if ((c = dot_dev<T>(op, n, x, x, (T *)op->scal))) return c;
        return read_scalar(op, 0, out);  // real part
    };
    double bn2;
    if ((rc = norm2(b, &bn2))) return rc;
    double bn = std::sqrt(bn2);
    if (bn == 0.0) bn = 1.0;
    std::vector<T> H((size_t)(R + 1) * R), gh(R + 1), y(R), ginit(R + 1);
    std::vector<double> stinit(8, 0.0);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        return fail(IGB_EHIP, "hipEventCreate");
    }
    struct Events {
        hipEvent_t *e;
        ~Events() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); }
    } events{ev};
    int it = 0, last_k = 0;
    double rel = 0.0, prev_rel = -1.0;
    // the network is dropped for Jacobi (the fallback) once a restart cycle of k steps fails to cut the true
    // residual by 0.9^k (a rate Jacobi beats on these operators: 1e-8 in 70-100 steps)
    const igb_cnn *pnet = net;
    int fell_back = 0;
    for (;;) {
        if ((rc = matvec_S<T>(op, w, t))) return rc;
        HIPCHK(hipMemcpyAsync(r, b, n * sizeof(T), hipMemcpyDeviceToDevice, op->st));
        hipLaunchKernelGGL((k_axpby<T>), dim3(gb), dim3(256), 0, op->st, n, from_real<T>(-1.0), (const T *)t,
                           from_real<T>(1.0), r);
        LAUNCHCHK();
        double beta2;
        if ((rc = norm2(r, &beta2))) return rc;
        const double beta = std::sqrt(beta2);
        rel = beta / bn;
        if (pnet && prev_rel > 0.0 && rel > std::pow(0.9, last_k) * prev_rel) {
            pnet = nullptr;
            fell_back = 1;
        }
        prev_rel = rel;
        if (rel <= tol || it >= maxit) break;
        hipLaunchKernelGGL((k_axpby<T>), dim3(gb), dim3(256), 0, op->st, n, from_real<T>(1.0 / beta), (const T *)r,
                           zero<T>(), V);
        LAUNCHCHK();
        // g = (beta, 0, ...), state = (|b|, -, not converged, tol); the stream is idle here
        std::fill(ginit.begin(), ginit.end(), zero<T>());
        ginit[0] = from_real<T>(beta);
        stinit[0] = bn;
        stinit[2] = -1.0;
        stinit[3] = tol;
        HIPCHK(hipMemcpyAsync(gdev, ginit.data(), (R + 1) * sizeof(T), hipMemcpyHostToDevice, op->st));
        HIPCHK(hipMemcpyAsync(st, stinit.data(), 8 * sizeof(double), hipMemcpyHostToDevice, op->st));
        const int kmax = std::min(R, maxit - it);
        int launched = 0, examined = 0, kuse = -1;
        rc = IGB_OK;
        while (true) {
            if (launched < kmax && launched - examined < 2) {
                const int k = launched;
                T *vk = V + (size_t)k * n, *vn = V + (size_t)(k + 1) * n, *zk = Z + (size_t)k * n;
                if constexpr (std::is_same<T, double>::value) {
                    if (pnet) {
                        if ((rc = cnn_precondition(pnet, s.npatch, s.ns1, s.ns1, vk, D, zk, op->st))) break;
                    }
                }
                if (!pnet && k == 0)
                    hipLaunchKernelGGL((k_div<T>), dim3(gb), dim3(256), 0, op->st, n, (const T *)vk, D, zk);
                // else (Jacobi) z_k = D^-1 v_k was formed when v_k was normalised
                if ((rc = matvec_S<T>(op, zk, vn))) break;
                for (int pass = 0; pass < 2; ++pass) {
                    T *hp = pass ? hB : hA;
                    hipLaunchKernelGGL((k_multidot_partial<T>), dim3(mdb, (unsigned)((k + 4) / 4)), dim3(256), 0,
                                       op->st, n, k + 1, (const T *)V, n, (const T *)vn, (T *)op->mpart, mdb);
                    hipLaunchKernelGGL((k_sub_Vh_red<T>), dim3(gsub), dim3(256), (size_t)(k + 1) * sizeof(T), op->st, n,
                                       k + 1, (const T *)V, n, (const T *)op->mpart, mdb, hp, vn,
                                       pass ? nrm : (double *)nullptr);
                }
                hipLaunchKernelGGL((k_arnoldi<T>), dim3(1), dim3(64), (size_t)(3 * k + 4) * sizeof(T), op->st, k, R,
                                   (const T *)hA, (const T *)hB, (const double *)nrm, (int)gsub, G, hout + 2 * (k & 1));
                T *znext = (!pnet && k + 1 < kmax) ? Z + (size_t)(k + 1) * n : nullptr;
                hipLaunchKernelGGL((k_scale_dev<T>), dim3(gb), dim3(256), 0, op->st, n, (const double *)(st + 1), vn, D,
                                   znext);
                if (hipGetLastError() != hipSuccess || hipEventRecord(ev[k & 1], op->st) != hipSuccess) {
                    rc = fail(IGB_EHIP, "GMRES kernel launch");
                    break;
                }
                ++launched;
                continue;
            }
            if (examined == launched) break;
            if (hipEventSynchronize(ev[examined & 1]) != hipSuccess) {
                rc = fail(IGB_EHIP, "hipEventSynchronize");
                break;
            }
            const double *h = op->h_scal + 12 + 2 * (examined & 1);
            ++examined;
            if (h[1] != 0.0) {
                kuse = examined;
                break;
            }
        }
        HIPCHK(hipStreamSynchronize(op->st));
        if (rc) return rc;
        const int k = kuse > 0 ? kuse : examined;
        it += k;
        last_k = k;
        // y = H^-1 g (upper triangular k x k); w += Z y
        HIPCHK(hipMemcpy(H.data(), G, (size_t)k * R * sizeof(T), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(gh.data(), gdev, (R + 1) * sizeof(T), hipMemcpyDeviceToHost));
        for (int j = k - 1; j >= 0; --j) {
            T sum = gh[j];
            for (int l = j + 1; l < k; ++l) sum -= H[(size_t)j * R + l] * y[l];
            y[j] = div_(sum, H[(size_t)j * R + j]);
        }
        for (int j = 0; j < k; ++j) y[j] = zero<T>() - y[j];
        HIPCHK(hipMemcpyAsync(hA, y.data(), k * sizeof(T), hipMemcpyHostToDevice, op->st));
        hipLaunchKernelGGL((k_sub_Vh<T>), dim3(gb), dim3(256), 0, op->st, n, k, (const T *)Z, n, (const T *)hA, w);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(op->st));
    }
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->converged = rel <= tol;
        info->fallback = fell_back;
    }
    return rel <= tol ? IGB_OK
                      : fail(IGB_ENOT_CONVERGED, "GMRES stopped at max_iter with relative residual " + std::to_string(rel));
}

__global__ void k_err64(int64_t n, const float *__restrict__ y, const float *__restrict__ f, const float *__restrict__ x,
                        double *__restrict__ e)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) e[i] = (double)y[i] + (double)f[i] - (double)x[i];
}

__global__ void k_grad32(int64_t n, const double *__restrict__ g, double scale, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(g[i] * scale);
}

__global__ void k_pairs_out(int64_t n, const double *__restrict__ t, const double *__restrict__ D,
                            const double *__restrict__ x, float *__restrict__ y32, float *__restrict__ x32)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y32[i] = (float)(t[i] / D[i]);
    x32[i] = (float)x[i];
}

// ===========================================================================
// C ABI
// ===========================================================================

#define CHECK_OP(op)                                                       \
    do {                                                                   \
        if (!(op)) return fail(IGB_EINVAL, "operator is null");            \
    } while (0)

// The entry points below have C linkage through their declarations in igabem.h.

const char *igb_last_error(void) { return g_err.c_str(); }

igb_status igb_geometry_create(int32_t n_patches, const igb_nurbs_patch *patches, igb_geometry **out)
{
    if (!out) return fail(IGB_EINVAL, "out is null");
    *out = nullptr;
    igb_geometry *g = new igb_geometry();
    std::string err = make_geometry(n_patches, patches, g->g);
    if (!err.empty()) {
        delete g;
        return fail(IGB_EINVAL, err);
    }
    *out = g;
    return IGB_OK;
}

void igb_geometry_destroy(igb_geometry *geo) { delete geo; }

void igb_operator_destroy(igb_operator *op)
{
    if (!op) return;
    // buffers go back to the pool only once the operator's stream has drained
    if (hipStreamSynchronize(op->st) == hipSuccess) {
        for (DevBlock &b : op->owned) pool_free(b);
        pool_free(op->Vblk);
        pool_free(op->Zblk);
        pool_free(op->Gblk);
        pool_free(op->hblk);
        pool_free(op->mblk);
    } else {
        for (DevBlock &b : op->owned) (void)hipFree(b.p);
        (void)hipFree(op->Vblk.p);
        (void)hipFree(op->Zblk.p);
        (void)hipFree(op->Gblk.p);
        (void)hipFree(op->hblk.p);
        (void)hipFree(op->mblk.p);
    }
    if (op->h_scal) (void)hipHostFree(op->h_scal);
    if (op->st2) {
        (void)hipStreamSynchronize(op->st2);
        (void)hipStreamDestroy(op->st2);
    }
    if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
    if (op->ev_join) (void)hipEventDestroy(op->ev_join);
    for (hipEvent_t e : op->qev)
        if (e) (void)hipEventDestroy(e);
    delete op;
}

igb_status igb_release_cached_memory(void)
{
    const hipError_t e = pool_release_all();
    return e == hipSuccess ? IGB_OK : fail(IGB_EHIP, std::string("hipFree: ") + hipGetErrorString(e));
}

igb_status igb_operator_create(const igb_geometry *geo, const igb_params *prm, void *hip_stream, igb_operator **out)
{
    if (!geo || !prm || !out) return fail(IGB_EINVAL, "null argument");
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    igb_operator *op = new igb_operator();
    op->st = (hipStream_t)hip_stream;
    if (hipGetDevice(&op->dev) != hipSuccess) {
        delete op;
        return fail(IGB_EHIP, "hipGetDevice failed");
    }
    for (hipEvent_t &e : op->qev)
        if (hipEventCreate(&e) != hipSuccess) {
            igb_operator_destroy(op);
            return fail(IGB_EHIP, "hipEventCreate failed");
        }
    std::string err;
    try {
        err = build_setup_tiles(geo->g, *prm, op->s);
    } catch (const std::bad_alloc &) {
        delete op;
        return fail(IGB_ENOMEM, "host allocation failed during setup");
    }
    if (!err.empty()) {
        delete op;
        return fail(IGB_EINVAL, err);
    }
    Setup &s = op->s;
    op->cplx = s.kernel == IGB_HELMHOLTZ;
    op->far_single = prm->far_precision == IGB_FP32;
    op->esz = op->cplx ? sizeof(cd) : sizeof(double);
    {
        int dv = 0, n = 0;
        if (hipGetDevice(&dv) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dv) == hipSuccess && n > 0)
            op->ncu = n;
    }
    op->lo = Layout{s.p, s.p + 1, s.nloc, s.nl, s.side, s.L, s.ne, s.ns1};
    // GPU: Gauss-node geometry and identical-pair quadrature, then the other touching
    // pairs; host meanwhile: element geometry, touching search, tree, partition, lists
    igb_status rc = create_device_geometry(op);
    if (rc == IGB_OK) {
        try {
            build_setup_elements(s);
        } catch (const std::bad_alloc &) {
            rc = fail(IGB_ENOMEM, "host allocation failed during setup");
        }
    }
    if (rc == IGB_OK) rc = op->cplx ? assemble_adjacent<cd>(op) : assemble_adjacent<double>(op);
    if (rc == IGB_OK) {
        try {
            err = build_setup_plan(s);
        } catch (const std::bad_alloc &) {
            err = "host allocation failed during setup";
        }
        if (!err.empty()) rc = fail(IGB_EINVAL, err);
    }
    if (rc == IGB_OK) {
        op->lmin = s.L + 1;
        for (size_t k = 0; k < s.far.size(); k += 3) op->lmin = std::min(op->lmin, (int)s.far[k]);
        rc = create_device_plan(op);
    }
    if (rc == IGB_OK && op->far_single && op->cplx && op->near_sym && s.nl <= 256 && op->near_bytes > 0) {
        // the near blocks of the inner single-precision products, rounded once the assembly has written them
        const int64_t nval = op->near_bytes / (int64_t)sizeof(cd);
        rc = dalloc(op, &op->nearb32, (size_t)nval * sizeof(cf));
        if (rc == IGB_OK) {
            hipLaunchKernelGGL(k_round_c32, dim3((unsigned)std::min<int64_t>(nblk(nval, 256), 65536)), dim3(256), 0,
                               op->st, nval, (const cd *)op->nearb, (cf *)op->nearb32);
            if (hipGetLastError() != hipSuccess) rc = fail(IGB_EHIP, "k_round_c32 launch");
        }
    }
    if (rc == IGB_OK) {
        hipError_t e = hipStreamSynchronize(op->st);
        if (e != hipSuccess) rc = fail(IGB_EHIP, std::string("assembly: ") + hipGetErrorString(e));
    }
    if (rc == IGB_OK) {
        // kernel time of the pair quadrature (HIP events around its launches on the operator's stream)
        float a = 0.f, b = 0.f, c = 0.f;
        if (hipEventElapsedTime(&a, op->qev[4], op->qev[5]) == hipSuccess &&
            hipEventElapsedTime(&b, op->qev[0], op->qev[1]) == hipSuccess &&
            hipEventElapsedTime(&c, op->qev[2], op->qev[3]) == hipSuccess) {
            op->quad_ms[0] = a;
            op->quad_ms[1] = (double)b + (double)c;
        }
    }
    if (rc != IGB_OK) {
        std::string msg = g_err;
        igb_operator_destroy(op);
        g_err = msg;
        return rc;
    }
    op->assembly_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = op;
    return IGB_OK;
}

static void fill_info(const Setup &s, size_t esz, igb_info *out);

igb_status igb_operator_info(const igb_operator *op, igb_info *out)
{
    CHECK_OP(op);
    if (!out) return fail(IGB_EINVAL, "out is null");
    fill_info(op->s, op->esz, out);
    out->assembly_seconds = op->assembly_seconds;
    out->quad_regular_ms = op->quad_ms[0];
    out->quad_touching_ms = op->quad_ms[1];
    return IGB_OK;
}

igb_status igb_rhs_points(const igb_operator *op, double *xyz_dev)
{
    CHECK_OP(op);
    if (!xyz_dev) return fail(IGB_EINVAL, "xyz_dev is null");
    int64_t n = (int64_t)op->s.nelem * op->s.grhs * op->s.grhs;
    hipLaunchKernelGGL(k_rhs_points, dim3(nblk(n, 256)), dim3(256), 0, op->st, n, op->rpts, xyz_dev);
    LAUNCHCHK();
    return IGB_OK;
}

template <class T>
static igb_status rhs_impl(igb_operator *op, const T *g, T *b)
{
    const Setup &s = op->s;
    hipLaunchKernelGGL((k_rhs_super<T>), dim3(nblk(s.nsup, 256)), dim3(256), 0, op->st, op->lo, s.nsup, s.grhs,
                       op->gx + s.goff[s.grhs], op->rpts, g, (T *)op->ys);
    LAUNCHCHK();
    return apply_T<T>(op, (const T *)op->ys, b);
}

igb_status igb_rhs_assemble(const igb_operator *cop, const void *g_dev, void *b_dev)
{
    CHECK_OP(cop);
    if (!g_dev || !b_dev) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? rhs_impl<cd>(op, (const cd *)g_dev, (cd *)b_dev) : rhs_impl<double>(op, (const double *)g_dev, (double *)b_dev);
}

igb_status igb_matvec(const igb_operator *cop, const void *x_dev, void *y_dev)
{
    CHECK_OP(cop);
    if (!x_dev || !y_dev) return fail(IGB_EINVAL, "null device pointer");
    if (x_dev == y_dev) return fail(IGB_EINVAL, "x and y must not alias");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? matvec_S<cd>(op, (const cd *)x_dev, (cd *)y_dev) : matvec_S<double>(op, (const double *)x_dev, (double *)y_dev);
}

template <class T>
static igb_status matvec_super_impl(igb_operator *op, const T *x, T *y)
{
    const Setup &s = op->s;
    hipLaunchKernelGGL((k_perm<T>), dim3(nblk(s.nsup, 256)), dim3(256), 0, op->st, op->lo, s.nsup, x, (T *)op->xs, 1);
    LAUNCHCHK();
    igb_status rc = matvec_internal<T>(op, (const T *)op->xs, (T *)op->ys);
    if (rc) return rc;
    hipLaunchKernelGGL((k_perm<T>), dim3(nblk(s.nsup, 256)), dim3(256), 0, op->st, op->lo, s.nsup, (const T *)op->ys, y, 0);
    LAUNCHCHK();
    return IGB_OK;
}

igb_status igb_matvec_super(const igb_operator *cop, const void *xs_dev, void *ys_dev)
{
    CHECK_OP(cop);
    if (!xs_dev || !ys_dev) return fail(IGB_EINVAL, "null device pointer");
    if (xs_dev == ys_dev) return fail(IGB_EINVAL, "xs and ys must not alias");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? matvec_super_impl<cd>(op, (const cd *)xs_dev, (cd *)ys_dev)
                    : matvec_super_impl<double>(op, (const double *)xs_dev, (double *)ys_dev);
}

template <class T>
static igb_status Tt_impl(igb_operator *op, const T *w, T *xs)
{
    igb_status rc = apply_Tt<T>(op, w, (T *)op->xs);
    if (rc) return rc;
    hipLaunchKernelGGL((k_perm<T>), dim3(nblk(op->s.nsup, 256)), dim3(256), 0, op->st, op->lo, op->s.nsup, (const T *)op->xs, xs, 0);
    LAUNCHCHK();
    return IGB_OK;
}

template <class T>
static igb_status T_impl(igb_operator *op, const T *ys, T *y)
{
    hipLaunchKernelGGL((k_perm<T>), dim3(nblk(op->s.nsup, 256)), dim3(256), 0, op->st, op->lo, op->s.nsup, ys, (T *)op->ys, 1);
    LAUNCHCHK();
    return apply_T<T>(op, (const T *)op->ys, y);
}

igb_status igb_apply_Tt(const igb_operator *cop, const void *w_dev, void *xs_dev)
{
    CHECK_OP(cop);
    if (!w_dev || !xs_dev) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? Tt_impl<cd>(op, (const cd *)w_dev, (cd *)xs_dev) : Tt_impl<double>(op, (const double *)w_dev, (double *)xs_dev);
}

igb_status igb_apply_T(const igb_operator *cop, const void *ys_dev, void *y_dev)
{
    CHECK_OP(cop);
    if (!ys_dev || !y_dev) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? T_impl<cd>(op, (const cd *)ys_dev, (cd *)y_dev) : T_impl<double>(op, (const double *)ys_dev, (double *)y_dev);
}

igb_status igb_jacobi_diag(const igb_operator *op, void *d_dev)
{
    CHECK_OP(op);
    if (!d_dev) return fail(IGB_EINVAL, "d_dev is null");
    HIPCHK(hipMemcpyAsync(d_dev, op->diag, op->s.ndof * op->esz, hipMemcpyDeviceToDevice, op->st));
    return IGB_OK;
}

// Helmholtz with the single-precision far field (IGB_FP32): iterative refinement.
// Each cycle solves the correction equation A~ d = r with the device GMRES on the
// single-precision operator A~ to the relative tolerance tau, adds d to w, and
// forms r = b - A w with the FP64 operator; it stops when that residual meets
// rel_tol.  tau = max(1e-4, rel_tol / (2 |r| / |b|)): the last cycle is asked for
// no more than it has to gain.  Iterations count the single-precision products of
// the inner solves and the FP64 residual products.
static igb_status solve_refined(igb_operator *op, const cd *b, cd *w, double tol, int maxit, int restart,
                                igb_solve_info *info)
{
    const int64_t n = op->s.ndof;
    cd *r = (cd *)op->rr, *d = (cd *)op->dw;
    const unsigned gb = std::min<unsigned>(nblk(n, 256), 1024);
    igb_status rc;
    struct Restore {
        igb_operator *o;
        bool v;
        ~Restore() { o->force_fp64 = v; }
    } restore{op, op->force_fp64};
    auto norm = [&](const cd *x, double *out) -> igb_status {
        igb_status c;
        if ((c = dot_dev<cd>(op, n, x, x, (cd *)op->scal))) return c;
        if ((c = read_scalar(op, 0, out))) return c;
        *out = std::sqrt(*out);
        return IGB_OK;
    };
    double bn;
    if ((rc = norm(b, &bn))) return rc;
    if (bn == 0.0) bn = 1.0;
    int it = 0;
    double rel = 0.0;
    for (;;) {
        op->force_fp64 = true;
        if ((rc = matvec_S<cd>(op, w, d))) return rc;
        HIPCHK(hipMemcpyAsync(r, b, n * sizeof(cd), hipMemcpyDeviceToDevice, op->st));
        hipLaunchKernelGGL((k_axpby<cd>), dim3(gb), dim3(256), 0, op->st, n, cd{-1.0, 0.0}, (const cd *)d,
                           cd{1.0, 0.0}, r);
        LAUNCHCHK();
        double rn;
        if ((rc = norm(r, &rn))) return rc;
        ++it;
        rel = rn / bn;
        if (rel <= tol || it >= maxit) break;
        HIPCHK(hipMemsetAsync(d, 0, n * sizeof(cd), op->st));
        igb_solve_info in{};
        rc = solve_gmres_dev<cd>(op, nullptr, r, d, std::max(1e-4, 0.5 * tol / rel), maxit - it, restart, &in, false);
        if (rc < 0) return rc;
        it += in.iterations;
        hipLaunchKernelGGL((k_axpby<cd>), dim3(gb), dim3(256), 0, op->st, n, cd{1.0, 0.0}, (const cd *)d,
                           cd{1.0, 0.0}, w);
        LAUNCHCHK();
    }
    if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->converged = rel <= tol;
        info->fallback = 0;
    }
    return rel <= tol ? IGB_OK
                      : fail(IGB_ENOT_CONVERGED, "refinement stopped at max_iter with relative residual " +
                                                     std::to_string(rel));
}

igb_status igb_solve(const igb_operator *cop, const void *b_dev, void *w_dev, double rel_tol, int32_t max_iter,
                     int32_t restart, igb_solve_info *info)
{
    CHECK_OP(cop);
    if (!b_dev || !w_dev) return fail(IGB_EINVAL, "null device pointer");
    if (b_dev == w_dev) return fail(IGB_EINVAL, "b and w must not alias");
    if (!(rel_tol > 0.0) || max_iter < 0) return fail(IGB_EINVAL, "rel_tol must be > 0 and max_iter >= 0");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (op->cplx) {
        if (restart < 1 || restart > 2048) return fail(IGB_EINVAL, "restart must be in 1..2048");
        if (op->far_single)
            return solve_refined(op, (const cd *)b_dev, (cd *)w_dev, rel_tol, max_iter, restart, info);
        return solve_gmres_dev<cd>(op, nullptr, (const cd *)b_dev, (cd *)w_dev, rel_tol, max_iter, restart, info);
    }
    return solve_cg(op, (const double *)b_dev, (double *)w_dev, rel_tol, max_iter, info);
}

igb_status igb_solve_many(int32_t n, igb_operator *const *ops, const void *const *b_devs, void *const *w_devs,
                          double rel_tol, int32_t max_iter, int32_t restart, igb_solve_info *infos)
{
    if (n < 0) return fail(IGB_EINVAL, "n must be >= 0");
    if (n > 0 && (!ops || !b_devs || !w_devs)) return fail(IGB_EINVAL, "null argument");
    if (!(rel_tol > 0.0) || max_iter < 0) return fail(IGB_EINVAL, "rel_tol must be > 0 and max_iter >= 0");
    // entries of one operator form a group, solved one after another in list order (a solve uses its
    // operator's buffers); groups run concurrently
    std::vector<std::vector<int32_t>> groups;
    std::map<const igb_operator *, size_t> gid;
    for (int32_t i = 0; i < n; ++i) {
        if (!ops[i] || !b_devs[i] || !w_devs[i]) return fail(IGB_EINVAL, "null operator or vector at " + std::to_string(i));
        if (ops[i]->cplx && restart < 1) return fail(IGB_EINVAL, "restart must be >= 1");
        auto it = gid.emplace(ops[i], groups.size());
        if (it.second) groups.emplace_back();
        groups[it.first->second].push_back(i);
    }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            if (w_devs[i] == w_devs[j] && i != j) return fail(IGB_EINVAL, "entries " + std::to_string(i) + " and " +
                                                                              std::to_string(j) + " share a solution vector");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::vector<igb_status> st(n, IGB_OK);
    std::vector<std::string> msg(n);
    const int ng = (int)groups.size();
    std::atomic<int> next{0};
    auto worker = [&]() {
        if (hipSetDevice(dev) != hipSuccess) return;
        for (;;) {
            const int gi = next.fetch_add(1);
            if (gi >= ng) break;
            for (const int32_t i : groups[gi]) {
                igb_solve_info inf{};
                try {
                    st[i] = igb_solve(ops[i], b_devs[i], w_devs[i], rel_tol, max_iter, restart, &inf);
                    if (st[i] != IGB_OK) msg[i] = g_err;
                } catch (const std::exception &ex) {  // nothing may escape a worker thread
                    st[i] = IGB_ENOMEM;
                    msg[i] = std::string("host exception: ") + ex.what();
                }
                if (infos) infos[i] = inf;
            }
        }
    };
    const int nt = std::min<int>(ng, 16);
    std::vector<std::thread> th;
    try {
        for (int t = 0; t < nt; ++t) th.emplace_back(worker);
    } catch (const std::system_error &) {
        for (auto &x : th) x.join();
        return fail(IGB_ENOMEM, "could not start solver threads");
    }
    for (auto &x : th) x.join();
    if (next.load() < ng) return fail(IGB_EHIP, "hipSetDevice failed in a solver thread");
    igb_status worst = IGB_OK;
    int wi = -1;
    for (int32_t i = 0; i < n; ++i)
        if (st[i] < 0 && (worst >= 0 || st[i] < worst)) {
            worst = st[i];
            wi = i;
        } else if (st[i] > 0 && worst == IGB_OK) {
            worst = st[i];
            wi = i;
        }
    if (worst != IGB_OK) return fail(worst, "instance " + std::to_string(wi) + ": " + msg[wi]);
    return IGB_OK;
}

igb_status igb_solve_fgmres(const igb_operator *cop, const igb_cnn *net, const void *b_dev, void *w_dev,
                            double rel_tol, int32_t max_iter, int32_t restart, igb_solve_info *info)
{
    CHECK_OP(cop);
    if (!b_dev || !w_dev) return fail(IGB_EINVAL, "null device pointer");
    if (b_dev == w_dev) return fail(IGB_EINVAL, "b and w must not alias");
    if (!(rel_tol > 0.0) || max_iter < 0) return fail(IGB_EINVAL, "rel_tol must be > 0 and max_iter >= 0");
    if (restart < 1 || restart > 2048) return fail(IGB_EINVAL, "restart must be in 1..2048");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (op->cplx) return fail(IGB_EUNSUPPORTED, "flexible GMRES is built for real (Laplace) operators");
    return solve_gmres_dev<double>(op, net, (const double *)b_dev, (double *)w_dev, rel_tol, max_iter, restart, info);
}

igb_status igb_solve_fgmres_select(const igb_operator *cop, const igb_cnn *const *nets, int32_t n_nets,
                                   const void *v_dev, const void *b_dev, void *w_dev, double rel_tol,
                                   int32_t max_iter, int32_t restart, int32_t *chosen, igb_solve_info *info)
{
    CHECK_OP(cop);
    if (!v_dev || !b_dev || !w_dev || !chosen) return fail(IGB_EINVAL, "null argument");
    if (n_nets < 0 || (n_nets > 0 && !nets)) return fail(IGB_EINVAL, "n_nets must be >= 0 with a network array");
    for (int32_t i = 0; i < n_nets; ++i)
        if (!nets[i]) return fail(IGB_EINVAL, "null network at " + std::to_string(i));
    if (b_dev == w_dev || v_dev == w_dev) return fail(IGB_EINVAL, "b, v and w must not alias");
    if (!(rel_tol > 0.0) || max_iter < 0) return fail(IGB_EINVAL, "rel_tol must be > 0 and max_iter >= 0");
    if (restart < 1 || restart > 2048) return fail(IGB_EINVAL, "restart must be in 1..2048");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (op->cplx) return fail(IGB_EUNSUPPORTED, "flexible GMRES is built for real (Laplace) operators");
    const int64_t n = op->s.ndof;
    double *vw = (double *)op->pv;  // the CG direction vector, idle during flexible GMRES
    // validation: Jacobi first, then each network, all from a zero initial guess; a network is kept only if
    // it converges without falling back and in fewer steps than every earlier choice
    int32_t best = -1, best_it = 0;
    for (int32_t i = -1; i < n_nets; ++i) {
        HIPCHK(hipMemsetAsync(vw, 0, n * sizeof(double), op->st));
        igb_solve_info vi{};
        const igb_status rc = solve_gmres_dev<double>(op, i < 0 ? nullptr : nets[i], (const double *)v_dev, vw,
                                                      rel_tol, max_iter, restart, &vi);
        if (rc != IGB_OK && rc != IGB_ENOT_CONVERGED) return rc;
        if (i < 0)
            best_it = vi.converged ? vi.iterations : max_iter + 1;
        else if (vi.converged && !vi.fallback && vi.iterations < best_it) {
            best = i;
            best_it = vi.iterations;
        }
    }
    *chosen = best;
    return solve_gmres_dev<double>(op, best < 0 ? nullptr : nets[best], (const double *)b_dev, (double *)w_dev,
                                   rel_tol, max_iter, restart, info);
}

igb_status igb_cnn_train_operator(igb_cnn *net, const igb_operator *cop, const float *y_dev, const float *x_dev,
                                  int64_t n_pairs, int32_t epochs, int32_t batch, float lr, double *loss_host)
{
    CHECK_OP(cop);
    if (!net || !y_dev || !x_dev) return fail(IGB_EINVAL, "null argument");
    if (n_pairs < 1 || epochs < 0 || batch < 1) return fail(IGB_EINVAL, "n_pairs and batch must be >= 1, epochs >= 0");
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(IGB_EINVAL, "learning rate must be > 0");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (op->cplx) return fail(IGB_EUNSUPPORTED, "the network is built for real (Laplace) operators");
    struct Restore {
        igb_operator *o;
        bool v;
        ~Restore() { o->force_fp64 = v; }
    } restore{op, op->force_fp64};
    op->force_fp64 = true;
    const Setup &s = op->s;
    const int64_t n = s.ndof, b = std::min<int64_t>(batch, n_pairs);
    double *e = (double *)op->r, *t = (double *)op->tmp, *u = (double *)op->z;
    const double *D = (const double *)op->diag;
    const unsigned gb = std::min<unsigned>(nblk(n, 256), 1024);
    igb_status rc;
    for (int ep = 0; ep < epochs; ++ep) {
        double tot = 0.0;
        for (int64_t s0 = 0; s0 < n_pairs; s0 += b) {
            const int64_t nb = std::min(b, n_pairs - s0);
            float *f = nullptr, *dout = nullptr;
            if ((rc = cnn_batch_forward(net, y_dev + s0 * n, (int32_t)(nb * s.npatch), s.ns1, s.ns1, op->st, &f, &dout)))
                return rc;
            const double scale = 1.0 / (double)(nb * n);
            for (int64_t k = 0; k < nb; ++k) {
                // e = M(y) - x; u = D^-1 A e; loss += |u|^2; dL/dM(y) = A D^-1 u / N
                hipLaunchKernelGGL(k_err64, dim3(nblk(n, 256)), dim3(256), 0, op->st, n, y_dev + (s0 + k) * n,
                                   (const float *)f + k * n, x_dev + (s0 + k) * n, e);
                LAUNCHCHK();
                if ((rc = matvec_S<double>(op, e, t))) return rc;
                hipLaunchKernelGGL((k_div<double>), dim3(gb), dim3(256), 0, op->st, n, (const double *)t, D, u);
                LAUNCHCHK();
                double uu;
                if ((rc = dot_dev<double>(op, n, u, u, op->scal + 2))) return rc;
                if ((rc = read_scalar(op, 2, &uu))) return rc;
                tot += uu;
                hipLaunchKernelGGL((k_div<double>), dim3(gb), dim3(256), 0, op->st, n, (const double *)u, D, e);
                LAUNCHCHK();
                if ((rc = matvec_S<double>(op, e, t))) return rc;
                hipLaunchKernelGGL(k_grad32, dim3(nblk(n, 256)), dim3(256), 0, op->st, n, (const double *)t, scale,
                                   dout + k * n);
                LAUNCHCHK();
            }
            if ((rc = cnn_batch_backward_adam(net, y_dev + s0 * n, (int32_t)(nb * s.npatch), s.ns1, s.ns1, lr, op->st)))
                return rc;
        }
        if (loss_host) loss_host[ep] = tot / (2.0 * (double)(n_pairs * n));
    }
    HIPCHK(hipStreamSynchronize(op->st));
    return IGB_OK;
}

igb_status igb_cnn_training_pairs(const igb_operator *cop, const double *x_dev, int64_t n_pairs, float *y_dev,
                                  float *x32_dev)
{
    CHECK_OP(cop);
    if (!x_dev || !y_dev || !x32_dev) return fail(IGB_EINVAL, "null device pointer");
    if (n_pairs < 0) return fail(IGB_EINVAL, "n_pairs must be >= 0");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (op->cplx) return fail(IGB_EUNSUPPORTED, "training pairs are built for real (Laplace) operators");
    struct Restore {
        igb_operator *o;
        bool v;
        ~Restore() { o->force_fp64 = v; }
    } restore{op, op->force_fp64};
    op->force_fp64 = true;
    const int64_t n = op->s.ndof;
    igb_status rc;
    for (int64_t k = 0; k < n_pairs; ++k) {
        if ((rc = matvec_S<double>(op, x_dev + k * n, (double *)op->tmp))) return rc;
        hipLaunchKernelGGL(k_pairs_out, dim3(nblk(n, 256)), dim3(256), 0, op->st, n, (const double *)op->tmp,
                           (const double *)op->diag, x_dev + k * n, y_dev + k * n, x32_dev + k * n);
        LAUNCHCHK();
    }
    return IGB_OK;
}

// Source chunks of the potential's direct sum: enough (x, chunk) workgroups to fill the GPU, at most
// max_parts partial values (nchunk * npts) when max_parts > 0.
static int64_t potential_chunks(int64_t npts, int64_t nq, int64_t max_parts)
{
    const int64_t tb = (npts + 255) / 256;
    int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(4096 / tb + 1, (nq + 4095) / 4096));
    if (max_parts > 0) nchunk = std::max<int64_t>(1, std::min<int64_t>(nchunk, max_parts / npts));
    return nchunk;
}

// S -> S*, weighted density at the quadrature points, then the direct sum into
// nchunk partial values per point (part, nchunk * npts values) and their sum.
template <class T>
static igb_status potential_launch(igb_operator *op, const T *w, int64_t npts, const double *X, T *u, T *part,
                                   int64_t nchunk)
{
    const Setup &s = op->s;
    igb_status rc = apply_Tt<T>(op, w, (T *)op->xs);
    if (rc) return rc;
    const int64_t nq = (int64_t)s.nelem * s.grhs * s.grhs;
    hipLaunchKernelGGL((k_pot_prep<T>), dim3(nblk(nq, 256)), dim3(256), 0, op->st, op->lo, s.nelem, s.grhs,
                       op->gx + s.goff[s.grhs], op->rpts, (const T *)op->xs, (T *)op->potc);
    LAUNCHCHK();
    if (npts == 0) return IGB_OK;
    if (NComp<T>::value == 2 && !op->sctab) return fail(IGB_EHIP, "potential: sine/cosine table missing");
    const int64_t tb = (npts + 255) / 256, chunk = (nq + nchunk - 1) / nchunk;
    hipLaunchKernelGGL((k_pot_eval<T>), dim3((unsigned)tb, (unsigned)nchunk), dim3(256), 0, op->st, npts, X, nq, op->rpts,
                       (const T *)op->potc, s.kappa, chunk, part, (const double *)op->sctab, s.hull_c[0], s.hull_c[1],
                       s.hull_c[2], s.hull_r);
    LAUNCHCHK();
    hipLaunchKernelGGL((k_pot_reduce<T>), dim3((unsigned)tb), dim3(256), 0, op->st, npts, (int)nchunk, (const T *)part, u);
    LAUNCHCHK();
    return IGB_OK;
}

template <class T>
static igb_status potential_impl(igb_operator *op, const T *w, int64_t npts, const double *X, T *u)
{
    const Setup &s = op->s;
    const int64_t nq = (int64_t)s.nelem * s.grhs * s.grhs;
    if (npts == 0) return potential_launch<T>(op, w, npts, X, u, nullptr, 1);
    const int64_t nchunk = potential_chunks(npts, nq, 0);
    DevBlock pb{};
    HIPCHK(pool_alloc(pb, (size_t)nchunk * npts * sizeof(T)));
    const igb_status rc = potential_launch<T>(op, w, npts, X, u, (T *)pb.p, nchunk);
    const hipError_t e = hipStreamSynchronize(op->st);  // the partial sums go back to the pool afterwards
    if (e == hipSuccess) pool_free(pb);
    else (void)hipFree(pb.p);
    if (rc) return rc;
    if (e != hipSuccess) return fail(IGB_EHIP, "potential evaluation failed");
    return IGB_OK;
}

// The potential with the far field interpolated (k_pot_h2): density to S*, the upward pass to the moments,
// the weighted density at the quadrature points, then one wave per point.  Without far-field levels, or
// when a point's traversal overflows, the direct sum.
template <class T>
static igb_status potential_h2_impl(igb_operator *op, const T *w, int64_t npts, const double *X, T *u)
{
    const Setup &s = op->s;
    if (op->lmin > s.L || s.L > kH2MaxLevel || s.mode == IGB_DENSE) return potential_impl<T>(op, w, npts, X, u);
    if (npts == 0) return IGB_OK;
    if (NComp<T>::value == 2 && !op->sctab) return fail(IGB_EHIP, "potential: sine/cosine table missing");
    igb_status rc;
    const int64_t ncl_all = s.cl_off[s.L + 1];
    if (!op->clgeo) {  // first call: the cluster bounds of the far-field levels
        std::vector<double> h((size_t)ncl_all * 5 + 1, 0.0), lv;
        for (int l = op->lmin; l <= s.L; ++l) {
            cluster_spheres(s, l, lv);
            std::copy(lv.begin(), lv.end(), h.begin() + s.cl_off[l] * 5);
        }
        if ((rc = upload(op, &op->clgeo, h.data(), h.size() * sizeof(double)))) return rc;
        HIPCHK(hipStreamSynchronize(op->st));  // the host array goes out of scope
    }
    if ((rc = apply_Tt<T>(op, w, (T *)op->xs))) return rc;
    for (const TreeLaunch &t : tree_slices(op, sizeof(T))) {
        if (t.shm > 64 * 1024) {
            if (t.shm > 160 * 1024) return fail(IGB_EUNSUPPORTED, "cluster-tree transfers: q too large for LDS");
            (void)hipFuncSetAttribute((const void *)k_up_tree<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)t.shm);
        }
        hipLaunchKernelGGL((k_up_tree<T>), dim3(t.roots), dim3(64 * t.waves), t.shm, op->st, t.A, t.SL,
                           (const T *)op->xs, (T *)op->Xh);
        LAUNCHCHK();
    }
    const int64_t nq = (int64_t)s.nelem * s.grhs * s.grhs;
    hipLaunchKernelGGL((k_pot_prep<T>), dim3(nblk(nq, 256)), dim3(256), 0, op->st, op->lo, s.nelem, s.grhs,
                       op->gx + s.goff[s.grhs], op->rpts, (const T *)op->xs, (T *)op->potc);
    LAUNCHCHK();
    int *flag = (int *)(op->clgeo + (size_t)ncl_all * 5);
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), op->st));
    PotH2Args A{};
    A.lmin = op->lmin;
    A.L = s.L;
    A.npatch = s.npatch;
    A.q2 = s.q * s.q;
    A.ne = s.ne;
    A.side = s.side;
    A.gg = s.grhs * s.grhs;
    for (int l = 0; l <= s.L + 1; ++l) A.cl_off[l] = s.cl_off[l];
    A.clg = op->clgeo;
    A.nodes = op->nodes;
    A.Xh = op->Xh;
    A.rp = op->rpts;
    A.c = op->potc;
    A.eta = s.eta;
    A.kappa = s.kappa;
    A.kappa_diam = s.kernel == IGB_HELMHOLTZ
                       ? (s.kappa_diam > 0.0 ? std::min(s.kappa_diam, kPotKappaDiam) : kPotKappaDiam)
                       : __builtin_inf();
    A.hx = s.hull_c[0];
    A.hy = s.hull_c[1];
    A.hz = s.hull_c[2];
    A.hr = s.hull_r;
    A.tab = op->sctab;
    A.flag = flag;
    hipLaunchKernelGGL((k_pot_h2<T>), dim3((unsigned)((npts + 3) / 4)), dim3(256), 0, op->st, npts, X, A, u);
    LAUNCHCHK();
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
    if (hflag) return potential_impl<T>(op, w, npts, X, u);
    return IGB_OK;
}

// Scratch of igb_potential_noalloc: the partial sums of the potential's direct sum, a file-scope device
// array of kScratchBytes on every device the library runs on (held until the process ends).  Host code
// never passes the array's name to a kernel: on the first call on a device, with that device current, its
// address is taken with hipGetSymbolAddress and kept per device.
constexpr size_t kScratchBytes = 32u << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;

static igb_status scratch_address(int dev, void **ptr)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *ptr = it->second;
        return IGB_OK;
    }
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
        return fail(IGB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    *ptr = p;
    return IGB_OK;
}

igb_status igb_potential(const igb_operator *cop, const void *w_dev, int64_t n_pts, const double *xyz_dev, void *u_dev)
{
    CHECK_OP(cop);
    if (n_pts < 0) return fail(IGB_EINVAL, "n_pts < 0");
    if (!w_dev || (n_pts > 0 && (!xyz_dev || !u_dev))) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? potential_impl<cd>(op, (const cd *)w_dev, n_pts, xyz_dev, (cd *)u_dev)
                    : potential_impl<double>(op, (const double *)w_dev, n_pts, xyz_dev, (double *)u_dev);
}

igb_status igb_potential_noalloc(const igb_operator *cop, const void *w_dev, int64_t n_pts, const double *xyz_dev,
                                 void *u_dev)
{
    CHECK_OP(cop);
    if (n_pts < 0) return fail(IGB_EINVAL, "n_pts < 0");
    if (!w_dev || (n_pts > 0 && (!xyz_dev || !u_dev))) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    const size_t esz = op->cplx ? sizeof(cd) : sizeof(double);
    const int64_t cap = (int64_t)(kScratchBytes / esz);
    if (n_pts > cap)
        return fail(IGB_EINVAL, "igb_potential_noalloc: n_pts " + std::to_string(n_pts) + " exceeds the scratch capacity of " +
                                    std::to_string(cap) + " points");
    void *part = nullptr;
    igb_status rc = scratch_address(op->dev, &part);
    if (rc) return rc;
    const Setup &s = op->s;
    const int64_t nq = (int64_t)s.nelem * s.grhs * s.grhs;
    const int64_t nchunk = n_pts ? potential_chunks(n_pts, nq, cap) : 1;
    return op->cplx ? potential_launch<cd>(op, (const cd *)w_dev, n_pts, xyz_dev, (cd *)u_dev, (cd *)part, nchunk)
                    : potential_launch<double>(op, (const double *)w_dev, n_pts, xyz_dev, (double *)u_dev,
                                               (double *)part, nchunk);
}

igb_status igb_potential_h2(const igb_operator *cop, const void *w_dev, int64_t n_pts, const double *xyz_dev,
                            void *u_dev)
{
    CHECK_OP(cop);
    if (n_pts < 0) return fail(IGB_EINVAL, "n_pts < 0");
    if (!w_dev || (n_pts > 0 && (!xyz_dev || !u_dev))) return fail(IGB_EINVAL, "null device pointer");
    igb_operator *op = const_cast<igb_operator *>(cop);
    return op->cplx ? potential_h2_impl<cd>(op, (const cd *)w_dev, n_pts, xyz_dev, (cd *)u_dev)
                    : potential_h2_impl<double>(op, (const double *)w_dev, n_pts, xyz_dev, (double *)u_dev);
}

igb_status igb_export_partition(const igb_operator *op, int32_t *near_host, int32_t *far_host)
{
    CHECK_OP(op);
    if ((!near_host && !op->s.near.empty()) || (!far_host && !op->s.far.empty())) return fail(IGB_EINVAL, "null host pointer");
    if (!op->s.near.empty()) std::memcpy(near_host, op->s.near.data(), op->s.near.size() * sizeof(int32_t));
    if (!op->s.far.empty()) std::memcpy(far_host, op->s.far.data(), op->s.far.size() * sizeof(int32_t));
    return IGB_OK;
}

igb_status igb_export_pair_classes(const igb_operator *op, int32_t *pairs_host)
{
    CHECK_OP(op);
    if (!pairs_host && !op->s.pairs.empty()) return fail(IGB_EINVAL, "null host pointer");
    sorted_pair_classes(op->s, pairs_host);
    return IGB_OK;
}

igb_status igb_export_near_block(const igb_operator *op, int32_t E, int32_t F, double *blk_host)
{
    CHECK_OP(op);
    const Setup &s = op->s;
    if (!blk_host || E < 0 || F < 0 || E >= s.nelem || F >= s.nelem) return fail(IGB_EINVAL, "bad element index");
    auto leaf_of = [&](int e, int &el) {
        int pt = e / (s.ne * s.ne), r = e % (s.ne * s.ne), e2 = r / s.ne, e1 = r % s.ne, nL = 1 << s.L;
        el = (e2 % s.side) * s.side + e1 % s.side;
        return pt * nL * nL + (e2 / s.side) * nL + e1 / s.side;
    };
    int elE, elF;
    int lE = leaf_of(E, elE), lF = leaf_of(F, elF);
    int64_t e = csr_find_host(s, lE, lF);
    if (e < 0) return fail(IGB_EINVAL, "element pair is not in the near field");
    // a block that is not stored is read from its mirror, transposed
    int64_t k = op->sb_host[e];
    const bool tr = k < 0;
    if (tr) {
        int64_t m = csr_find_host(s, lF, lE);
        if (m < 0 || op->sb_host[m] < 0) return fail(IGB_EINVAL, "near-field block storage is inconsistent");
        k = op->sb_host[m];
    }
    const int ld = op->near_ld;
    size_t nb = (size_t)s.nl * ld;
    std::vector<unsigned char> buf(nb * op->esz);
    HIPCHK(hipStreamSynchronize(op->st));
    HIPCHK(hipMemcpy(buf.data(), (const char *)op->nearb + k * nb * op->esz, nb * op->esz, hipMemcpyDeviceToHost));
    int nc = op->cplx ? 2 : 1;
    const double *B = (const double *)buf.data();
    for (int a = 0; a < s.nloc; ++a)
        for (int c = 0; c < s.nloc; ++c) {
            int64_t pos = tr ? (int64_t)(elE * s.nloc + a) * ld + elF * s.nloc + c
                             : (int64_t)(elF * s.nloc + c) * ld + elE * s.nloc + a;
            for (int z = 0; z < nc; ++z) blk_host[(a * s.nloc + c) * nc + z] = B[pos * nc + z];
        }
    return IGB_OK;
}

igb_status igb_export_coupling_block(const igb_operator *op, int32_t level, int32_t tgt, int32_t src, double *blk_host)
{
    CHECK_OP(op);
    const Setup &s = op->s;
    if (!blk_host || level < 0 || level > s.L) return fail(IGB_EINVAL, "bad level");
    int64_t ncl = (int64_t)s.npatch << (2 * level);
    if (tgt < 0 || src < 0 || tgt >= ncl || src >= ncl) return fail(IGB_EINVAL, "bad cluster id");
    int64_t row = s.cl_off[level] + tgt;
    int32_t key = (int32_t)(s.cl_off[level] + src);
    auto b = s.far_src.begin() + s.far_ptr[row], e = s.far_src.begin() + s.far_ptr[row + 1];
    auto it = std::lower_bound(b, e, key);
    if (it == e || *it != key) return fail(IGB_EINVAL, "cluster pair is not a far block");
    int64_t k = it - s.far_src.begin();
    int q2 = s.q * s.q;
    size_t nb = (size_t)q2 * q2;
    std::vector<unsigned char> buf(nb * op->esz);
    HIPCHK(hipStreamSynchronize(op->st));
    if (s.mode == IGB_H2_STORED) {
        HIPCHK(hipMemcpy(buf.data(), (const char *)op->coup + k * nb * op->esz, nb * op->esz, hipMemcpyDeviceToHost));
    } else {
        // generate this one block with the coupling kernel
        int32_t hp[2] = {(int32_t)row, key};
        int32_t *dp = nullptr;
        void *db = nullptr;
        HIPCHK(hipMalloc((void **)&dp, sizeof hp));
        hipError_t e = hipMalloc(&db, nb * op->esz);
        if (e == hipSuccess) e = hipMemcpy(dp, hp, sizeof hp, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            if (op->cplx)
                hipLaunchKernelGGL((k_coupling<cd>), dim3(1), dim3(256), 0, op->st, (int64_t)1, dp, dp + 1, q2, op->nodes,
                                   s.kappa, (cd *)db);
            else
                hipLaunchKernelGGL((k_coupling<double>), dim3(1), dim3(256), 0, op->st, (int64_t)1, dp, dp + 1, q2,
                                   op->nodes, s.kappa, (double *)db);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(op->st);
        if (e == hipSuccess) e = hipMemcpy(buf.data(), db, nb * op->esz, hipMemcpyDeviceToHost);
        (void)hipFree(dp);
        (void)hipFree(db);
        if (e != hipSuccess) return fail(IGB_EHIP, std::string("coupling block export: ") + hipGetErrorString(e));
    }
    int nc = op->cplx ? 2 : 1;
    const double *B = (const double *)buf.data();
    for (int mu = 0; mu < q2; ++mu)
        for (int nu = 0; nu < q2; ++nu)
            for (int z = 0; z < nc; ++z) blk_host[((size_t)mu * q2 + nu) * nc + z] = B[((size_t)nu * q2 + mu) * nc + z];
    return IGB_OK;
}



// ---------------------------------------------------------------------------
// host-only planning
// ---------------------------------------------------------------------------
struct igb_plan {
    Setup s;
};

static void fill_info(const Setup &s, size_t esz, igb_info *out)
{
    std::memset(out, 0, sizeof(*out));
    out->n_dof = s.ndof;
    out->n_dof_super = s.nsup;
    out->n_elements = s.nelem;
    out->n_rhs_points = (int64_t)s.nelem * s.grhs * s.grhs;
    out->leaf_level = s.L;
    out->gauss_singular = s.gs;
    out->gauss_rhs = s.grhs;
    out->n_near_blocks = (int64_t)s.near_src.size();
    out->n_far_blocks = (int64_t)s.far_src.size();
    for (int c = 0; c < 4; ++c) out->n_pairs[c] = s.npairs_class[c];
    int64_t q2 = (int64_t)s.q * s.q, ncl = s.cl_off[s.L + 1];
    {
        NearLayout NL = near_layout(s, esz);
        out->near_bytes = NL.nsb * s.nl * NL.ld * (int64_t)esz;
        const bool fm = far_mirrored(s);
        out->layout_flags =
            (NL.sym ? 1 : 0) | (fm ? 2 : 0) | (fm && fused_products(NL.sym, s.nl, NL.ld, esz, s.q * s.q) ? 4 : 0);
    }
    out->coupling_bytes = s.mode == IGB_H2_STORED ? out->n_far_blocks * q2 * q2 * (int64_t)esz : 0;
    // one superspace matvec moves every stored block once, the S* vector in and
    // out, the moment vectors of all clusters, and (on the fly) the node data
    out->matvec_bytes = out->near_bytes + out->coupling_bytes + (int64_t)esz * (3 * s.nsup + 4 * q2 * ncl) +
                        (s.mode == IGB_H2_ONTHEFLY ? (int64_t)32 * q2 * ncl : 0);
    out->setup_seconds = s.setup_seconds;
    // quadrature points of the near-field pairs: g^4 per regular pair (orders g0, g0 + 2, g0 + 4 by the
    // pair's group), regions x gs^4 per touching pair (identical 4 integrated regions, edge 6, vertex 4)
    const int ords[3] = {s.g0, std::min(40, s.g0 + 2), std::min(40, s.g0 + 4)};
    for (int k = 0; k < 3; ++k) {
        const int64_t g2 = (int64_t)ords[k] * ords[k];
        out->quad_points_regular += (s.pair_off[k + 1] - s.pair_off[k]) * g2 * g2;
    }
    const int64_t gs4 = (int64_t)s.gs * s.gs * s.gs * s.gs;
    out->quad_points_touching = gs4 * (4 * s.npairs_class[1] + 6 * s.npairs_class[2] + 4 * s.npairs_class[3]);
}

igb_status igb_plan_create(const igb_geometry *geo, const igb_params *prm, igb_plan **out)
{
    if (!geo || !prm || !out) return fail(IGB_EINVAL, "null argument");
    *out = nullptr;
    igb_plan *pl = new igb_plan();
    std::string err = build_setup(geo->g, *prm, pl->s);
    if (!err.empty()) {
        delete pl;
        return fail(IGB_EINVAL, err);
    }
    *out = pl;
    return IGB_OK;
}

void igb_plan_destroy(igb_plan *plan) { delete plan; }

igb_status igb_plan_info(const igb_plan *plan, igb_info *out)
{
    if (!plan || !out) return fail(IGB_EINVAL, "null argument");
    fill_info(plan->s, plan->s.kernel == IGB_HELMHOLTZ ? sizeof(cd) : sizeof(double), out);
    return IGB_OK;
}

igb_status igb_plan_export_partition(const igb_plan *plan, int32_t *near_host, int32_t *far_host)
{
    if (!plan) return fail(IGB_EINVAL, "plan is null");
    const Setup &s = plan->s;
    if ((!near_host && !s.near.empty()) || (!far_host && !s.far.empty())) return fail(IGB_EINVAL, "null host pointer");
    if (!s.near.empty()) std::memcpy(near_host, s.near.data(), s.near.size() * sizeof(int32_t));
    if (!s.far.empty()) std::memcpy(far_host, s.far.data(), s.far.size() * sizeof(int32_t));
    return IGB_OK;
}

igb_status igb_plan_export_pair_classes(const igb_plan *plan, int32_t *pairs_host)
{
    if (!plan) return fail(IGB_EINVAL, "plan is null");
    const Setup &s = plan->s;
    if (!pairs_host && !s.pairs.empty()) return fail(IGB_EINVAL, "null host pointer");
    sorted_pair_classes(s, pairs_host);
    return IGB_OK;
}

// ---------------------------------------------------------------------------
// per-stage timing of the superspace matvec (HIP events on the operator stream)
// ---------------------------------------------------------------------------
template <class T>
static igb_status profile_impl(igb_operator *op, int reps, bool separate, double *ms)
{
    constexpr int NS = IGB_NUM_MATVEC_STAGES;
    hipEvent_t ev[NS + 1], evn[2];
    for (int k = 0; k <= NS; ++k) HIPCHK(hipEventCreate(&ev[k]));
    HIPCHK(hipEventCreate(&evn[0]));
    HIPCHK(hipEventCreate(&evn[1]));
    for (int k = 0; k < NS; ++k) ms[k] = 0.0;
    igb_status rc = IGB_OK;
    for (int r = 0; r < reps && rc == IGB_OK; ++r) {
        bool forked = false;
        rc = matvec_internal<T>(op, (const T *)op->xs, (T *)op->ys, ev, separate, evn, &forked);
        if (rc) break;
        if (hipEventSynchronize(ev[NS]) != hipSuccess) { rc = fail(IGB_EHIP, "event synchronize"); break; }
        float tn = 0.f;
        if (forked && hipEventElapsedTime(&tn, evn[0], evn[1]) != hipSuccess) {
            rc = fail(IGB_EHIP, "event elapsed");
            break;
        }
        for (int k = 0; k < NS; ++k) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[k], ev[k + 1]) != hipSuccess) { rc = fail(IGB_EHIP, "event elapsed"); break; }
            // forked: stage 3 is the near GEMV on the side stream (concurrent with stages 0-2); the wait
            // for it on the main stream is not a stage
            ms[k] += (forked && k == 3) ? tn : t;
        }
    }
    for (int k = 0; k <= NS; ++k) (void)hipEventDestroy(ev[k]);
    (void)hipEventDestroy(evn[0]);
    (void)hipEventDestroy(evn[1]);
    if (rc) return rc;
    for (int k = 0; k < IGB_NUM_MATVEC_STAGES; ++k) ms[k] /= reps;
    return IGB_OK;
}

igb_status igb_matvec_profile(const igb_operator *cop, int32_t reps, int32_t flags, double *stage_ms_host)
{
    CHECK_OP(cop);
    if (reps < 1 || !stage_ms_host) return fail(IGB_EINVAL, "reps < 1 or null output");
    igb_operator *op = const_cast<igb_operator *>(cop);
    if (flags & ~IGB_PROFILE_SEPARATE) return fail(IGB_EINVAL, "unknown profile flags");
    const bool sep = (flags & IGB_PROFILE_SEPARATE) != 0;
    return op->cplx ? profile_impl<cd>(op, reps, sep, stage_ms_host) : profile_impl<double>(op, reps, sep, stage_ms_host);
}
