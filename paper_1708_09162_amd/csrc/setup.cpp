// Host-side setup of libigabem: geometry validation, Bezier extraction by
// knot insertion, Gauss rules, Chebyshev moment/transfer tables, the per-patch
// cluster tree with its block partition (Sec. 4.1, Sec. 4.2 Def.) and the
// near-field element-pair work lists (Sec. 4 item 4).
#include "setup.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

namespace igb {

// A process-wide pool of worker threads, created on first use and kept until
// the process ends (never destroyed, so no thread outlives its state).  One
// parallel region runs at a time; a caller that finds the pool busy (another
// host thread inside a region) runs its chunks itself.
namespace {
class Pool {
  public:
    static Pool &get()
    {
        static Pool *p = new Pool();
        return *p;
    }
    int size() const { return (int)workers_.size() + 1; }
    // run job(c) for c in [0, n); the caller takes part
    template <class J>
    void run(int n, J &job)
    {
        std::unique_lock<std::mutex> region(region_, std::try_to_lock);
        if (!region.owns_lock() || n <= 1) {
            for (int c = 0; c < n; ++c) job(c);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            fn_ = [&job](int c) { job(c); };
            nchunk_ = n;
            next_.store(0);
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        int c, mine = 0;
        while ((c = next_.fetch_add(1)) < n) { job(c); ++mine; }
        std::unique_lock<std::mutex> g(mu_);
        done_ += mine;
        // every chunk ran and no worker still holds this region's job
        finished_.wait(g, [&] { return done_ == nchunk_ && active_ == 0; });
        fn_ = nullptr;
    }

  private:
    Pool()
    {
        unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
        for (unsigned i = 1; i < hw; ++i) workers_.emplace_back([this] { loop(); });
        for (auto &t : workers_) t.detach();
    }
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            std::function<void(int)> fn;
            int n;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return gen_ != seen; });
                seen = gen_;
                if (!fn_) continue;  // woke after that region had ended
                fn = fn_;
                n = nchunk_;
                ++active_;
            }
            int c, mine = 0;
            while ((c = next_.fetch_add(1)) < n) { fn(c); ++mine; }
            std::lock_guard<std::mutex> g(mu_);
            done_ += mine;
            --active_;
            if (done_ == nchunk_ && active_ == 0) finished_.notify_all();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex region_, mu_;
    std::condition_variable cv_, finished_;
    std::function<void(int)> fn_;
    std::atomic<int> next_{0};
    int nchunk_ = 0, done_ = 0, active_ = 0;
    uint64_t gen_ = 0;
};
}  // namespace

// Run f(begin, end, chunk) over [0, n) split into contiguous chunks (at most
// max_chunks, at most one per pool thread).  Results that must stay ordered
// are written per chunk by the callers and concatenated in chunk order.
template <class F>
static void parallel_chunks(int64_t n, int max_chunks, F f)
{
    int nch = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)Pool::get().size(), (int64_t)max_chunks, n}));
    if (nch <= 1 || n < 64) {
        f((int64_t)0, n, 0);
        return;
    }
    auto job = [&](int c) { f(n * c / nch, n * (c + 1) / nch, c); };
    Pool::get().run(nch, job);
}

static int num_workers(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)Pool::get().size(), n));
}

// ---------------------------------------------------------------------------
// Gauss-Legendre on [0,1]: Newton on P_n from Chebyshev-like initial guesses.
// ---------------------------------------------------------------------------
void gauss_rule(int n, double *x, double *w)
{
    for (int k = 0; k < (n + 1) / 2; ++k) {
        double t = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * n + 2.0));
        double pn = 0, dpn = 1;
        for (int it = 0; it < 60; ++it) {
            double a = 1.0, b = t;  // P_0, P_1
            for (int j = 2; j <= n; ++j) {
                double c = ((2 * j - 1) * t * b - (j - 1) * a) / j;
                a = b;
                b = c;
            }
            pn = (n == 1) ? t : b;
            double pm = (n == 1) ? 1.0 : a;
            dpn = n * (pm - t * pn) / (1.0 - t * t);
            double step = pn / dpn;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        {
            double a = 1.0, b = t;
            for (int j = 2; j <= n; ++j) {
                double c = ((2 * j - 1) * t * b - (j - 1) * a) / j;
                a = b;
                b = c;
            }
            pn = (n == 1) ? t : b;
            double pm = (n == 1) ? 1.0 : a;
            dpn = n * (pm - t * pn) / (1.0 - t * t);
        }
        double wt = 1.0 / ((1.0 - t * t) * dpn * dpn);  // half of the [-1,1] weight
        // t is the k-th largest root; mirror pairs
        x[n - 1 - k] = 0.5 * (1.0 + t);
        w[n - 1 - k] = wt;
        x[k] = 0.5 * (1.0 - t);
        w[k] = wt;
    }
    if (n % 2 == 1) x[n / 2] = 0.5;
}

// ---------------------------------------------------------------------------
// geometry validation
// ---------------------------------------------------------------------------
static bool p_open(const double *U, int n, int p, std::string &why)
{
    int nk = n + p + 1;
    for (int i = 0; i < nk; ++i)
        if (!std::isfinite(U[i])) { why = "non-finite knot"; return false; }
    for (int i = 0; i + 1 < nk; ++i)
        if (U[i + 1] < U[i]) { why = "decreasing knot vector"; return false; }
    for (int i = 0; i <= p; ++i)
        if (U[i] != 0.0 || U[nk - 1 - i] != 1.0) { why = "knot vector is not p-open on [0,1]"; return false; }
    for (int i = p + 1; i < n; ++i) {
        int mult = 1;
        while (i + mult < n && U[i + mult] == U[i]) ++mult;
        if (mult > p && p > 0) { why = "interior knot multiplicity exceeds the degree"; return false; }
        if (U[i] <= 0.0 || U[i] >= 1.0) { why = "interior knot outside (0,1)"; return false; }
    }
    return true;
}

std::string make_geometry(int32_t n, const igb_nurbs_patch *in, Geometry &out)
{
    if (n < 1 || !in) return "n_patches < 1 or null patch array";
    out.patches.clear();
    for (int i = 0; i < n; ++i) {
        const igb_nurbs_patch &s = in[i];
        if (!s.knots_u || !s.knots_v || !s.cpw) return "patch " + std::to_string(i) + ": null pointer";
        if (s.deg_u < 0 || s.deg_u > 8 || s.deg_v < 0 || s.deg_v > 8)
            return "patch " + std::to_string(i) + ": degree outside 0..8";
        if (s.n_u < s.deg_u + 1 || s.n_v < s.deg_v + 1 || s.n_u > 4096 || s.n_v > 4096)
            return "patch " + std::to_string(i) + ": control point count";
        std::string why;
        if (!p_open(s.knots_u, s.n_u, s.deg_u, why)) return "patch " + std::to_string(i) + " u: " + why;
        if (!p_open(s.knots_v, s.n_v, s.deg_v, why)) return "patch " + std::to_string(i) + " v: " + why;
        Patch P;
        P.pu = s.deg_u;
        P.pv = s.deg_v;
        P.nu = s.n_u;
        P.nv = s.n_v;
        P.U.assign(s.knots_u, s.knots_u + s.n_u + s.deg_u + 1);
        P.V.assign(s.knots_v, s.knots_v + s.n_v + s.deg_v + 1);
        P.cpw.assign(s.cpw, s.cpw + (size_t)4 * s.n_u * s.n_v);
        for (size_t k = 0; k < P.cpw.size(); ++k)
            if (!std::isfinite(P.cpw[k])) return "patch " + std::to_string(i) + ": non-finite control data";
        for (size_t k = 3; k < P.cpw.size(); k += 4)
            if (!(P.cpw[k] > 0.0)) return "patch " + std::to_string(i) + ": weight <= 0";
        out.patches.push_back(std::move(P));
    }
    return "";
}

// ---------------------------------------------------------------------------
// Bezier extraction by repeated knot insertion (Boehm).  Returns, for a
// degree-p spline space with knots U (n functions), the matrix M (rows =
// functions of the refined space with every breakpoint k/ne at multiplicity p,
// columns = original functions): N_j = sum_k M[k][j] N'_k.  On element e the
// refined functions e*p .. e*p+p are the Bernstein polynomials of degree p.
// ---------------------------------------------------------------------------
static std::string extraction(int p, const std::vector<double> &U0, int n0, int ne, std::vector<double> &M, int &nr)
{
    std::vector<double> U = U0;
    int n = n0;
    // interior knots must lie on the grid
    for (int i = p + 1; i < n; ++i) {
        double t = U[i] * ne;
        if (std::fabs(t - std::round(t)) > 1e-12) return "interior knot off the refinement grid k/2^m";
        U[i] = std::round(t) / ne;
    }
    M.assign((size_t)n * n0, 0.0);
    for (int i = 0; i < n; ++i) M[(size_t)i * n0 + i] = 1.0;
    if (p == 0) {
        // piecewise constants: every breakpoint once
        for (int k = 1; k < ne; ++k) {
            double t = (double)k / ne;
            int span = -1;
            for (int i = 0; i + 1 < (int)U.size(); ++i)
                if (U[i] <= t && t < U[i + 1]) span = i;
            if (U[span] == t) continue;
            // insert: function span is split into two copies
            std::vector<double> Mn((size_t)(n + 1) * n0);
            for (int i = 0; i <= n; ++i) {
                int src = i <= span ? i : i - 1;
                std::memcpy(&Mn[(size_t)i * n0], &M[(size_t)src * n0], sizeof(double) * n0);
            }
            M.swap(Mn);
            U.insert(U.begin() + span + 1, t);
            ++n;
        }
        nr = n;
        return "";
    }
    for (int k = 1; k < ne; ++k) {
        double t = (double)k / ne;
        int mult = 0;
        for (double u : U)
            if (u == t) ++mult;
        for (int rep = mult; rep < p; ++rep) {
            int span = 0;
            for (int i = 0; i + 1 < (int)U.size(); ++i)
                if (U[i] <= t && t < U[i + 1]) span = i;
            std::vector<double> Mn((size_t)(n + 1) * n0, 0.0);
            for (int i = 0; i <= n; ++i) {
                double *row = &Mn[(size_t)i * n0];
                if (i <= span - p) {
                    std::memcpy(row, &M[(size_t)i * n0], sizeof(double) * n0);
                } else if (i >= span + 1) {
                    std::memcpy(row, &M[(size_t)(i - 1) * n0], sizeof(double) * n0);
                } else {
                    double a = (t - U[i]) / (U[i + p] - U[i]);
                    for (int c = 0; c < n0; ++c) row[c] = a * M[(size_t)i * n0 + c] + (1.0 - a) * M[(size_t)(i - 1) * n0 + c];
                }
            }
            M.swap(Mn);
            U.insert(U.begin() + span + 1, t);
            ++n;
        }
    }
    nr = n;
    if (nr != p * ne + 1) return "extraction produced an unexpected number of functions";
    return "";
}

// Bernstein values and derivatives of degree p at t
static inline void bern(int p, double t, double *B, double *dB)
{
    double s = 1.0 - t;
    // values of degree p-1 for the derivative
    double lo[16];
    if (p == 0) {
        B[0] = 1.0;
        if (dB) dB[0] = 0.0;
        return;
    }
    lo[0] = 1.0;
    for (int k = 1; k < p; ++k) {
        lo[k] = 0.0;
        for (int i = k; i >= 1; --i) lo[i] = s * lo[i] + t * lo[i - 1];
        lo[0] = s * lo[0];
    }
    // degree p from degree p-1
    B[p] = t * lo[p - 1];
    for (int i = p - 1; i >= 1; --i) B[i] = s * lo[i] + t * lo[i - 1];
    B[0] = s * lo[0];
    if (dB) {
        dB[0] = -p * lo[0];
        for (int i = 1; i < p; ++i) dB[i] = p * (lo[i - 1] - lo[i]);
        dB[p] = p * lo[p - 1];
    }
}

void tile_eval(const Setup &s, int E, double u, double v, double X[3], double *kap)
{
    int pu = s.tile_deg[2 * E], pv = s.tile_deg[2 * E + 1];
    const double *H = &s.tiles[(size_t)E * s.tile_stride];
    double Bu[16], dBu[16], Bv[16], dBv[16];
    bern(pu, u, Bu, dBu);
    bern(pv, v, Bv, dBv);
    if (!kap) {  // position only: the same sums for S, no tangents
        double S[4] = {0, 0, 0, 0};
        for (int j = 0; j <= pv; ++j) {
            double A[4] = {0, 0, 0, 0};
            for (int i = 0; i <= pu; ++i) {
                const double *h = H + 4 * (j * (pu + 1) + i);
                for (int c = 0; c < 4; ++c) A[c] += Bu[i] * h[c];
            }
            for (int c = 0; c < 4; ++c) S[c] += Bv[j] * A[c];
        }
        const double iw = 1.0 / S[3];
        for (int c = 0; c < 3; ++c) X[c] = S[c] * iw;
        return;
    }
    double S[4] = {0, 0, 0, 0}, Su[4] = {0, 0, 0, 0}, Sv[4] = {0, 0, 0, 0};
    for (int j = 0; j <= pv; ++j) {
        double A[4] = {0, 0, 0, 0}, Ad[4] = {0, 0, 0, 0};
        for (int i = 0; i <= pu; ++i) {
            const double *h = H + 4 * (j * (pu + 1) + i);
            for (int c = 0; c < 4; ++c) {
                A[c] += Bu[i] * h[c];
                Ad[c] += dBu[i] * h[c];
            }
        }
        for (int c = 0; c < 4; ++c) {
            S[c] += Bv[j] * A[c];
            Su[c] += Bv[j] * Ad[c];
            Sv[c] += dBv[j] * A[c];
        }
    }
    double iw = 1.0 / S[3];
    double x[3], xu[3], xv[3];
    for (int c = 0; c < 3; ++c) {
        x[c] = S[c] * iw;
        xu[c] = (Su[c] - x[c] * Su[3]) * iw;
        xv[c] = (Sv[c] - x[c] * Sv[3]) * iw;
    }
    X[0] = x[0];
    X[1] = x[1];
    X[2] = x[2];
    if (kap) {
        double n0 = xu[1] * xv[2] - xu[2] * xv[1];
        double n1 = xu[2] * xv[0] - xu[0] * xv[2];
        double n2 = xu[0] * xv[1] - xu[1] * xv[0];
        *kap = std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    }
}

// point at patch parameter (u, v) via the element tiles
static void patch_point(const Setup &s, int patch, double u, double v, double X[3])
{
    double a = u * s.ne, b = v * s.ne;
    int e1 = (int)std::floor(a), e2 = (int)std::floor(b);
    e1 = std::min(std::max(e1, 0), s.ne - 1);
    e2 = std::min(std::max(e2, 0), s.ne - 1);
    int E = patch * s.ne * s.ne + e2 * s.ne + e1;
    tile_eval(s, E, a - e1, b - e2, X, nullptr);
}

static inline double dist(const double *a, const double *b)
{
    double x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
    return std::sqrt(x * x + y * y + z * z);
}

// Lagrange basis polynomial mu on the Chebyshev nodes z, evaluated at t
static double lagr(const std::vector<double> &z, int mu, double t)
{
    double r = 1.0;
    for (size_t k = 0; k < z.size(); ++k)
        if ((int)k != mu) r *= (t - z[k]) / (z[mu] - z[k]);
    return r;
}

// ---------------------------------------------------------------------------
// the partition: level-synchronous recursion over block pairs
// ---------------------------------------------------------------------------
namespace {
struct LevelGeo {
    std::vector<double> pts;   // ncl*25*3
    std::vector<double> diam;  // ncl
    std::vector<double> cen;   // ncl*3 (grid centre point)
    std::vector<double> rad;   // ncl (max distance centre -> grid point)
};
}  // namespace

static void level_geo(const Setup &s, int l, LevelGeo &G)
{
    int n = 1 << l;
    int ncl = s.npatch * n * n;
    G.pts.resize((size_t)ncl * 75);
    G.diam.resize(ncl);
    G.cen.resize((size_t)ncl * 3);
    G.rad.resize(ncl);
    double sc = 1.0 / n;
    parallel_chunks(ncl, 64, [&](int64_t cb, int64_t ce, int) {
    for (int c = (int)cb; c < (int)ce; ++c) {
        int patch = c / (n * n), r = c % (n * n), k2 = r / n, k1 = r % n;
        double *P = &G.pts[(size_t)c * 75];
        for (int b = 0; b < 5; ++b)
            for (int a = 0; a < 5; ++a) patch_point(s, patch, (k1 + 0.25 * a) * sc, (k2 + 0.25 * b) * sc, P + 3 * (b * 5 + a));
        double d = 0.0;
        for (int i = 0; i < 25; ++i)
            for (int j = i + 1; j < 25; ++j) d = std::max(d, dist(P + 3 * i, P + 3 * j));
        G.diam[c] = d;
        const double *C = P + 3 * 12;
        G.cen[3 * c] = C[0];
        G.cen[3 * c + 1] = C[1];
        G.cen[3 * c + 2] = C[2];
        double rr = 0.0;
        for (int i = 0; i < 25; ++i) rr = std::max(rr, dist(C, P + 3 * i));
        G.rad[c] = rr;
    }
    });
}

// admissibility max(diam) < eta * dist over the 5x5 grids (bounds decide clear cases); with the
// wavenumber option also kappa * max(diam) <= kappa_diam, so that no admissible cluster spans more than
// kappa_diam / (2 pi) wavelengths
static bool admissible(const Setup &s, const LevelGeo &G, int a, int b)
{
    double md = std::max(G.diam[a], G.diam[b]);
    if (s.kappa_diam > 0.0 && s.kappa * md > s.kappa_diam) return false;
    double cc = dist(&G.cen[3 * a], &G.cen[3 * b]);
    double lb = cc - G.rad[a] - G.rad[b];
    if (lb > 0 && md < s.eta * lb * (1.0 - 1e-12)) return true;
    if (md > s.eta * cc * (1.0 + 1e-12)) return false;
    // md < eta * min_ij |A_i - B_j| holds iff it holds for every pair (i, j)
    // (rounded sqrt and product are monotone); rows of A whose distance bound
    // to B's sphere clears the threshold with margin are skipped
    const double *A = &G.pts[(size_t)a * 75], *B = &G.pts[(size_t)b * 75];
    const double thr = md / s.eta * (1.0 + 1e-12);
    for (int i = 0; i < 25; ++i) {
        if (dist(A + 3 * i, &G.cen[3 * b]) - G.rad[b] > thr) continue;
        for (int j = 0; j < 25; ++j)
            if (!(md < s.eta * dist(A + 3 * i, B + 3 * j))) return false;
    }
    return true;
}

void cluster_spheres(const Setup &s, int l, std::vector<double> &out)
{
    LevelGeo G;
    level_geo(s, l, G);
    const size_t ncl = G.rad.size();
    out.resize(ncl * 5);
    for (size_t c = 0; c < ncl; ++c) {
        out[5 * c] = G.cen[3 * c];
        out[5 * c + 1] = G.cen[3 * c + 1];
        out[5 * c + 2] = G.cen[3 * c + 2];
        out[5 * c + 3] = G.rad[c];
        out[5 * c + 4] = G.diam[c];
    }
}

static void build_partition(Setup &s)
{
    struct BP { int32_t t, src; };
    std::vector<BP> cur;
    for (int i = 0; i < s.npatch; ++i)
        for (int j = 0; j < s.npatch; ++j) cur.push_back({i, j});
    s.near.clear();
    s.far.clear();
    for (int l = 0; l <= s.L; ++l) {
        LevelGeo G;
        bool dense = (s.mode == IGB_DENSE);
        if (!dense) level_geo(s, l, G);
        std::vector<BP> nxt;
        nxt.reserve(l < s.L ? 16 * cur.size() : 0);
        int n = 1 << l, nn = 2 * n;
        std::vector<char> adm(cur.size(), 0);
        if (!dense)
            parallel_chunks((int64_t)cur.size(), 1 << 30, [&](int64_t b, int64_t e, int) {
                for (int64_t k = b; k < e; ++k) adm[k] = admissible(s, G, cur[k].t, cur[k].src) ? 1 : 0;
            });
        for (size_t k = 0; k < cur.size(); ++k) {
            const BP &bp = cur[k];
            if (adm[k]) {
                s.far.push_back(l);
                s.far.push_back(bp.t);
                s.far.push_back(bp.src);
            } else if (l == s.L) {
                s.near.push_back(bp.t);
                s.near.push_back(bp.src);
            } else {
                int pt = bp.t / (n * n), rt = bp.t % (n * n), t2 = rt / n, t1 = rt % n;
                int ps = bp.src / (n * n), rs = bp.src % (n * n), s2 = rs / n, s1 = rs % n;
                for (int a2 = 0; a2 < 2; ++a2)
                    for (int a1 = 0; a1 < 2; ++a1)
                        for (int b2 = 0; b2 < 2; ++b2)
                            for (int b1 = 0; b1 < 2; ++b1)
                                nxt.push_back({pt * nn * nn + (2 * t2 + a2) * nn + 2 * t1 + a1,
                                               ps * nn * nn + (2 * s2 + b2) * nn + 2 * s1 + b1});
            }
        }
        cur.swap(nxt);
    }
    // CSR by target (counting sort), sources ascending within a row: the order
    // of (target, source) for the near list and (level, target, source) for
    // the far list; both lists are then rewritten in that order
    {
        const size_t nb = s.near.size() / 2;
        s.near_ptr.assign(s.nleaf + 1, 0);
        for (size_t k = 0; k < nb; ++k) s.near_ptr[s.near[2 * k] + 1]++;
        for (int i = 0; i < s.nleaf; ++i) s.near_ptr[i + 1] += s.near_ptr[i];
        s.near_src.assign(nb, 0);
        std::vector<int64_t> fill(s.near_ptr.begin(), s.near_ptr.end() - 1);
        for (size_t k = 0; k < nb; ++k) s.near_src[fill[s.near[2 * k]]++] = s.near[2 * k + 1];
        parallel_chunks(s.nleaf, 1 << 30, [&](int64_t b, int64_t e, int) {
            for (int64_t t = b; t < e; ++t)
                std::sort(s.near_src.begin() + s.near_ptr[t], s.near_src.begin() + s.near_ptr[t + 1]);
        });
        for (int64_t t = 0; t < s.nleaf; ++t)
            for (int64_t k = s.near_ptr[t]; k < s.near_ptr[t + 1]; ++k) {
                s.near[2 * k] = (int32_t)t;
                s.near[2 * k + 1] = s.near_src[k];
            }
    }
    {
        const size_t nb = s.far.size() / 3;
        const int64_t ncl_all = s.cl_off[s.L + 1];
        s.far_ptr.assign(ncl_all + 1, 0);
        for (size_t k = 0; k < nb; ++k) s.far_ptr[s.cl_off[s.far[3 * k]] + s.far[3 * k + 1] + 1]++;
        for (int64_t i = 0; i < ncl_all; ++i) s.far_ptr[i + 1] += s.far_ptr[i];
        s.far_src.assign(nb, 0);
        std::vector<int64_t> fill(s.far_ptr.begin(), s.far_ptr.end() - 1);
        for (size_t k = 0; k < nb; ++k) {
            const int l = s.far[3 * k];
            s.far_src[fill[s.cl_off[l] + s.far[3 * k + 1]]++] = (int32_t)(s.cl_off[l] + s.far[3 * k + 2]);
        }
        parallel_chunks(ncl_all, 1 << 30, [&](int64_t b, int64_t e, int) {
            for (int64_t g = b; g < e; ++g) std::sort(s.far_src.begin() + s.far_ptr[g], s.far_src.begin() + s.far_ptr[g + 1]);
        });
        for (int l = 0; l <= s.L; ++l)
            for (int64_t g = s.cl_off[l]; g < s.cl_off[l + 1]; ++g)
                for (int64_t k = s.far_ptr[g]; k < s.far_ptr[g + 1]; ++k) {
                    s.far[3 * k] = l;
                    s.far[3 * k + 1] = (int32_t)(g - s.cl_off[l]);
                    s.far[3 * k + 2] = (int32_t)(s.far_src[k] - s.cl_off[l]);
                }
    }
}

// ---------------------------------------------------------------------------
// near-field element pairs: classification and frames (same reading as the
// paper's "order raised towards the singularity"; see build notes)
// ---------------------------------------------------------------------------
static const int kCorner[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};

static int other_adjacent(int o, int a)
{
    int n1 = (o + 1) & 3, n2 = (o + 3) & 3;
    return a == n1 ? n2 : n1;
}

// element corners (physical), 3x3 grids and grid diameters, used by the
// touching test and the regular-pair order
static void element_geometry_one(Setup &s, int E)
{
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) tile_eval(s, E, 0.5 * a, 0.5 * b, &s.egrid[(size_t)E * 27 + 3 * (3 * b + a)], nullptr);
    // the corners are grid points (same parameters, same values)
    for (int c = 0; c < 4; ++c)
        std::memcpy(&s.ecorner[(size_t)E * 12 + 3 * c], &s.egrid[(size_t)E * 27 + 3 * (3 * 2 * kCorner[c][1] + 2 * kCorner[c][0])],
                    3 * sizeof(double));
    double d = 0.0;
    for (int i = 0; i < 9; ++i)
        for (int j = i + 1; j < 9; ++j) d = std::max(d, dist(&s.egrid[(size_t)E * 27 + 3 * i], &s.egrid[(size_t)E * 27 + 3 * j]));
    s.ediam[E] = d;
    // bounding sphere of the 3x3 grid about its centre point
    const double *C = &s.egrid[(size_t)E * 27 + 12];
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r = std::max(r, dist(C, &s.egrid[(size_t)E * 27 + 3 * i]));
    s.erad[E] = r;
}

// Classification of one element pair E <= F (class, Gauss order, canonical frames).
// Touching is decided physically: corners coincide within 1e-10 * max diam.
static void classify_pair(const Setup &s, int E, int F, PairRec &R, bool touching_only = false)
{
    R.E = E;
    R.F = F;
    R.oE = 0; R.aE = 1; R.bE = 3; R.oF = 0; R.aF = 1; R.bF = 3;
    double md = std::max(s.ediam[E], s.ediam[F]);
    if (E == F) {
        R.cls = kIdentical;
        R.order = s.gs;
        return;
    }
    const double *cE = &s.ecorner[(size_t)E * 12], *cF = &s.ecorner[(size_t)F * 12];
    double tol = 1e-10 * md;
    // lower bound on every grid-point distance from the two bounding spheres
    // (corners are grid points); it settles most pairs without the full search
    double cc = dist(&s.egrid[(size_t)E * 27 + 12], &s.egrid[(size_t)F * 27 + 12]);
    double lb = cc - s.erad[E] - s.erad[F] - 1e-14 * cc;
    if (lb > tol) {
        R.cls = kRegular;
        if (touching_only) {
            R.order = s.g0;
            return;
        }
        if (lb >= 1.2 * md * (1.0 + 1e-12)) {
            R.order = s.g0;
            return;
        }
    }
    int match[4], nsh = 0;
    for (int c = 0; c < 4; ++c) {
        match[c] = -1;
        for (int dd = 0; dd < 4; ++dd)
            if (dist(cE + 3 * c, cF + 3 * dd) <= tol) match[c] = dd;
        if (match[c] >= 0) ++nsh;
    }
    if (nsh == 2) {
        int i = -1, j = -1;
        for (int c = 0; c < 4; ++c)
            if (match[c] >= 0) { if (i < 0) i = c; else j = c; }
        R.cls = kEdge;
        R.order = s.gs;
        R.oE = i; R.aE = j; R.bE = other_adjacent(i, j);
        R.oF = match[i]; R.aF = match[j]; R.bF = other_adjacent(match[i], match[j]);
        return;
    }
    if (nsh == 1) {
        int i = 0;
        for (int c = 0; c < 4; ++c)
            if (match[c] >= 0) i = c;
        R.cls = kVertex;
        R.order = s.gs;
        R.oE = i; R.aE = (i + 1) & 3; R.bE = (i + 3) & 3;
        int kk = match[i];
        R.oF = kk; R.aF = (kk + 1) & 3; R.bF = (kk + 3) & 3;
        return;
    }
    R.cls = kRegular;
    R.order = s.g0;
    if (touching_only) return;
    const double *gE = &s.egrid[(size_t)E * 27], *gF = &s.egrid[(size_t)F * 27];
    double dmin = 1e300;
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b) dmin = std::min(dmin, dist(gE + 3 * a, gF + 3 * b));
    double r = dmin / md;
    int g = s.g0;
    if (r < 0.6) g = s.g0 + 4;
    else if (r < 1.2) g = s.g0 + 2;
    if (g > 40) g = 40;
    R.cls = kRegular;
    R.order = g;
}

std::string enumerate_touching(const Setup &s, std::vector<PairRec> &out, bool with_identical)
{
    out.clear();
    double dmin = 1e300, dmax = 0.0;
    for (double d : s.ediam) { dmin = std::min(dmin, d); dmax = std::max(dmax, d); }
    if (!(dmax > 0.0)) return "degenerate elements (zero diameter)";
    // Corners are binned on a grid of cell size dmin/4.  Two corners within the
    // touching tolerance (at most 1e-10 dmax apart) share a cell unless one of
    // them lies within that tolerance of a cell face; only then are the
    // neighbouring cells across that face searched as well.
    const double cell = (dmin > 0.0 ? dmin : dmax) * 0.25;
    const double margin = 4e-10 * dmax / cell + 1e-12;
    auto cell_hash = [](int64_t i, int64_t j, int64_t k) {
        uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)j * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
        h ^= (uint64_t)k * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
        return h;
    };
    const int64_t ncorner = (int64_t)s.nelem * 4;
    std::vector<std::pair<uint64_t, int32_t>> tab(ncorner);
    parallel_chunks(ncorner, 1 << 30, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k) {
            const double *x = &s.ecorner[(size_t)k * 3];
            tab[k] = {cell_hash((int64_t)std::floor(x[0] / cell), (int64_t)std::floor(x[1] / cell),
                                (int64_t)std::floor(x[2] / cell)),
                      (int32_t)(k / 4)};
        }
    });
    std::sort(tab.begin(), tab.end());
    int nw = num_workers(s.nelem / 64 + 1);
    std::vector<std::vector<PairRec>> part(nw);
    parallel_chunks(s.nelem, nw, [&](int64_t eb, int64_t ee, int w) {
        std::vector<int32_t> cand;
        for (int E = (int)eb; E < (int)ee; ++E) {
            cand.clear();
            for (int c = 0; c < 4; ++c) {
                const double *x = &s.ecorner[(size_t)E * 12 + 3 * c];
                int64_t id[3];
                int lo[3], hi[3];
                for (int a = 0; a < 3; ++a) {
                    double t = x[a] / cell, f = std::floor(t);
                    id[a] = (int64_t)f;
                    lo[a] = (t - f < margin) ? -1 : 0;
                    hi[a] = (t - f > 1.0 - margin) ? 1 : 0;
                }
                for (int dx = lo[0]; dx <= hi[0]; ++dx)
                    for (int dy = lo[1]; dy <= hi[1]; ++dy)
                        for (int dz = lo[2]; dz <= hi[2]; ++dz) {
                            uint64_t h = cell_hash(id[0] + dx, id[1] + dy, id[2] + dz);
                            auto it = std::lower_bound(tab.begin(), tab.end(), std::make_pair(h, (int32_t)INT32_MIN));
                            for (; it != tab.end() && it->first == h; ++it)
                                if (it->second > E) cand.push_back(it->second);
                        }
            }
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            PairRec R;
            std::memset(&R, 0, sizeof R);
            if (with_identical) {
                classify_pair(s, E, E, R);
                part[w].push_back(R);
            }
            for (int32_t F : cand) {
                std::memset(&R, 0, sizeof R);
                classify_pair(s, E, F, R, true);
                if (R.cls != kRegular) part[w].push_back(R);
            }
        }
    });
    size_t tot = 0;
    for (auto &v : part) tot += v.size();
    out.reserve(tot);
    for (auto &v : part) out.insert(out.end(), v.begin(), v.end());
    return "";
}

// Near-field element pairs E <= F, in block order (target leaf, source leaf,
// then the elements of each leaf row by row).  A pair is generated from the
// block (leaf(E), leaf(F)) only; blk2 is the mirrored block (leaf(F), leaf(E)).
static std::string build_pairs(Setup &s)
{
    auto block_index = [&](int t, int src) -> int32_t {
        auto b = s.near_src.begin() + s.near_ptr[t], e = s.near_src.begin() + s.near_ptr[t + 1];
        auto it = std::lower_bound(b, e, src);
        if (it == e || *it != src) return -1;
        return (int32_t)(it - s.near_src.begin());
    };
    s.pairs.clear();
    for (int c = 0; c < 4; ++c) s.npairs_class[c] = 0;
    int nL = 1 << s.L;
    int64_t nnear = (int64_t)(s.near.size() / 2);
    int nw = num_workers(nnear / 16 + 1);
    // per worker, four groups: regular pairs by Gauss order (g0, g0 + 2, g0 + 4, capped at 40), touching
    const int o1 = std::min(40, s.g0 + 2);
    auto group = [&](const PairRec &R) { return R.cls != kRegular ? 3 : (R.order == s.g0 ? 0 : (R.order == o1 ? 1 : 2)); };
    std::vector<std::array<std::vector<PairRec>, 4>> part(nw);
    std::vector<int> bad(nw, 0);
    parallel_chunks(nnear, nw, [&](int64_t kb, int64_t ke, int w) {
        std::array<std::vector<PairRec>, 4> &out = part[w];
        for (int64_t k = kb; k < ke; ++k) {
            int t = s.near[2 * k], src = s.near[2 * k + 1];
            int32_t blk1 = (int32_t)k, blk2 = block_index(src, t);
            if (blk2 < 0) {
                bad[w] = 1;
                continue;
            }
            int pt = t / (nL * nL), rt = t % (nL * nL), t2 = rt / nL, t1 = rt % nL;
            int ps = src / (nL * nL), rs = src % (nL * nL), s2 = rs / nL, s1 = rs % nL;
            for (int a2 = 0; a2 < s.side; ++a2)
                for (int a1 = 0; a1 < s.side; ++a1) {
                    int E = pt * s.ne * s.ne + (t2 * s.side + a2) * s.ne + t1 * s.side + a1;
                    for (int b2 = 0; b2 < s.side; ++b2)
                        for (int b1 = 0; b1 < s.side; ++b1) {
                            int F = ps * s.ne * s.ne + (s2 * s.side + b2) * s.ne + s1 * s.side + b1;
                            if (F < E) continue;
                            PairRec R;
                            std::memset(&R, 0, sizeof R);
                            classify_pair(s, E, F, R);
                            R.elE = (int8_t)(a2 * s.side + a1);
                            R.elF = (int8_t)(b2 * s.side + b1);
                            R.blk1 = blk1;
                            R.blk2 = (E == F) ? -1 : blk2;
                            out[group(R)].push_back(R);
                        }
                }
        }
    });
    for (int w = 0; w < nw; ++w)
        if (bad[w]) return "near-field partition is not symmetric";
    // group k of worker w goes to pair_off[k] + (sizes of group k in workers before w): one parallel copy
    std::vector<std::array<int64_t, 4>> at(nw);
    int64_t pos = 0;
    for (int g = 0; g < 4; ++g) {
        s.pair_off[g] = pos;
        for (int w = 0; w < nw; ++w) {
            at[w][g] = pos;
            pos += (int64_t)part[w][g].size();
        }
    }
    s.pair_off[4] = pos;
    s.pairs.resize(pos);
    // the copy in pieces of at most 32768 pairs (1 MiB), spread over the pool
    struct Piece { int w, g; int64_t from, n; };
    std::vector<Piece> pieces;
    for (int w = 0; w < nw; ++w)
        for (int g = 0; g < 4; ++g)
            for (int64_t f = 0; f < (int64_t)part[w][g].size(); f += 32768)
                pieces.push_back({w, g, f, std::min<int64_t>(32768, (int64_t)part[w][g].size() - f)});
    parallel_chunks((int64_t)pieces.size(), 1 << 30, [&](int64_t pb, int64_t pe, int) {
        for (int64_t i = pb; i < pe; ++i) {
            const Piece &P = pieces[i];
            std::memcpy(&s.pairs[at[P.w][P.g] + P.from], part[P.w][P.g].data() + P.from, P.n * sizeof(PairRec));
        }
    });
    for (int g = 0; g < 3; ++g) s.npairs_class[kRegular] += s.pair_off[g + 1] - s.pair_off[g];
    for (int64_t k = s.pair_off[3]; k < s.pair_off[4]; ++k) s.npairs_class[s.pairs[k].cls]++;
    return "";
}

// ---------------------------------------------------------------------------
// Degree elevation of a rational Bezier tile in homogeneous form from (pu, pv)
// to (PG, PG): c'_i = i/(p+1) c_{i-1} + (1 - i/(p+1)) c_i, one degree at a time.
// ---------------------------------------------------------------------------
static void elevate_tile(const std::vector<double> &Hin, int pu, int pv, int PG, double *out)
{
    std::vector<double> H = Hin;
    int cu = pu, cv = pv;
    auto at = [&](std::vector<double> &A, int nu, int i, int j) { return &A[4 * ((size_t)j * (nu + 1) + i)]; };
    while (cu < PG) {
        std::vector<double> N((size_t)(cu + 2) * (cv + 1) * 4, 0.0);
        for (int j = 0; j <= cv; ++j)
            for (int i = 0; i <= cu + 1; ++i) {
                double a = (double)i / (cu + 1);
                for (int c = 0; c < 4; ++c) {
                    double v = 0.0;
                    if (i >= 1) v += a * at(H, cu, i - 1, j)[c];
                    if (i <= cu) v += (1.0 - a) * at(H, cu, i, j)[c];
                    at(N, cu + 1, i, j)[c] = v;
                }
            }
        H.swap(N);
        ++cu;
    }
    while (cv < PG) {
        std::vector<double> N((size_t)(cu + 1) * (cv + 2) * 4, 0.0);
        for (int j = 0; j <= cv + 1; ++j)
            for (int i = 0; i <= cu; ++i) {
                double a = (double)j / (cv + 1);
                for (int c = 0; c < 4; ++c) {
                    double v = 0.0;
                    if (j >= 1) v += a * at(H, cu, i, j - 1)[c];
                    if (j <= cv) v += (1.0 - a) * at(H, cu, i, j)[c];
                    at(N, cu, i, j)[c] = v;
                }
            }
        H.swap(N);
        ++cv;
    }
    std::memcpy(out, H.data(), sizeof(double) * 4 * (PG + 1) * (PG + 1));
}

// ---------------------------------------------------------------------------
std::string build_setup_tiles(const Geometry &geo, const igb_params &prm, Setup &s)
{
    auto t0 = std::chrono::steady_clock::now();
    if (prm.kernel != IGB_LAPLACE && prm.kernel != IGB_HELMHOLTZ) return "kernel must be IGB_LAPLACE or IGB_HELMHOLTZ";
    if (prm.p < 0 || prm.p > 6) return "p outside 0..6";
    if (prm.m < 0 || prm.m > 10) return "m outside 0..10";
    if (prm.q < 1 || prm.q > 16) return "q outside 1..16";
    if (!(prm.eta > 0.0) || !std::isfinite(prm.eta)) return "eta must be > 0";
    if (!(prm.kappa_diam >= 0.0) || !std::isfinite(prm.kappa_diam)) return "kappa_diam must be >= 0";
    if (prm.kernel == IGB_HELMHOLTZ && (!(prm.wavenumber >= 0.0) || !std::isfinite(prm.wavenumber)))
        return "wavenumber must be >= 0";
    if (prm.gauss_regular < 1 || prm.gauss_regular > 36) return "gauss_regular outside 1..36";
    if (prm.gauss_singular != -1 && (prm.gauss_singular < 1 || prm.gauss_singular > 40)) return "gauss_singular outside 1..40";
    if (prm.gauss_rhs != -1 && (prm.gauss_rhs < 1 || prm.gauss_rhs > 40)) return "gauss_rhs outside 1..40";
    if (prm.mode != IGB_DENSE && prm.mode != IGB_H2_STORED && prm.mode != IGB_H2_ONTHEFLY)
        return "mode must be IGB_DENSE, IGB_H2_STORED or IGB_H2_ONTHEFLY";
    if (prm.far_precision != IGB_FP64 && prm.far_precision != IGB_FP32)
        return "far_precision must be IGB_FP64 or IGB_FP32";
    if (prm.far_precision == IGB_FP32 &&
        (prm.mode != IGB_H2_ONTHEFLY || prm.q * prm.q > (prm.kernel == IGB_HELMHOLTZ ? 104 : 64)))
        return "far_precision IGB_FP32 needs on-the-fly coupling and q <= 8 (Laplace) or q <= 10 (Helmholtz)";
    if (prm.leaf_depth < -1 || prm.leaf_depth > 10) return "leaf_depth outside -1..10";
    // the surface lies in the hull of its control points, whose bounding box bounds |x - y| between
    // surface points (and places the surface in a ball for the potential's phase range)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (const auto &pt : geo.patches)
        for (size_t i = 0; i + 3 < pt.cpw.size(); i += 4)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], pt.cpw[i + c]);
                hi[c] = std::max(hi[c], pt.cpw[i + c]);
            }
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) d2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
    // the kernels reduce the phase kappa |x - y| between surface points for |kappa r| < 2^19
    if (prm.kernel == IGB_HELMHOLTZ && prm.wavenumber * std::sqrt(d2) >= 262144.0)
        return "wavenumber times the size of the geometry must stay below 2^18";
    for (int c = 0; c < 3; ++c) s.hull_c[c] = 0.5 * (lo[c] + hi[c]);
    s.hull_r = 0.5 * std::sqrt(d2);

    s.kernel = prm.kernel;
    s.kappa = prm.kernel == IGB_HELMHOLTZ ? prm.wavenumber : 0.0;
    s.p = prm.p;
    s.m = prm.m;
    s.q = prm.q;
    s.eta = prm.eta;
    s.kappa_diam = prm.kappa_diam;
    s.g0 = prm.gauss_regular;
    s.gs = prm.gauss_singular > 0 ? prm.gauss_singular : std::min(40, s.g0 + 2);
    s.grhs = prm.gauss_rhs > 0 ? prm.gauss_rhs : std::max(s.g0, s.p + 4);
    s.mode = prm.mode;
    int d = prm.leaf_depth;
    if (d < 0) {
        d = 0;
        while ((s.p + 1) * (s.p + 1) * (1 << (2 * d)) < s.q * s.q && d < s.m) ++d;
    }
    d = std::min(d, s.m);
    if (d > 3) return "leaf_depth > 3 (more than 64 elements per leaf) is not supported";
    s.d = d;
    s.L = s.m - d;
    s.npatch = (int)geo.patches.size();
    if (((int64_t)s.npatch << (2 * s.m)) >= ((int64_t)1 << 29)) return "too many elements (n_patches * 4^m >= 2^29)";
    s.ne = 1 << s.m;
    s.nelem = s.npatch * s.ne * s.ne;
    s.nloc = (s.p + 1) * (s.p + 1);
    s.ns1 = s.ne + s.p;
    s.nsup = (int64_t)s.nelem * s.nloc;
    s.ndof = (int64_t)s.npatch * s.ns1 * s.ns1;
    s.side = 1 << d;
    s.nl = s.side * s.side * s.nloc;
    s.n1 = s.side * (s.p + 1);
    s.nleaf = s.npatch << (2 * s.L);
    s.cl_off.assign(s.L + 2, 0);
    for (int l = 0; l <= s.L; ++l) s.cl_off[l + 1] = s.cl_off[l] + ((int64_t)s.npatch << (2 * l));

    // Gauss rules 1..40 (the same table for every operator: built once)
    {
        struct Table {
            std::vector<int32_t> off;
            std::vector<double> x, w;
            Table() : off(42, 0)
            {
                for (int n = 1; n <= 40; ++n) off[n + 1] = off[n] + n;
                x.assign(off[41], 0.0);
                w.assign(off[41], 0.0);
                for (int n = 1; n <= 40; ++n) gauss_rule(n, &x[off[n]], &w[off[n]]);
            }
        };
        static const Table table;
        s.goff = table.off;
        s.gx = table.x;
        s.gw = table.w;
    }

    // element tiles by Bezier extraction, degree-elevated to one common bidegree
    // (exact) so that every tile has the same compile-time shape on the device.
    // Separable: the u-extraction rows are applied once per element column e1,
    // then each element contracts the v-extraction rows over that result.
    int pmax = 0;
    for (const Patch &P : geo.patches) pmax = std::max(pmax, std::max(P.pu, P.pv));
    int PG = pmax <= 1 ? 1 : (pmax <= 2 ? 2 : (pmax <= 4 ? 4 : 8));
    s.tile_degree = PG;
    s.tile_stride = (PG + 1) * (PG + 1) * 4;
    s.tiles.assign((size_t)s.nelem * s.tile_stride, 0.0);
    s.tile_deg.assign((size_t)s.nelem * 2, PG);
    struct PatchExtraction {
        std::vector<double> Mv, A;
        std::vector<int> vlo, vhi;
    };
    std::vector<PatchExtraction> px(s.npatch);
    // nonzero column range of every extraction row
    auto support = [](const std::vector<double> &M, int rows, int cols, std::vector<int> &lo, std::vector<int> &hi) {
        lo.assign(rows, 0);
        hi.assign(rows, -1);
        for (int k = 0; k < rows; ++k) {
            int a = cols, b = -1;
            for (int j = 0; j < cols; ++j)
                if (M[(size_t)k * cols + j] != 0.0) { a = std::min(a, j); b = j; }
            lo[k] = a;
            hi[k] = b;
        }
    };
    for (int pt = 0; pt < s.npatch; ++pt) {
        const Patch &P = geo.patches[pt];
        PatchExtraction &X = px[pt];
        std::vector<double> Mu;
        int nru, nrv;
        std::string err = extraction(P.pu, P.U, P.nu, s.ne, Mu, nru);
        if (!err.empty()) return "patch " + std::to_string(pt) + " u: " + err;
        err = extraction(P.pv, P.V, P.nv, s.ne, X.Mv, nrv);
        if (!err.empty()) return "patch " + std::to_string(pt) + " v: " + err;
        std::vector<int> ulo, uhi;
        support(Mu, nru, P.nu, ulo, uhi);
        support(X.Mv, nrv, P.nv, X.vlo, X.vhi);
        // A[((e1 * nv + j) * (pu+1) + ru) * 4 + c] = sum_i Mu[ku][i] * w_ji * (x, y, z, 1)_ji
        const int pu1 = P.pu + 1;
        X.A.assign((size_t)s.ne * P.nv * pu1 * 4, 0.0);
        for (int e1 = 0; e1 < s.ne; ++e1)
            for (int ru = 0; ru < pu1; ++ru) {
                int ku = P.pu == 0 ? e1 : e1 * P.pu + ru;
                for (int j = 0; j < P.nv; ++j) {
                    double acc[4] = {0, 0, 0, 0};
                    for (int i = ulo[ku]; i <= uhi[ku]; ++i) {
                        const double *c = &P.cpw[4 * ((size_t)j * P.nu + i)];
                        double f = Mu[(size_t)ku * P.nu + i] * c[3];
                        acc[0] += f * c[0];
                        acc[1] += f * c[1];
                        acc[2] += f * c[2];
                        acc[3] += f;
                    }
                    for (int c = 0; c < 4; ++c) X.A[(((size_t)e1 * P.nv + j) * pu1 + ru) * 4 + c] = acc[c];
                }
            }
    }
    // per element: v-contraction, degree elevation
    parallel_chunks(s.nelem, 1 << 30, [&](int64_t b, int64_t e, int) {
        std::vector<double> H;
        for (int64_t k = b; k < e; ++k) {
            int E = (int)k;
            int pt = E / (s.ne * s.ne), r = E % (s.ne * s.ne), e2 = r / s.ne, e1 = r % s.ne;
            const Patch &P = geo.patches[pt];
            const PatchExtraction &X = px[pt];
            const int pu1 = P.pu + 1, pv1 = P.pv + 1;
            H.assign((size_t)pu1 * pv1 * 4, 0.0);
            for (int rv = 0; rv < pv1; ++rv) {
                int kv = P.pv == 0 ? e2 : e2 * P.pv + rv;
                for (int ru = 0; ru < pu1; ++ru) {
                    double acc[4] = {0, 0, 0, 0};
                    for (int j = X.vlo[kv]; j <= X.vhi[kv]; ++j) {
                        double cv = X.Mv[(size_t)kv * P.nv + j];
                        const double *a = &X.A[(((size_t)e1 * P.nv + j) * pu1 + ru) * 4];
                        for (int c = 0; c < 4; ++c) acc[c] += cv * a[c];
                    }
                    for (int c = 0; c < 4; ++c) H[4 * (rv * pu1 + ru) + c] = acc[c];
                }
            }
            elevate_tile(H, P.pu, P.pv, PG, &s.tiles[(size_t)E * s.tile_stride]);
        }
    });
    // T band on Xi_{p,m}
    {
        int p = s.p;
        std::vector<double> U(s.ns1 + p + 1);
        for (int i = 0; i <= p; ++i) { U[i] = 0.0; U[s.ns1 + i] = 1.0; }
        for (int i = 1; i < s.ne; ++i) U[p + i] = (double)i / s.ne;
        std::vector<double> M;
        int nr;
        std::string err = extraction(p, U, s.ns1, s.ne, M, nr);
        if (!err.empty()) return "spline space: " + err;
        s.Tb.assign((size_t)s.ne * (p + 1) * (p + 1), 0.0);
        for (int e = 0; e < s.ne; ++e)
            for (int r = 0; r <= p; ++r)
                for (int jj = 0; jj <= p; ++jj) {
                    int j = e + jj;
                    int k = (p == 0) ? e : e * p + r;
                    s.Tb[((size_t)e * (p + 1) + r) * (p + 1) + jj] = (j < s.ns1) ? M[(size_t)k * s.ns1 + j] : 0.0;
                }
    }
    // Chebyshev nodes, moments, transfers
    s.z.resize(s.q);
    for (int k = 0; k < s.q; ++k) s.z[k] = 0.5 * (1.0 + std::cos((2.0 * k + 1.0) * M_PI / (2.0 * s.q)));
    {
        int ng = (s.q + s.p) / 2 + 2;
        const double *x = &s.gx[s.goff[ng]], *w = &s.gw[s.goff[ng]];
        auto mom = [&](int nsub, int el, int r, int mu) {
            double acc = 0.0;
            double B[16];
            for (int i = 0; i < ng; ++i) {
                bern(s.p, x[i], B, nullptr);
                acc += w[i] * lagr(s.z, mu, (el + x[i]) / nsub) * B[r];
            }
            return acc / nsub;
        };
        s.M1.assign((size_t)s.n1 * s.q, 0.0);
        for (int el = 0; el < s.side; ++el)
            for (int r = 0; r <= s.p; ++r)
                for (int mu = 0; mu < s.q; ++mu) s.M1[(size_t)(el * (s.p + 1) + r) * s.q + mu] = mom(s.side, el, r, mu);
        s.E2.assign((size_t)2 * s.q * s.q, 0.0);
        for (int c = 0; c < 2; ++c)
            for (int nu = 0; nu < s.q; ++nu)
                for (int mu = 0; mu < s.q; ++mu) s.E2[((size_t)c * s.q + nu) * s.q + mu] = lagr(s.z, mu, 0.5 * (c + s.z[nu]));
        s.Mlev_off.assign(s.L + 2, 0);
        for (int l = 0; l <= s.L; ++l) s.Mlev_off[l + 1] = s.Mlev_off[l] + (int64_t)(s.ne >> l) * (s.p + 1) * s.q;
        s.Mlev.assign(s.Mlev_off[s.L + 1], 0.0);
        for (int l = 0; l <= s.L; ++l) {
            int nsub = s.ne >> l;
            for (int el = 0; el < nsub; ++el)
                for (int r = 0; r <= s.p; ++r)
                    for (int mu = 0; mu < s.q; ++mu)
                        s.Mlev[s.Mlev_off[l] + (size_t)(el * (s.p + 1) + r) * s.q + mu] = mom(nsub, el, r, mu);
        }
    }
    s.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return "";
}

void build_setup_elements(Setup &s)
{
    auto t0 = std::chrono::steady_clock::now();
    s.ecorner.assign((size_t)s.nelem * 12, 0.0);
    s.egrid.assign((size_t)s.nelem * 27, 0.0);
    s.ediam.assign(s.nelem, 0.0);
    s.erad.assign(s.nelem, 0.0);
    // corners / 3x3 grid / diameter / grid radius per element
    parallel_chunks(s.nelem, 1 << 30, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k) element_geometry_one(s, (int)k);
    });
    s.setup_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

std::string build_setup_geometry(const Geometry &geo, const igb_params &prm, Setup &s)
{
    std::string err = build_setup_tiles(geo, prm, s);
    if (err.empty()) build_setup_elements(s);
    return err;
}

std::string build_setup_plan(Setup &s)
{
    auto t0 = std::chrono::steady_clock::now();
    build_partition(s);
    std::string perr = build_pairs(s);
    s.setup_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return perr;
}

std::string check_touching(const Setup &s, const std::vector<PairRec> &touch, std::vector<PairRec> *plan_touch)
{
    std::vector<PairRec> mine;
    std::vector<PairRec> &pt = plan_touch ? *plan_touch : mine;
    pt.clear();
    for (int64_t k = s.pair_off[3]; k < s.pair_off[4]; ++k) pt.push_back(s.pairs[k]);
    std::sort(pt.begin(), pt.end(), [](const PairRec &a, const PairRec &b) {
        return ((uint64_t)(uint32_t)a.E << 32 | (uint32_t)a.F) < ((uint64_t)(uint32_t)b.E << 32 | (uint32_t)b.F);
    });
    if (pt.size() != touch.size()) return "touching pair enumeration differs from the near-field pairs (count)";
    for (size_t k = 0; k < pt.size(); ++k) {
        const PairRec &R = pt[k], &T = touch[k];
        if (T.E != R.E || T.F != R.F || T.cls != R.cls || T.order != R.order || T.oE != R.oE || T.aE != R.aE ||
            T.bE != R.bE || T.oF != R.oF || T.aF != R.aF || T.bF != R.bF)
            return "touching pair enumeration differs from the near-field pairs";
    }
    return "";
}

void sorted_pair_classes(const Setup &s, int32_t *out)
{
    std::vector<uint64_t> idx(s.pairs.size());
    for (size_t k = 0; k < s.pairs.size(); ++k) idx[k] = k;
    std::sort(idx.begin(), idx.end(), [&](uint64_t x, uint64_t y) {
        const PairRec &a = s.pairs[x], &b = s.pairs[y];
        return a.E < b.E || (a.E == b.E && a.F < b.F);
    });
    for (size_t k = 0; k < idx.size(); ++k) {
        const PairRec &R = s.pairs[idx[k]];
        out[4 * k] = R.E;
        out[4 * k + 1] = R.F;
        out[4 * k + 2] = R.cls;
        out[4 * k + 3] = R.order;
    }
}

std::string build_setup(const Geometry &geo, const igb_params &prm, Setup &s)
{
    std::string err = build_setup_geometry(geo, prm, s);
    if (!err.empty()) return err;
    std::vector<PairRec> touch;
    err = enumerate_touching(s, touch, true);
    if (!err.empty()) return err;
    err = build_setup_plan(s);
    if (!err.empty()) return err;
    return check_touching(s, touch);
}

}  // namespace igb
