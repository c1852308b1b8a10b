/*
 * Plain FP64 CPU oracle for the isogeometric single-layer BEM with
 * interpolation-based (H2) compression, after Doelz, Harbrecht, Kurz, Schoeps,
 * Wolf, "A Fast Isogeometric BEM for the Three Dimensional Laplace- and
 * Helmholtz Problems" (arXiv 1708.09162).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP path against a slow,
 * obviously correct reference.  It shares no code with the HIP library.
 *
 * Every arithmetic step is done in double precision (complex<double> for
 * Helmholtz), written the direct way:
 *   - B-splines by the Cox-de Boor recursion (Sec. 2.1, Def. of b_j^p),
 *   - NURBS by the rational tensor formula (Sec. 2.2, eq. def::geom),
 *     derivatives by the quotient rule, surface measure (Sec. 3.2),
 *   - the superspace of element-wise Bernstein polynomials and the
 *     B-spline -> Bernstein matrix T by collocation (Sec. 4.3),
 *   - Galerkin element-pair integrals (Sec. 3.2) by tensor Gauss rules and
 *     Duffy-type regularising transformations for touching pairs (Sec. 4,
 *     item 4),
 *   - the per-patch quadtree, admissibility and block partition (Sec. 4.1,
 *     Sec. 4.2 Def.),
 *   - the degenerate-kernel far field with tensor Chebyshev interpolation and
 *     moments computed *directly* for every cluster (no nested transfers)
 *     (Sec. 4.2),
 *   - Jacobi-preconditioned CG / GMRES (Sec. 4, item 3; Sec. 5.3),
 *   - the representation formula for the potential (Sec. 3.1, eq. eq::repform).
 * Readings of points where the paper is silent are stated at the code that
 * implements them.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_LAPLACE 0
#define OR_HELMHOLTZ 1

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [0,1] (Sec. 4, item 4: orders up to 40).           */
/* Newton iteration on the three-term Legendre recurrence; weights from P_n'. */
/* ------------------------------------------------------------------------ */
int or_gauss(int n, double *x, double *w)
{
    if (n < 1 || n > 64) return -1;
    for (int i = 0; i < n; ++i) {
        double t = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) {
                /* one more step with the final derivative */
                break;
            }
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = t; p0 = 1.0; }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        /* map [-1,1] -> [0,1]; node i is the i-th largest on [-1,1] */
        x[n - 1 - i] = 0.5 * (t + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp); /* = (2/((1-t^2)P'^2)) / 2 */
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* B-splines by Cox-de Boor (Sec. 2.1).  All k = nknots-p-1 functions at x,   */
/* with derivatives.  Reading of the half-open interval: at x = 1 the last    */
/* non-empty knot interval is taken as closed on the right.  0/0 := 0.        */
/* ------------------------------------------------------------------------ */
static void bspline_all(int p, const double *U, int nk, double x, double *N, double *dN)
{
    int k = nk - p - 1;
    int nint = nk - 1;
    double *b = (double *)calloc((size_t)nint + 1, sizeof(double));
    /* degree 0 */
    int last = -1;
    for (int j = 0; j < nint; ++j)
        if (U[j + 1] > U[j]) last = j;
    for (int j = 0; j < nint; ++j) {
        int in = (U[j] <= x && x < U[j + 1]);
        if (j == last && x == U[j + 1]) in = 1;
        b[j] = in ? 1.0 : 0.0;
    }
    double *bm1 = (double *)calloc((size_t)nint + 1, sizeof(double));
    for (int d = 1; d <= p; ++d) {
        memcpy(bm1, b, sizeof(double) * (size_t)nint);
        for (int j = 0; j + d < nint; ++j) {
            double a = 0.0, c = 0.0;
            double den1 = U[j + d] - U[j];
            double den2 = U[j + d + 1] - U[j + 1];
            if (den1 > 0.0) a = (x - U[j]) / den1 * bm1[j];
            if (den2 > 0.0) c = (U[j + d + 1] - x) / den2 * bm1[j + 1];
            b[j] = a + c;
        }
        if (d == p && dN) {
            /* derivative of degree-p functions from degree p-1 ones */
            for (int j = 0; j < k; ++j) {
                double t1 = 0.0, t2 = 0.0;
                double den1 = U[j + p] - U[j];
                double den2 = U[j + p + 1] - U[j + 1];
                if (den1 > 0.0) t1 = p / den1 * bm1[j];
                if (den2 > 0.0) t2 = p / den2 * bm1[j + 1];
                dN[j] = t1 - t2;
            }
        }
    }
    if (p == 0 && dN)
        for (int j = 0; j < k; ++j) dN[j] = 0.0;
    for (int j = 0; j < k; ++j) N[j] = b[j];
    free(b);
    free(bm1);
}

/* Bernstein polynomial B_{i,p}(x) = C(p,i) x^i (1-x)^(p-i) (Sec. 4.3). */
static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
static double bernstein(int p, int i, double x)
{
    return binom(p, i) * pow(x, i) * pow(1.0 - x, p - i);
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int pu, pv, nu, nv;
    double *U, *V;
    double *cpw; /* nv*nu*4: x,y,z,w */
} or_patch;

typedef struct {
    int level, tgt, src; /* cluster ids within their level: patch*4^l + k2*2^l + k1 */
} or_block;

typedef struct or_problem {
    int npatch;
    or_patch *patches;
    int kernel;
    double kappa;
    int p, m, q, L, g0, gs, grhs;
    double eta;
    double kdmax; /* > 0: also kappa * max(diam) <= kdmax for admissibility (an option, not the paper's) */
    int nel1, nelem, nloc, nsup, ns1, ndof;
    double h;
    double *T1;     /* ns1 x (nel1*(p+1)) */
    double *corner; /* nelem x 4 x 3 */
    double *grid9;  /* nelem x 9 x 3 */
    double *ediam;  /* nelem */
    /* Chebyshev nodes */
    double *z;
    /* partition */
    int64_t nnear, nfar;
    or_block *near; /* level = L */
    or_block *far;
    /* near-field element CSR (built on demand) */
    int64_t *nb_ptr; /* nelem+1 */
    int *nb_idx;
    cplx *nb_blk;   /* nloc*nloc per entry, or NULL if not assembled */
    /* far-field blocks per level: CSR by target, sorted sources (for lookups) */
    int64_t **far_ptr; /* [level][ncl(level)+1] */
    int **far_src;
    int64_t **far_id;  /* index into far[] */
    cplx *far_K;       /* stored coupling (nfar * q^4) or NULL */
    int nthreads;
} or_problem;

static int ipow2(int l) { return 1 << l; }
static int ncl_level(const or_problem *P, int l) { return P->npatch * ipow2(l) * ipow2(l); }

/* NURBS map, first derivatives and surface measure (Sec. 2.2, Sec. 3.2). */
static void nurbs_eval(const or_patch *pt, double u, double v, double X[3], double Xu[3], double Xv[3])
{
    double Nu[64], dNu[64], Nv[64], dNv[64];
    bspline_all(pt->pu, pt->U, pt->nu + pt->pu + 1, u, Nu, dNu);
    bspline_all(pt->pv, pt->V, pt->nv + pt->pv + 1, v, Nv, dNv);
    double S[4] = {0, 0, 0, 0}, Su[4] = {0, 0, 0, 0}, Sv[4] = {0, 0, 0, 0};
    for (int j = 0; j < pt->nv; ++j)
        for (int i = 0; i < pt->nu; ++i) {
            const double *c = pt->cpw + 4 * ((size_t)j * pt->nu + i);
            double w = c[3];
            double bb = Nu[i] * Nv[j], bu = dNu[i] * Nv[j], bv = Nu[i] * dNv[j];
            for (int d = 0; d < 3; ++d) {
                S[d] += c[d] * w * bb;
                Su[d] += c[d] * w * bu;
                Sv[d] += c[d] * w * bv;
            }
            S[3] += w * bb;
            Su[3] += w * bu;
            Sv[3] += w * bv;
        }
    for (int d = 0; d < 3; ++d) {
        X[d] = S[d] / S[3];
        if (Xu) Xu[d] = (Su[d] - X[d] * Su[3]) / S[3];
        if (Xv) Xv[d] = (Sv[d] - X[d] * Sv[3]) / S[3];
    }
}

static double surface_measure(const double Xu[3], const double Xv[3])
{
    double n0 = Xu[1] * Xv[2] - Xu[2] * Xv[1];
    double n1 = Xu[2] * Xv[0] - Xu[0] * Xv[2];
    double n2 = Xu[0] * Xv[1] - Xu[1] * Xv[0];
    return sqrt(n0 * n0 + n1 * n1 + n2 * n2);
}

/* Point and surface measure at patch parameter (u,v). */
static void geom(const or_problem *P, int patch, double u, double v, double X[3], double *kap)
{
    double Xu[3], Xv[3];
    nurbs_eval(&P->patches[patch], u, v, X, Xu, Xv);
    *kap = surface_measure(Xu, Xv);
}

static double dist3(const double *a, const double *b)
{
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

/* Fundamental solutions (Sec. 3.1, eq. eq::fundament1 and eq::fundament2). */
static cplx fundamental(const or_problem *P, const double *x, const double *y)
{
    double r = dist3(x, y);
    if (P->kernel == OR_LAPLACE) return 1.0 / (4.0 * M_PI * r);
    return cexp(I * P->kappa * r) / (4.0 * M_PI * r);
}

/* ------------------------------------------------------------------------ */
/* Superspace and the matrix T (Sec. 4.3).                                   */
/* T1[j, (e,r)]: coefficients with b_j restricted to element e equal to       */
/* sum_r T1[j,(e,r)] B_{r,p}((x - e h)/h).  Obtained by collocation: on each  */
/* element, solve the (p+1)x(p+1) Bernstein-Vandermonde system at p+1 points. */
/* ------------------------------------------------------------------------ */
static int solve_dense(int n, double *A, double *b)
{
    /* Gaussian elimination with partial pivoting, in place; b overwritten */
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
        b[c] = s / A[c * n + c];
    }
    return 0;
}

static void build_T1(or_problem *P)
{
    int p = P->p, ne = P->nel1, ns1 = P->ns1, nk = ns1 + p + 1;
    double *U = (double *)malloc(sizeof(double) * nk);
    /* uniform p-open knot vector Xi_{p,m} (Sec. 2.2) */
    for (int i = 0; i <= p; ++i) U[i] = 0.0;
    for (int i = 1; i < ne; ++i) U[p + i] = (double)i / ne;
    for (int i = 0; i <= p; ++i) U[p + ne + i] = 1.0;
    P->T1 = (double *)calloc((size_t)ns1 * ne * (p + 1), sizeof(double));
    double *N = (double *)malloc(sizeof(double) * ns1);
    double *A = (double *)malloc(sizeof(double) * (p + 1) * (p + 1));
    double *rhs = (double *)malloc(sizeof(double) * (p + 1));
    for (int e = 0; e < ne; ++e) {
        for (int j = 0; j < ns1; ++j) {
            for (int c = 0; c <= p; ++c) {
                double t = (p == 0) ? 0.5 : (0.1 + 0.8 * c / p); /* interior collocation points */
                double x = (e + t) / ne;
                bspline_all(p, U, nk, x, N, NULL);
                rhs[c] = N[j];
                for (int r = 0; r <= p; ++r) A[c * (p + 1) + r] = bernstein(p, r, t);
            }
            solve_dense(p + 1, A, rhs);
            for (int r = 0; r <= p; ++r) {
                double v = rhs[r];
                if (fabs(v) < 1e-15) v = 0.0;
                P->T1[(size_t)j * ne * (p + 1) + e * (p + 1) + r] = v;
            }
        }
    }
    free(U);
    free(N);
    free(A);
    free(rhs);
}

/* ------------------------------------------------------------------------ */
/* Elements: E = patch*4^m + e2*2^m + e1; corners c0=(0,0), c1=(1,0),         */
/* c2=(1,1), c3=(0,1) in element-local coordinates (counter-clockwise).       */
/* ------------------------------------------------------------------------ */
static void elem_decode(const or_problem *P, int E, int *patch, int *e1, int *e2)
{
    int per = P->nel1 * P->nel1;
    *patch = E / per;
    int r = E % per;
    *e2 = r / P->nel1;
    *e1 = r % P->nel1;
}

static void elem_param(const or_problem *P, int E, double s, double t, int *patch, double *u, double *v)
{
    int e1, e2;
    elem_decode(P, E, patch, &e1, &e2);
    *u = (e1 + s) * P->h;
    *v = (e2 + t) * P->h;
}

static const double corner_loc[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};

static void build_elements(or_problem *P)
{
    P->corner = (double *)malloc(sizeof(double) * P->nelem * 12);
    P->grid9 = (double *)malloc(sizeof(double) * P->nelem * 27);
    P->ediam = (double *)malloc(sizeof(double) * P->nelem);
    for (int E = 0; E < P->nelem; ++E) {
        int patch;
        double u, v, k;
        for (int c = 0; c < 4; ++c) {
            elem_param(P, E, corner_loc[c][0], corner_loc[c][1], &patch, &u, &v);
            geom(P, patch, u, v, P->corner + E * 12 + 3 * c, &k);
        }
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                elem_param(P, E, 0.5 * a, 0.5 * b, &patch, &u, &v);
                geom(P, patch, u, v, P->grid9 + E * 27 + 3 * (b * 3 + a), &k);
            }
        double d = 0.0;
        for (int i = 0; i < 9; ++i)
            for (int j = i + 1; j < 9; ++j) {
                double t = dist3(P->grid9 + E * 27 + 3 * i, P->grid9 + E * 27 + 3 * j);
                if (t > d) d = t;
            }
        P->ediam[E] = d;
    }
}

/* ------------------------------------------------------------------------ */
/* Classification of an element pair.                                         */
/* Touching is decided physically: corners coincide within 1e-10 * max diam.  */
/* class: 0 regular, 1 identical, 2 common edge, 3 common vertex.             */
/* Regular order (reading of "order increased logarithmically towards the     */
/* singularity"): r = dist/max(diam), both from the 3x3 element grids         */
/* (corners, edge midpoints, centre); g = g0 if r >= 1.2, g0+2 if             */
/* 0.6 <= r < 1.2, g0+4 if r < 0.6, capped at 40.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int cls, order;
    int oE, aE, bE;  /* canonical frame of E: origin corner, corner at (1,0), at (0,1) */
    int oF, aF, bF;  /* same for E' */
} pair_info;

static int adj_other(int o, int a) { /* the adjacent corner of o that is not a */
    int n1 = (o + 1) & 3, n2 = (o + 3) & 3;
    return (a == n1) ? n2 : n1;
}

static pair_info classify(const or_problem *P, int E, int F)
{
    pair_info pi;
    memset(&pi, 0, sizeof pi);
    pi.oE = 0; pi.aE = 1; pi.bE = 3;
    pi.oF = 0; pi.aF = 1; pi.bF = 3;
    double md = fmax(P->ediam[E], P->ediam[F]);
    if (E == F) {
        pi.cls = 1;
        pi.order = P->gs;
        return pi;
    }
    double tol = 1e-10 * md;
    int match[4]; /* match[c] = corner of F equal to corner c of E, or -1 */
    int nshared = 0;
    for (int c = 0; c < 4; ++c) {
        match[c] = -1;
        for (int d = 0; d < 4; ++d)
            if (dist3(P->corner + E * 12 + 3 * c, P->corner + F * 12 + 3 * d) <= tol) match[c] = d;
        if (match[c] >= 0) ++nshared;
    }
    if (nshared == 2) {
        int i = -1, j = -1;
        for (int c = 0; c < 4; ++c)
            if (match[c] >= 0) { if (i < 0) i = c; else j = c; }
        /* i < j: the shared edge runs from E's corner i to corner j */
        pi.cls = 2;
        pi.order = P->gs;
        pi.oE = i; pi.aE = j; pi.bE = adj_other(i, j);
        pi.oF = match[i]; pi.aF = match[j]; pi.bF = adj_other(pi.oF, pi.aF);
        return pi;
    }
    if (nshared == 1) {
        int i = -1;
        for (int c = 0; c < 4; ++c)
            if (match[c] >= 0) i = c;
        pi.cls = 3;
        pi.order = P->gs;
        pi.oE = i; pi.aE = (i + 1) & 3; pi.bE = (i + 3) & 3;
        int k = match[i];
        pi.oF = k; pi.aF = (k + 1) & 3; pi.bF = (k + 3) & 3;
        return pi;
    }
    double dmin = 1e300;
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b) {
            double t = dist3(P->grid9 + E * 27 + 3 * a, P->grid9 + F * 27 + 3 * b);
            if (t < dmin) dmin = t;
        }
    double r = dmin / md;
    int g = P->g0;
    if (r < 0.6) g = P->g0 + 4;
    else if (r < 1.2) g = P->g0 + 2;
    if (g > 40) g = 40;
    pi.cls = 0;
    pi.order = g;
    return pi;
}

/* canonical coordinates -> element-local coordinates for a frame (o, a, b) */
static void frame_map(int o, int a, int b, double s, double t, double *x, double *y)
{
    *x = corner_loc[o][0] + s * (corner_loc[a][0] - corner_loc[o][0]) + t * (corner_loc[b][0] - corner_loc[o][0]);
    *y = corner_loc[o][1] + s * (corner_loc[a][1] - corner_loc[o][1]) + t * (corner_loc[b][1] - corner_loc[o][1]);
}

/* Accumulate one quadrature point: blk[a][b] += W * K * phi_a(xl) * phi_b(yl). */
static void accumulate(const or_problem *P, int E, int F, double xs, double xt, double ys, double yt, double W,
                       cplx *blk)
{
    int pE, pF;
    double u, v, X[3], Y[3], kx, ky;
    elem_param(P, E, xs, xt, &pE, &u, &v);
    geom(P, pE, u, v, X, &kx);
    elem_param(P, F, ys, yt, &pF, &u, &v);
    geom(P, pF, u, v, Y, &ky);
    double h2 = P->h * P->h;
    cplx K = fundamental(P, X, Y) * (kx * h2) * (ky * h2) * W;
    int p = P->p, nl = P->nloc;
    double bx1[16], bx2[16], by1[16], by2[16];
    for (int r = 0; r <= p; ++r) {
        bx1[r] = bernstein(p, r, xs);
        bx2[r] = bernstein(p, r, xt);
        by1[r] = bernstein(p, r, ys);
        by2[r] = bernstein(p, r, yt);
    }
    for (int a2 = 0; a2 <= p; ++a2)
        for (int a1 = 0; a1 <= p; ++a1) {
            double fa = bx1[a1] * bx2[a2];
            for (int b2 = 0; b2 <= p; ++b2)
                for (int b1 = 0; b1 <= p; ++b1)
                    blk[(a2 * (p + 1) + a1) * nl + b2 * (p + 1) + b1] += K * fa * by1[b1] * by2[b2];
        }
}

/* Galerkin integral of one element pair (Sec. 3.2):                          */
/*   I[a][b] = int_E int_F u*(F x, F y) k(x) k(y) phi_a(x) phi_b(y) dy dx      */
/* with E the x-element.  Written for the given order (E, F).                 */
void or_pair_block(const or_problem *P, int E, int F, cplx *blk)
{
    int nl = P->nloc;
    for (int i = 0; i < nl * nl; ++i) blk[i] = 0.0;
    pair_info pi = classify(P, E, F);
    double gx[64], gw[64];
    int g = pi.order;
    or_gauss(g, gx, gw);
    if (pi.cls == 0) {
        /* regular: tensor Gauss in all four variables */
        for (int i2 = 0; i2 < g; ++i2)
            for (int i1 = 0; i1 < g; ++i1)
                for (int j2 = 0; j2 < g; ++j2)
                    for (int j1 = 0; j1 < g; ++j1)
                        accumulate(P, E, F, gx[i1], gx[i2], gx[j1], gx[j2], gw[i1] * gw[i2] * gw[j1] * gw[j2], blk);
        return;
    }
    if (pi.cls == 1) {
        /* identical: difference variables z = y - x per direction (both signs),  */
        /* x = (1-z)s (+z), then the z-square split into two triangles with the   */
        /* Duffy map z_big = xi, z_small = xi*eta.  8 regions.                    */
        for (int sg1 = 0; sg1 < 2; ++sg1)
            for (int sg2 = 0; sg2 < 2; ++sg2)
                for (int tri = 0; tri < 2; ++tri)
                    for (int a = 0; a < g; ++a)
                        for (int b = 0; b < g; ++b)
                            for (int c = 0; c < g; ++c)
                                for (int d = 0; d < g; ++d) {
                                    double xi = gx[a], eta = gx[b], s1 = gx[c], s2 = gx[d];
                                    double z1 = tri == 0 ? xi : xi * eta;
                                    double z2 = tri == 0 ? xi * eta : xi;
                                    double x1, y1, x2, y2;
                                    if (sg1 == 0) { x1 = (1 - z1) * s1; y1 = x1 + z1; }
                                    else { y1 = (1 - z1) * s1; x1 = y1 + z1; }
                                    if (sg2 == 0) { x2 = (1 - z2) * s2; y2 = x2 + z2; }
                                    else { y2 = (1 - z2) * s2; x2 = y2 + z2; }
                                    double W = gw[a] * gw[b] * gw[c] * gw[d] * xi * (1 - z1) * (1 - z2);
                                    accumulate(P, E, F, x1, x2, y1, y2, W, blk);
                                }
        return;
    }
    if (pi.cls == 2) {
        /* common edge: canonical frames put the shared edge at {t = 0} of both   */
        /* elements, same direction.  Along the edge: difference variable z with  */
        /* both signs, (1-z)s; the cube (z, x_t, y_t) is split into 3 pyramids by  */
        /* its largest coordinate (Duffy, Jacobian xi^2).  6 regions.              */
        for (int sg = 0; sg < 2; ++sg)
            for (int pyr = 0; pyr < 3; ++pyr)
                for (int a = 0; a < g; ++a)
                    for (int b = 0; b < g; ++b)
                        for (int c = 0; c < g; ++c)
                            for (int d = 0; d < g; ++d) {
                                double xi = gx[a], e1 = gx[b], e2 = gx[c], s = gx[d];
                                double z, xt, yt;
                                if (pyr == 0) { z = xi; xt = xi * e1; yt = xi * e2; }
                                else if (pyr == 1) { xt = xi; z = xi * e1; yt = xi * e2; }
                                else { yt = xi; z = xi * e1; xt = xi * e2; }
                                double xs, ys;
                                if (sg == 0) { xs = (1 - z) * s; ys = xs + z; }
                                else { ys = (1 - z) * s; xs = ys + z; }
                                double W = gw[a] * gw[b] * gw[c] * gw[d] * xi * xi * (1 - z);
                                double lx1, lx2, ly1, ly2;
                                frame_map(pi.oE, pi.aE, pi.bE, xs, xt, &lx1, &lx2);
                                frame_map(pi.oF, pi.aF, pi.bF, ys, yt, &ly1, &ly2);
                                accumulate(P, E, F, lx1, lx2, ly1, ly2, W, blk);
                            }
        return;
    }
    /* common vertex: shared corner at canonical (0,0) of both (rotation only); */
    /* the 4-cube split into 4 pyramids by its largest coordinate (Jacobian     */
    /* xi^3).  4 regions.                                                       */
    for (int reg = 0; reg < 4; ++reg)
        for (int a = 0; a < g; ++a)
            for (int b = 0; b < g; ++b)
                for (int c = 0; c < g; ++c)
                    for (int d = 0; d < g; ++d) {
                        double xi = gx[a], e1 = gx[b], e2 = gx[c], e3 = gx[d];
                        double v4[4];
                        int k = 0;
                        for (int t = 0; t < 4; ++t) {
                            if (t == reg) v4[t] = xi;
                            else v4[t] = xi * (k == 0 ? e1 : (k == 1 ? e2 : e3)), ++k;
                        }
                        double W = gw[a] * gw[b] * gw[c] * gw[d] * xi * xi * xi;
                        double lx1, lx2, ly1, ly2;
                        frame_map(pi.oE, pi.aE, pi.bE, v4[0], v4[1], &lx1, &lx2);
                        frame_map(pi.oF, pi.aF, pi.bF, v4[2], v4[3], &ly1, &ly2);
                        accumulate(P, E, F, lx1, lx2, ly1, ly2, W, blk);
                    }
}

/* Symmetric convention: the block of an ordered pair is computed for        */
/* (min, max) in global element order and transposed when E > F; identical  */
/* blocks are symmetrised as (B + B^T)/2.                                      */
static void pair_block_sym(const or_problem *P, int E, int F, cplx *out)
{
    int nl = P->nloc;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * nl * nl);
    if (E <= F) {
        or_pair_block(P, E, F, tmp);
        if (E == F) {
            for (int a = 0; a < nl; ++a)
                for (int b = 0; b < nl; ++b) out[a * nl + b] = 0.5 * (tmp[a * nl + b] + tmp[b * nl + a]);
        } else {
            memcpy(out, tmp, sizeof(cplx) * nl * nl);
        }
    } else {
        or_pair_block(P, F, E, tmp);
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nl; ++b) out[a * nl + b] = tmp[b * nl + a];
    }
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Cluster tree and block partition (Sec. 4.1; Sec. 4.2 Def.).               */
/* Cluster (patch, l, k1, k2) covers [k1,k1+1]x[k2,k2+1] * 2^-l.              */
/* Readings: diam and dist are taken over the images of a 5x5 uniform grid   */
/* of the cluster's parameter square (corners included); admissible iff       */
/* max(diam, diam') < eta * dist.  Option (not in the paper): with kdmax > 0 */
/* a block must also satisfy kappa * max(diam, diam') <= kdmax.              */
/* Far field = admissible blocks whose                                        */
/* parents are not admissible; near field = non-admissible leaf blocks.       */
/* ------------------------------------------------------------------------ */
static void cluster_decode(const or_problem *P, int l, int id, int *patch, int *k1, int *k2)
{
    int n = ipow2(l);
    *patch = id / (n * n);
    int r = id % (n * n);
    *k2 = r / n;
    *k1 = r % n;
}

typedef struct {
    double *pts;  /* ncl x 25 x 3 */
    double *diam; /* ncl */
} level_grid;

static void build_level_grid(const or_problem *P, int l, level_grid *G)
{
    int ncl = ncl_level(P, l);
    double sc = 1.0 / ipow2(l);
    G->pts = (double *)malloc(sizeof(double) * ncl * 75);
    G->diam = (double *)malloc(sizeof(double) * ncl);
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < ncl; ++c) {
        int patch, k1, k2;
        cluster_decode(P, l, c, &patch, &k1, &k2);
        double kap;
        for (int b = 0; b < 5; ++b)
            for (int a = 0; a < 5; ++a)
                geom(P, patch, (k1 + 0.25 * a) * sc, (k2 + 0.25 * b) * sc, G->pts + (size_t)c * 75 + 3 * (b * 5 + a), &kap);
        double d = 0.0;
        for (int i = 0; i < 25; ++i)
            for (int j = i + 1; j < 25; ++j) {
                double t = dist3(G->pts + (size_t)c * 75 + 3 * i, G->pts + (size_t)c * 75 + 3 * j);
                if (t > d) d = t;
            }
        G->diam[c] = d;
    }
}

static int admissible(const or_problem *P, const level_grid *G, int a, int b)
{
    double md = fmax(G->diam[a], G->diam[b]);
    if (P->kdmax > 0 && P->kernel == OR_HELMHOLTZ && P->kappa * md > P->kdmax) return 0;
    double dmin = 1e300;
    for (int i = 0; i < 25; ++i)
        for (int j = 0; j < 25; ++j) {
            double t = dist3(G->pts + (size_t)a * 75 + 3 * i, G->pts + (size_t)b * 75 + 3 * j);
            if (t < dmin) dmin = t;
        }
    return md < P->eta * dmin;
}

static int child_id(int l, int id, int c1, int c2, int npatch_unused)
{
    (void)npatch_unused;
    int n = ipow2(l);
    int patch = id / (n * n), r = id % (n * n);
    int k2 = r / n, k1 = r % n;
    int nn = 2 * n;
    return patch * nn * nn + (2 * k2 + c2) * nn + (2 * k1 + c1);
}

static int cmp_block(const void *x, const void *y)
{
    const or_block *a = (const or_block *)x, *b = (const or_block *)y;
    if (a->level != b->level) return a->level - b->level;
    if (a->tgt != b->tgt) return a->tgt - b->tgt;
    return a->src - b->src;
}

static void build_partition(or_problem *P)
{
    int64_t cap = (int64_t)P->npatch * P->npatch;
    or_block *cur = (or_block *)malloc(sizeof(or_block) * cap);
    int64_t ncur = 0;
    for (int i = 0; i < P->npatch; ++i)
        for (int j = 0; j < P->npatch; ++j) cur[ncur++] = (or_block){0, i, j};
    int64_t farcap = 1024, nearcap = 1024;
    P->far = (or_block *)malloc(sizeof(or_block) * farcap);
    P->near = (or_block *)malloc(sizeof(or_block) * nearcap);
    P->nfar = P->nnear = 0;
    for (int l = 0; l <= P->L; ++l) {
        level_grid G;
        build_level_grid(P, l, &G);
        char *adm = (char *)malloc(ncur > 0 ? ncur : 1);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < ncur; ++k) adm[k] = (char)admissible(P, &G, cur[k].tgt, cur[k].src);
        int64_t nnext = 0;
        for (int64_t k = 0; k < ncur; ++k) {
            if (adm[k]) {
                if (P->nfar == farcap) { farcap *= 2; P->far = (or_block *)realloc(P->far, sizeof(or_block) * farcap); }
                P->far[P->nfar++] = cur[k];
            } else if (l == P->L) {
                if (P->nnear == nearcap) { nearcap *= 2; P->near = (or_block *)realloc(P->near, sizeof(or_block) * nearcap); }
                P->near[P->nnear++] = cur[k];
            } else {
                nnext += 16;
            }
        }
        if (l < P->L) {
            or_block *nxt = (or_block *)malloc(sizeof(or_block) * (nnext > 0 ? nnext : 1));
            int64_t t = 0;
            for (int64_t k = 0; k < ncur; ++k) {
                if (adm[k]) continue;
                for (int a2 = 0; a2 < 2; ++a2)
                    for (int a1 = 0; a1 < 2; ++a1)
                        for (int b2 = 0; b2 < 2; ++b2)
                            for (int b1 = 0; b1 < 2; ++b1)
                                nxt[t++] = (or_block){l + 1, child_id(l, cur[k].tgt, a1, a2, P->npatch),
                                                      child_id(l, cur[k].src, b1, b2, P->npatch)};
            }
            free(cur);
            cur = nxt;
            ncur = nnext;
        }
        free(adm);
        free(G.pts);
        free(G.diam);
    }
    free(cur);
    qsort(P->far, P->nfar, sizeof(or_block), cmp_block);
    qsort(P->near, P->nnear, sizeof(or_block), cmp_block);
    /* per-level CSR of far blocks for lookups */
    P->far_ptr = (int64_t **)calloc(P->L + 1, sizeof(int64_t *));
    P->far_src = (int **)calloc(P->L + 1, sizeof(int *));
    P->far_id = (int64_t **)calloc(P->L + 1, sizeof(int64_t *));
    for (int l = 0; l <= P->L; ++l) {
        int ncl = ncl_level(P, l);
        P->far_ptr[l] = (int64_t *)calloc(ncl + 1, sizeof(int64_t));
        int64_t cnt = 0;
        for (int64_t k = 0; k < P->nfar; ++k)
            if (P->far[k].level == l) { P->far_ptr[l][P->far[k].tgt + 1]++; ++cnt; }
        for (int c = 0; c < ncl; ++c) P->far_ptr[l][c + 1] += P->far_ptr[l][c];
        P->far_src[l] = (int *)malloc(sizeof(int) * (cnt > 0 ? cnt : 1));
        P->far_id[l] = (int64_t *)malloc(sizeof(int64_t) * (cnt > 0 ? cnt : 1));
        int64_t t = 0;
        for (int64_t k = 0; k < P->nfar; ++k)
            if (P->far[k].level == l) { P->far_src[l][t] = P->far[k].src; P->far_id[l][t] = k; ++t; }
    }
}

/* far block id of (tgt, src) at level l, or -1 */
static int64_t far_lookup(const or_problem *P, int l, int tgt, int src)
{
    int64_t lo = P->far_ptr[l][tgt], hi = P->far_ptr[l][tgt + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int s = P->far_src[l][mid];
        if (s == src) return P->far_id[l][mid];
        if (s < src) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* cluster at level l containing element E */
static int elem_cluster(const or_problem *P, int E, int l)
{
    int patch, e1, e2;
    elem_decode(P, E, &patch, &e1, &e2);
    int sh = P->m - l;
    int n = ipow2(l);
    return patch * n * n + (e2 >> sh) * n + (e1 >> sh);
}

/* ------------------------------------------------------------------------ */
/* Interpolation: tensor Chebyshev nodes of the first kind on [0,1] (reading */
/* of the unnamed interpolation points, Sec. 4.2), q per direction, and the  */
/* Lagrange basis.                                                            */
/* ------------------------------------------------------------------------ */
static double lagrange(const or_problem *P, int mu, double s)
{
    double v = 1.0;
    for (int k = 0; k < P->q; ++k)
        if (k != mu) v *= (s - P->z[k]) / (P->z[mu] - P->z[k]);
    return v;
}

/* 1D moment of the Bernstein function r on local element el (of nsub per    */
/* cluster side) against L_mu, over the cluster's unit interval:              */
/*   int_0^1 L_mu(s) B_r(nsub s - el) ds, exact Gauss rule.                    */
static double moment1d(const or_problem *P, int nsub, int el, int r, int mu)
{
    int ng = (P->q + P->p + 1) / 2 + 1;
    double gx[64], gw[64];
    or_gauss(ng, gx, gw);
    double s = 0.0;
    for (int i = 0; i < ng; ++i) s += gw[i] * lagrange(P, mu, (el + gx[i]) / nsub) * bernstein(P->p, r, gx[i]);
    return s / nsub;
}

/* Chebyshev node geometry of a cluster: point and surface measure at        */
/* chi_lambda(z_mu), mu = mu2*q + mu1.                                        */
static void cluster_nodes(const or_problem *P, int l, int id, double *X, double *kap)
{
    int patch, k1, k2;
    cluster_decode(P, l, id, &patch, &k1, &k2);
    double sc = 1.0 / ipow2(l);
    for (int m2 = 0; m2 < P->q; ++m2)
        for (int m1 = 0; m1 < P->q; ++m1) {
            int mu = m2 * P->q + m1;
            geom(P, patch, (k1 + P->z[m1]) * sc, (k2 + P->z[m2]) * sc, X + 3 * mu, kap + mu);
        }
}

/* Coupling block of an admissible pair (Sec. 4.2): the localised kernel     */
/* (fundamental solution composed with the geometry, times both surface      */
/* measures and the affine Jacobians 4^-l of the cluster maps) at the        */
/* interpolation node pairs.  K[mu*q^2 + nu].                                 */
void or_coupling_block(const or_problem *P, int l, int tgt, int src, cplx *K)
{
    int q2 = P->q * P->q;
    double *X = (double *)malloc(sizeof(double) * 3 * q2), *Y = (double *)malloc(sizeof(double) * 3 * q2);
    double *kx = (double *)malloc(sizeof(double) * q2), *ky = (double *)malloc(sizeof(double) * q2);
    cluster_nodes(P, l, tgt, X, kx);
    cluster_nodes(P, l, src, Y, ky);
    double jac = 1.0 / ((double)ipow2(l) * ipow2(l));
    for (int a = 0; a < q2; ++a)
        for (int b = 0; b < q2; ++b) K[(size_t)a * q2 + b] = fundamental(P, X + 3 * a, Y + 3 * b) * kx[a] * ky[b] * jac * jac;
    free(X); free(Y); free(kx); free(ky);
}

/* ------------------------------------------------------------------------ */
/* creation                                                                   */
/* ------------------------------------------------------------------------ */
or_problem *or_create(int npatch, const int *deg, const int *ncp, const double *knots, const double *cpw, int kernel,
                      double kappa, int p, int m, int q, double eta, double kdmax, int leaf_depth, int g0, int gs,
                      int grhs, int nthreads)
{
    if (npatch < 1 || p < 0 || p > 8 || m < 0 || m > 12 || q < 1 || q > 24 || !(eta > 0) || !(kdmax >= 0) || g0 < 1 ||
        g0 > 40)
        return NULL;
    or_problem *P = (or_problem *)calloc(1, sizeof(or_problem));
    P->npatch = npatch;
    P->kernel = kernel;
    P->kappa = kappa;
    P->p = p;
    P->m = m;
    P->q = q;
    P->eta = eta;
    P->kdmax = kdmax;
    P->g0 = g0;
    P->gs = gs > 0 ? gs : (g0 + 2 > 40 ? 40 : g0 + 2);
    P->grhs = grhs > 0 ? grhs : (g0 > p + 4 ? g0 : p + 4);
    P->nthreads = nthreads;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    P->patches = (or_patch *)calloc(npatch, sizeof(or_patch));
    const double *kp = knots, *cp = cpw;
    for (int i = 0; i < npatch; ++i) {
        or_patch *pt = &P->patches[i];
        pt->pu = deg[2 * i];
        pt->pv = deg[2 * i + 1];
        pt->nu = ncp[2 * i];
        pt->nv = ncp[2 * i + 1];
        int nku = pt->nu + pt->pu + 1, nkv = pt->nv + pt->pv + 1;
        pt->U = (double *)malloc(sizeof(double) * nku);
        pt->V = (double *)malloc(sizeof(double) * nkv);
        memcpy(pt->U, kp, sizeof(double) * nku);
        kp += nku;
        memcpy(pt->V, kp, sizeof(double) * nkv);
        kp += nkv;
        pt->cpw = (double *)malloc(sizeof(double) * 4 * pt->nu * pt->nv);
        memcpy(pt->cpw, cp, sizeof(double) * 4 * pt->nu * pt->nv);
        cp += 4 * pt->nu * pt->nv;
    }
    P->nel1 = 1 << m;
    P->h = 1.0 / P->nel1;
    P->nelem = npatch * P->nel1 * P->nel1;
    P->nloc = (p + 1) * (p + 1);
    P->nsup = P->nelem * P->nloc;
    P->ns1 = P->nel1 + p;
    P->ndof = npatch * P->ns1 * P->ns1;
    /* leaf depth d (reading): smallest d with (p+1)^2 4^d >= q^2, at most m */
    int d = leaf_depth;
    if (d < 0) {
        d = 0;
        while ((p + 1) * (p + 1) * (1 << (2 * d)) < q * q && d < m) ++d;
    }
    if (d > m) d = m;
    P->L = m - d;
    P->z = (double *)malloc(sizeof(double) * q);
    for (int k = 0; k < q; ++k) P->z[k] = 0.5 * (1.0 + cos((2.0 * k + 1.0) * M_PI / (2.0 * q)));
    build_T1(P);
    build_elements(P);
    build_partition(P);
    return P;
}

void or_destroy(or_problem *P)
{
    if (!P) return;
    for (int i = 0; i < P->npatch; ++i) {
        free(P->patches[i].U);
        free(P->patches[i].V);
        free(P->patches[i].cpw);
    }
    free(P->patches);
    free(P->T1); free(P->corner); free(P->grid9); free(P->ediam); free(P->z);
    free(P->near); free(P->far);
    if (P->far_ptr)
        for (int l = 0; l <= P->L; ++l) { free(P->far_ptr[l]); free(P->far_src[l]); free(P->far_id[l]); }
    free(P->far_ptr); free(P->far_src); free(P->far_id);
    free(P->nb_ptr); free(P->nb_idx); free(P->nb_blk); free(P->far_K);
    free(P);
}

/* info: ndof, nsup, nelem, nloc, L, nnear, nfar, nrhs_points, gs, grhs, ns1 */
void or_info(const or_problem *P, int64_t *out)
{
    out[0] = P->ndof; out[1] = P->nsup; out[2] = P->nelem; out[3] = P->nloc; out[4] = P->L;
    out[5] = P->nnear; out[6] = P->nfar; out[7] = (int64_t)P->nelem * P->grhs * P->grhs;
    out[8] = P->gs; out[9] = P->grhs; out[10] = P->ns1;
}

void or_export_partition(const or_problem *P, int32_t *near, int32_t *far)
{
    for (int64_t k = 0; k < P->nnear; ++k) { near[2 * k] = P->near[k].tgt; near[2 * k + 1] = P->near[k].src; }
    for (int64_t k = 0; k < P->nfar; ++k) {
        far[3 * k] = P->far[k].level; far[3 * k + 1] = P->far[k].tgt; far[3 * k + 2] = P->far[k].src;
    }
}

void or_T1(const or_problem *P, double *out)
{
    memcpy(out, P->T1, sizeof(double) * (size_t)P->ns1 * P->nel1 * (P->p + 1));
}

void or_chebyshev_nodes(const or_problem *P, double *out) { memcpy(out, P->z, sizeof(double) * P->q); }

/* geometry at patch parameters: out[i] = x,y,z,kappa */
void or_geometry(const or_problem *P, int patch, int n, const double *uv, double *out)
{
    for (int i = 0; i < n; ++i) geom(P, patch, uv[2 * i], uv[2 * i + 1], out + 4 * i, out + 4 * i + 3);
}

void or_pair_class(const or_problem *P, int E, int F, int32_t *out)
{
    pair_info pi = classify(P, E, F);
    out[0] = pi.cls; out[1] = pi.order;
    out[2] = pi.oE; out[3] = pi.aE; out[4] = pi.bE; out[5] = pi.oF; out[6] = pi.aF; out[7] = pi.bF;
}

/* element pair block with the symmetric convention, complex interleaved */
void or_pair_block_sym(const or_problem *P, int E, int F, double *out)
{
    pair_block_sym(P, E, F, (cplx *)out);
}

/* ------------------------------------------------------------------------ */
/* T and T^T (Sec. 4.3).  S dof: patch*ns1^2 + j2*ns1 + j1.  S* dof:          */
/* (patch*4^m + e2*2^m + e1)*(p+1)^2 + r2*(p+1) + r1.  ncomp = 1 (real) or 2  */
/* (complex interleaved).                                                     */
/* ------------------------------------------------------------------------ */
void or_apply_T(const or_problem *P, int ncomp, const double *xs, double *y)
{
    int p = P->p, ne = P->nel1, ns1 = P->ns1, pp = p + 1, nr = ne * pp;
    memset(y, 0, sizeof(double) * ncomp * P->ndof);
    for (int pt = 0; pt < P->npatch; ++pt)
        for (int j2 = 0; j2 < ns1; ++j2)
            for (int j1 = 0; j1 < ns1; ++j1)
                for (int e2 = 0; e2 < ne; ++e2)
                    for (int r2 = 0; r2 < pp; ++r2) {
                        double t2 = P->T1[(size_t)j2 * nr + e2 * pp + r2];
                        if (t2 == 0.0) continue;
                        for (int e1 = 0; e1 < ne; ++e1)
                            for (int r1 = 0; r1 < pp; ++r1) {
                                double t1 = P->T1[(size_t)j1 * nr + e1 * pp + r1];
                                if (t1 == 0.0) continue;
                                size_t a = ((size_t)(pt * ne * ne + e2 * ne + e1)) * P->nloc + r2 * pp + r1;
                                size_t i = (size_t)pt * ns1 * ns1 + j2 * ns1 + j1;
                                for (int c = 0; c < ncomp; ++c) y[ncomp * i + c] += t1 * t2 * xs[ncomp * a + c];
                            }
                    }
}

void or_apply_Tt(const or_problem *P, int ncomp, const double *w, double *xs)
{
    int p = P->p, ne = P->nel1, ns1 = P->ns1, pp = p + 1, nr = ne * pp;
    memset(xs, 0, sizeof(double) * ncomp * P->nsup);
    for (int pt = 0; pt < P->npatch; ++pt)
        for (int j2 = 0; j2 < ns1; ++j2)
            for (int j1 = 0; j1 < ns1; ++j1)
                for (int e2 = 0; e2 < ne; ++e2)
                    for (int r2 = 0; r2 < pp; ++r2) {
                        double t2 = P->T1[(size_t)j2 * nr + e2 * pp + r2];
                        if (t2 == 0.0) continue;
                        for (int e1 = 0; e1 < ne; ++e1)
                            for (int r1 = 0; r1 < pp; ++r1) {
                                double t1 = P->T1[(size_t)j1 * nr + e1 * pp + r1];
                                if (t1 == 0.0) continue;
                                size_t a = ((size_t)(pt * ne * ne + e2 * ne + e1)) * P->nloc + r2 * pp + r1;
                                size_t i = (size_t)pt * ns1 * ns1 + j2 * ns1 + j1;
                                for (int c = 0; c < ncomp; ++c) xs[ncomp * a + c] += t1 * t2 * w[ncomp * i + c];
                            }
                    }
}

/* ------------------------------------------------------------------------ */
/* Dense Galerkin matrix A* over S* (all element pairs), complex interleaved */
/* row-major nsup x nsup.                                                     */
/* ------------------------------------------------------------------------ */
void or_dense_assemble(const or_problem *P, double *Aout)
{
    cplx *A = (cplx *)Aout;
    int nl = P->nloc;
    int64_t ns = P->nsup;
    int ne = P->nelem;
#pragma omp parallel
    {
        cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < (int64_t)ne * ne; ++k) {
            int E = (int)(k / ne), F = (int)(k % ne);
            if (E > F) continue;
            pair_block_sym(P, E, F, blk);
            for (int a = 0; a < nl; ++a)
                for (int b = 0; b < nl; ++b) {
                    A[((int64_t)E * nl + a) * ns + (int64_t)F * nl + b] = blk[a * nl + b];
                    A[((int64_t)F * nl + b) * ns + (int64_t)E * nl + a] = blk[a * nl + b];
                }
        }
        free(blk);
    }
}

/* ------------------------------------------------------------------------ */
/* Right-hand side (Sec. 3.2): g*_a = int g(F x) k(x) phi_a(x) dx with tensor */
/* Gauss of order grhs per element.  Points: element-major, then v-node      */
/* outer, u-node inner.                                                       */
/* ------------------------------------------------------------------------ */
void or_rhs_points(const or_problem *P, double *xyz)
{
    double gx[64], gw[64];
    or_gauss(P->grhs, gx, gw);
    int g = P->grhs;
    for (int E = 0; E < P->nelem; ++E)
        for (int j = 0; j < g; ++j)
            for (int i = 0; i < g; ++i) {
                int patch;
                double u, v, k;
                elem_param(P, E, gx[i], gx[j], &patch, &u, &v);
                geom(P, patch, u, v, xyz + 3 * ((size_t)E * g * g + j * g + i), &k);
            }
}

void or_rhs(const or_problem *P, const double *gvals, double *gstar_out)
{
    cplx *gs = (cplx *)gstar_out;
    const cplx *gv = (const cplx *)gvals;
    double gx[64], gw[64];
    int g = P->grhs, p = P->p;
    or_gauss(g, gx, gw);
    for (int64_t a = 0; a < P->nsup; ++a) gs[a] = 0.0;
    for (int E = 0; E < P->nelem; ++E)
        for (int j = 0; j < g; ++j)
            for (int i = 0; i < g; ++i) {
                int patch;
                double u, v, k, X[3];
                elem_param(P, E, gx[i], gx[j], &patch, &u, &v);
                geom(P, patch, u, v, X, &k);
                cplx val = gv[(size_t)E * g * g + j * g + i] * k * P->h * P->h * gw[i] * gw[j];
                for (int r2 = 0; r2 <= p; ++r2)
                    for (int r1 = 0; r1 <= p; ++r1)
                        gs[(size_t)E * P->nloc + r2 * (p + 1) + r1] += val * bernstein(p, r1, gx[i]) * bernstein(p, r2, gx[j]);
            }
}

/* ------------------------------------------------------------------------ */
/* H2 operator, non-nested form (Sec. 4.2):                                   */
/*   y* = A_near x* + sum_{far (l,t,s)} V_t K_ts V_s^T x*                      */
/* with V_c[a,mu] = int_[0,1]^2 L_mu(s) phi_a(chi_c s) ds computed directly   */
/* for every function a in cluster c at every level.                          */
/* ------------------------------------------------------------------------ */
static void build_near_csr(or_problem *P)
{
    if (P->nb_ptr) return;
    int ne = P->nelem;
    int d = P->m - P->L, side = 1 << d;
    int per = side * side;
    P->nb_ptr = (int64_t *)calloc(ne + 1, sizeof(int64_t));
    /* each near leaf pair contributes per*per element pairs */
    for (int64_t k = 0; k < P->nnear; ++k) {
        int patch, k1, k2;
        cluster_decode(P, P->L, P->near[k].tgt, &patch, &k1, &k2);
        for (int a2 = 0; a2 < side; ++a2)
            for (int a1 = 0; a1 < side; ++a1) {
                int E = patch * P->nel1 * P->nel1 + (k2 * side + a2) * P->nel1 + k1 * side + a1;
                P->nb_ptr[E + 1] += per;
            }
    }
    for (int E = 0; E < ne; ++E) P->nb_ptr[E + 1] += P->nb_ptr[E];
    P->nb_idx = (int *)malloc(sizeof(int) * (P->nb_ptr[ne] > 0 ? P->nb_ptr[ne] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ne);
    for (int E = 0; E < ne; ++E) fill[E] = P->nb_ptr[E];
    for (int64_t k = 0; k < P->nnear; ++k) {
        int pa, ka1, ka2, pb, kb1, kb2;
        cluster_decode(P, P->L, P->near[k].tgt, &pa, &ka1, &ka2);
        cluster_decode(P, P->L, P->near[k].src, &pb, &kb1, &kb2);
        for (int a2 = 0; a2 < side; ++a2)
            for (int a1 = 0; a1 < side; ++a1) {
                int E = pa * P->nel1 * P->nel1 + (ka2 * side + a2) * P->nel1 + ka1 * side + a1;
                for (int b2 = 0; b2 < side; ++b2)
                    for (int b1 = 0; b1 < side; ++b1)
                        P->nb_idx[fill[E]++] = pb * P->nel1 * P->nel1 + (kb2 * side + b2) * P->nel1 + kb1 * side + b1;
            }
    }
    free(fill);
}

/* assemble all near-field blocks and (optionally) store all coupling blocks */
void or_h2_assemble(or_problem *P, int store_coupling)
{
    build_near_csr(P);
    int nl = P->nloc;
    int64_t nnz = P->nb_ptr[P->nelem];
    if (!P->nb_blk) {
        P->nb_blk = (cplx *)malloc(sizeof(cplx) * nl * nl * (nnz > 0 ? nnz : 1));
#pragma omp parallel for schedule(dynamic, 1)
        for (int E = 0; E < P->nelem; ++E)
            for (int64_t k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k)
                pair_block_sym(P, E, P->nb_idx[k], P->nb_blk + k * nl * nl);
    }
    if (store_coupling && !P->far_K) {
        int64_t q4 = (int64_t)P->q * P->q * P->q * P->q;
        P->far_K = (cplx *)malloc(sizeof(cplx) * q4 * (P->nfar > 0 ? P->nfar : 1));
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t k = 0; k < P->nfar; ++k)
            or_coupling_block(P, P->far[k].level, P->far[k].tgt, P->far[k].src, P->far_K + k * q4);
    }
}

/* X^_c = V_c^T x* for all clusters of level l (direct, non-nested) */
static void level_moments(const or_problem *P, int l, const cplx *xs, cplx *Xh)
{
    int q = P->q, q2 = q * q, p = P->p, pp = p + 1;
    int ncl = ncl_level(P, l);
    int nsub = 1 << (P->m - l);
    double *M = (double *)malloc(sizeof(double) * nsub * pp * q); /* M[(el*pp + r)*q + mu] */
    for (int el = 0; el < nsub; ++el)
        for (int r = 0; r < pp; ++r)
            for (int mu = 0; mu < q; ++mu) M[(el * pp + r) * q + mu] = moment1d(P, nsub, el, r, mu);
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < ncl; ++c) {
        int patch, k1, k2;
        cluster_decode(P, l, c, &patch, &k1, &k2);
        cplx *out = Xh + (size_t)c * q2;
        for (int mu = 0; mu < q2; ++mu) out[mu] = 0.0;
        for (int el2 = 0; el2 < nsub; ++el2)
            for (int el1 = 0; el1 < nsub; ++el1) {
                int E = patch * P->nel1 * P->nel1 + (k2 * nsub + el2) * P->nel1 + k1 * nsub + el1;
                for (int r2 = 0; r2 < pp; ++r2)
                    for (int r1 = 0; r1 < pp; ++r1) {
                        cplx xv = xs[(size_t)E * P->nloc + r2 * pp + r1];
                        if (xv == 0.0) continue;
                        for (int m2 = 0; m2 < q; ++m2)
                            for (int m1 = 0; m1 < q; ++m1)
                                out[m2 * q + m1] += M[(el1 * pp + r1) * q + m1] * M[(el2 * pp + r2) * q + m2] * xv;
                    }
            }
    }
    free(M);
}

/* y*_a += sum_mu V_c[a,mu] Y^_c[mu] for all clusters of level l (direct) */
static void level_backmoments(const or_problem *P, int l, const cplx *Yh, cplx *ys)
{
    int q = P->q, q2 = q * q, p = P->p, pp = p + 1;
    int ncl = ncl_level(P, l);
    int nsub = 1 << (P->m - l);
    double *M = (double *)malloc(sizeof(double) * nsub * pp * q);
    for (int el = 0; el < nsub; ++el)
        for (int r = 0; r < pp; ++r)
            for (int mu = 0; mu < q; ++mu) M[(el * pp + r) * q + mu] = moment1d(P, nsub, el, r, mu);
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < ncl; ++c) {
        int patch, k1, k2;
        cluster_decode(P, l, c, &patch, &k1, &k2);
        const cplx *in = Yh + (size_t)c * q2;
        int any = 0;
        for (int mu = 0; mu < q2; ++mu) if (in[mu] != 0.0) { any = 1; break; }
        if (!any) continue;
        for (int el2 = 0; el2 < nsub; ++el2)
            for (int el1 = 0; el1 < nsub; ++el1) {
                int E = patch * P->nel1 * P->nel1 + (k2 * nsub + el2) * P->nel1 + k1 * nsub + el1;
                for (int r2 = 0; r2 < pp; ++r2)
                    for (int r1 = 0; r1 < pp; ++r1) {
                        cplx s = 0.0;
                        for (int m2 = 0; m2 < q; ++m2)
                            for (int m1 = 0; m1 < q; ++m1)
                                s += M[(el1 * pp + r1) * q + m1] * M[(el2 * pp + r2) * q + m2] * in[m2 * q + m1];
                        ys[(size_t)E * P->nloc + r2 * pp + r1] += s;
                    }
            }
    }
    free(M);
}

/* y* = A_H2 x* (S* vectors, complex interleaved) */
void or_h2_matvec_super(or_problem *P, const double *xsd, double *ysd)
{
    or_h2_assemble(P, 0);
    const cplx *xs = (const cplx *)xsd;
    cplx *ys = (cplx *)ysd;
    int nl = P->nloc, q2 = P->q * P->q;
    int64_t q4 = (int64_t)q2 * q2;
    for (int64_t a = 0; a < P->nsup; ++a) ys[a] = 0.0;
    /* near field */
#pragma omp parallel for schedule(dynamic, 8)
    for (int E = 0; E < P->nelem; ++E)
        for (int64_t k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k) {
            int F = P->nb_idx[k];
            const cplx *B = P->nb_blk + k * nl * nl;
            for (int a = 0; a < nl; ++a) {
                cplx s = 0.0;
                for (int b = 0; b < nl; ++b) s += B[a * nl + b] * xs[(size_t)F * nl + b];
                ys[(size_t)E * nl + a] += s;
            }
        }
    /* far field, level by level */
    for (int l = 0; l <= P->L; ++l) {
        int64_t nb = P->far_ptr[l][ncl_level(P, l)];
        if (nb == 0) continue;
        int ncl = ncl_level(P, l);
        cplx *Xh = (cplx *)malloc(sizeof(cplx) * q2 * ncl);
        cplx *Yh = (cplx *)calloc((size_t)q2 * ncl, sizeof(cplx));
        level_moments(P, l, xs, Xh);
#pragma omp parallel
        {
            cplx *K = P->far_K ? NULL : (cplx *)malloc(sizeof(cplx) * q4);
#pragma omp for schedule(dynamic, 1)
            for (int t = 0; t < ncl; ++t)
                for (int64_t k = P->far_ptr[l][t]; k < P->far_ptr[l][t + 1]; ++k) {
                    int s = P->far_src[l][k];
                    int64_t id = P->far_id[l][k];
                    const cplx *Kb;
                    if (P->far_K) Kb = P->far_K + id * q4;
                    else { or_coupling_block(P, l, t, s, K); Kb = K; }
                    for (int a = 0; a < q2; ++a) {
                        cplx acc = 0.0;
                        for (int b = 0; b < q2; ++b) acc += Kb[(size_t)a * q2 + b] * Xh[(size_t)s * q2 + b];
                        Yh[(size_t)t * q2 + a] += acc;
                    }
                }
            free(K);
        }
        level_backmoments(P, l, Yh, ys);
        free(Xh);
        free(Yh);
    }
}

/* Row-sampled H2 matvec: y* restricted to the given target leaves           */
/* (nleaf ids at level L), written leaf after leaf, elements of a leaf in     */
/* row-major order within the leaf, nloc values each.  No full assembly.      */
void or_h2_matvec_rows(or_problem *P, const double *xsd, int nleaf, const int32_t *leaves, double *outd)
{
    build_near_csr(P);
    const cplx *xs = (const cplx *)xsd;
    cplx *out = (cplx *)outd;
    int nl = P->nloc, q2 = P->q * P->q, q = P->q, pp = P->p + 1;
    int64_t q4 = (int64_t)q2 * q2;
    int side = 1 << (P->m - P->L), per = side * side;
    for (int64_t i = 0; i < (int64_t)nleaf * per * nl; ++i) out[i] = 0.0;
    /* moments at every level */
    cplx **Xh = (cplx **)calloc(P->L + 1, sizeof(cplx *));
    for (int l = 0; l <= P->L; ++l) {
        Xh[l] = (cplx *)malloc(sizeof(cplx) * q2 * ncl_level(P, l));
        level_moments(P, l, xs, Xh[l]);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int li = 0; li < nleaf; ++li) {
        int leaf = leaves[li];
        int patch, k1, k2;
        cluster_decode(P, P->L, leaf, &patch, &k1, &k2);
        cplx *blk = (cplx *)malloc(sizeof(cplx) * nl * nl);
        cplx *K = (cplx *)malloc(sizeof(cplx) * q4);
        cplx *Yh = (cplx *)malloc(sizeof(cplx) * q2);
        for (int a2 = 0; a2 < side; ++a2)
            for (int a1 = 0; a1 < side; ++a1) {
                int E = patch * P->nel1 * P->nel1 + (k2 * side + a2) * P->nel1 + k1 * side + a1;
                cplx *o = out + ((size_t)li * per + a2 * side + a1) * nl;
                for (int64_t k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k) {
                    int F = P->nb_idx[k];
                    pair_block_sym(P, E, F, blk);
                    for (int a = 0; a < nl; ++a) {
                        cplx s = 0.0;
                        for (int b = 0; b < nl; ++b) s += blk[a * nl + b] * xs[(size_t)F * nl + b];
                        o[a] += s;
                    }
                }
            }
        /* far contributions through each ancestor */
        for (int l = 0; l <= P->L; ++l) {
            int sh = P->L - l;
            int n = 1 << l;
            int anc = patch * n * n + (k2 >> sh) * n + (k1 >> sh);
            int64_t b0 = P->far_ptr[l][anc], b1 = P->far_ptr[l][anc + 1];
            if (b0 == b1) continue;
            for (int mu = 0; mu < q2; ++mu) Yh[mu] = 0.0;
            for (int64_t k = b0; k < b1; ++k) {
                int s = P->far_src[l][k];
                or_coupling_block(P, l, anc, s, K);
                for (int a = 0; a < q2; ++a) {
                    cplx acc = 0.0;
                    for (int b = 0; b < q2; ++b) acc += K[(size_t)a * q2 + b] * Xh[l][(size_t)s * q2 + b];
                    Yh[a] += acc;
                }
            }
            /* back-moments for the functions of this leaf inside ancestor anc */
            int nsub = 1 << (P->m - l);
            int ka1 = (k1 >> sh) * nsub, ka2 = (k2 >> sh) * nsub; /* first element of anc */
            for (int a2 = 0; a2 < side; ++a2)
                for (int a1 = 0; a1 < side; ++a1) {
                    int e1 = k1 * side + a1, e2 = k2 * side + a2;
                    int el1 = e1 - ka1, el2 = e2 - ka2;
                    cplx *o = out + ((size_t)li * per + a2 * side + a1) * nl;
                    for (int r2 = 0; r2 < pp; ++r2)
                        for (int r1 = 0; r1 < pp; ++r1) {
                            cplx s = 0.0;
                            for (int m2 = 0; m2 < q; ++m2) {
                                double v2 = moment1d(P, nsub, el2, r2, m2);
                                for (int m1 = 0; m1 < q; ++m1)
                                    s += moment1d(P, nsub, el1, r1, m1) * v2 * Yh[m2 * q + m1];
                            }
                            o[r2 * pp + r1] += s;
                        }
                }
        }
        free(blk); free(K); free(Yh);
    }
    for (int l = 0; l <= P->L; ++l) free(Xh[l]);
    free(Xh);
}

/* ------------------------------------------------------------------------ */
/* Operators in S:  y = T A T^T w  (dense: A = A*; h2: A = A_H2).             */
/* ------------------------------------------------------------------------ */
typedef struct {
    or_problem *P;
    const cplx *Adense; /* nsup x nsup or NULL (H2) */
} op_ctx;

static void op_apply(const op_ctx *C, const cplx *w, cplx *y)
{
    or_problem *P = C->P;
    cplx *xs = (cplx *)malloc(sizeof(cplx) * P->nsup);
    cplx *ys = (cplx *)malloc(sizeof(cplx) * P->nsup);
    or_apply_Tt(P, 2, (const double *)w, (double *)xs);
    if (C->Adense) {
        int64_t n = P->nsup;
#pragma omp parallel for
        for (int64_t a = 0; a < n; ++a) {
            cplx s = 0.0;
            for (int64_t b = 0; b < n; ++b) s += C->Adense[a * n + b] * xs[b];
            ys[a] = s;
        }
    } else {
        or_h2_matvec_super(P, (const double *)xs, (double *)ys);
    }
    or_apply_T(P, 2, (const double *)ys, (double *)y);
    free(xs);
    free(ys);
}

void or_matvec(or_problem *P, const double *Adense, const double *w, double *y)
{
    op_ctx C = {P, (const cplx *)Adense};
    op_apply(&C, (const cplx *)w, (cplx *)y);
}

/* Jacobi diagonal D_i = t_i^T A t_i, t_i = T^T e_i (exact diagonal of the    */
/* applied operator, far-field terms included).                               */
void or_jacobi_diag(or_problem *P, const double *Adense, double *Dout)
{
    cplx *D = (cplx *)Dout;
    int p = P->p, pp = p + 1, ne = P->nel1, ns1 = P->ns1, nr = ne * pp, nl = P->nloc;
    if (!Adense) or_h2_assemble(P, 0);
    int q2 = P->q * P->q, q = P->q;
    int64_t q4 = (int64_t)q2 * q2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < P->ndof; ++i) {
        int pt = i / (ns1 * ns1), j2 = (i / ns1) % ns1, j1 = i % ns1;
        /* support elements: e in [j-p, j] intersected with [0, ne) per direction */
        int elo1 = j1 - p < 0 ? 0 : j1 - p, ehi1 = j1 < ne - 1 ? j1 : ne - 1;
        int elo2 = j2 - p < 0 ? 0 : j2 - p, ehi2 = j2 < ne - 1 ? j2 : ne - 1;
        int nse = (ehi1 - elo1 + 1) * (ehi2 - elo2 + 1);
        int *el = (int *)malloc(sizeof(int) * nse);
        double *tv = (double *)malloc(sizeof(double) * nse * nl);
        int c = 0;
        for (int e2 = elo2; e2 <= ehi2; ++e2)
            for (int e1 = elo1; e1 <= ehi1; ++e1, ++c) {
                el[c] = pt * ne * ne + e2 * ne + e1;
                for (int r2 = 0; r2 < pp; ++r2)
                    for (int r1 = 0; r1 < pp; ++r1)
                        tv[c * nl + r2 * pp + r1] = P->T1[(size_t)j1 * nr + e1 * pp + r1] * P->T1[(size_t)j2 * nr + e2 * pp + r2];
            }
        cplx s = 0.0;
        if (Adense) {
            const cplx *A = (const cplx *)Adense;
            for (int x = 0; x < nse; ++x)
                for (int y = 0; y < nse; ++y)
                    for (int a = 0; a < nl; ++a)
                        for (int b = 0; b < nl; ++b)
                            s += tv[x * nl + a] * A[((int64_t)el[x] * nl + a) * P->nsup + (int64_t)el[y] * nl + b] * tv[y * nl + b];
        } else {
            cplx *K = (cplx *)malloc(sizeof(cplx) * q4);
            cplx *mx = (cplx *)malloc(sizeof(cplx) * q2), *my = (cplx *)malloc(sizeof(cplx) * q2);
            for (int x = 0; x < nse; ++x)
                for (int y = 0; y < nse; ++y) {
                    int E = el[x], F = el[y];
                    /* near? */
                    int64_t k;
                    int found = 0;
                    for (k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k)
                        if (P->nb_idx[k] == F) { found = 1; break; }
                    if (found) {
                        const cplx *B = P->nb_blk + k * nl * nl;
                        for (int a = 0; a < nl; ++a)
                            for (int b = 0; b < nl; ++b) s += tv[x * nl + a] * B[a * nl + b] * tv[y * nl + b];
                        continue;
                    }
                    for (int l = 0; l <= P->L; ++l) {
                        int cE = elem_cluster(P, E, l), cF = elem_cluster(P, F, l);
                        if (far_lookup(P, l, cE, cF) < 0) continue;
                        or_coupling_block(P, l, cE, cF, K);
                        int nsub = 1 << (P->m - l);
                        int pE, e1E, e2E, pF, e1F, e2F, dummy1, dummy2, dummy3;
                        elem_decode(P, E, &pE, &e1E, &e2E);
                        elem_decode(P, F, &pF, &e1F, &e2F);
                        (void)dummy1; (void)dummy2; (void)dummy3;
                        int elE1 = e1E % nsub, elE2 = e2E % nsub, elF1 = e1F % nsub, elF2 = e2F % nsub;
                        for (int m2 = 0; m2 < q; ++m2)
                            for (int m1 = 0; m1 < q; ++m1) {
                                cplx ax = 0.0, ay = 0.0;
                                for (int r2 = 0; r2 < pp; ++r2)
                                    for (int r1 = 0; r1 < pp; ++r1) {
                                        ax += tv[x * nl + r2 * pp + r1] * moment1d(P, nsub, elE1, r1, m1) * moment1d(P, nsub, elE2, r2, m2);
                                        ay += tv[y * nl + r2 * pp + r1] * moment1d(P, nsub, elF1, r1, m1) * moment1d(P, nsub, elF2, r2, m2);
                                    }
                                mx[m2 * q + m1] = ax;
                                my[m2 * q + m1] = ay;
                            }
                        for (int a = 0; a < q2; ++a)
                            for (int b = 0; b < q2; ++b) s += mx[a] * K[(size_t)a * q2 + b] * my[b];
                        break;
                    }
                }
            free(K); free(mx); free(my);
        }
        D[i] = s;
        free(el);
        free(tv);
    }
}

/* ------------------------------------------------------------------------ */
/* Krylov solvers (Sec. 4, item 3): Jacobi-preconditioned CG (Laplace) and   */
/* right-preconditioned restarted GMRES with modified Gram-Schmidt and Givens */
/* rotations (Helmholtz).  Zero initial guess unless w is given; stop on the  */
/* true relative residual ||b - A w|| <= tol ||b||.                           */
/* ------------------------------------------------------------------------ */
static double vnorm(int n, const cplx *v)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += creal(v[i] * conj(v[i]));
    return sqrt(s);
}

static int solve_cg(const op_ctx *C, const cplx *D, const cplx *b, cplx *w, double tol, int maxit, int *iters,
                    double *relres)
{
    int n = C->P->ndof;
    cplx *r = (cplx *)malloc(sizeof(cplx) * n), *z = (cplx *)malloc(sizeof(cplx) * n);
    cplx *pv = (cplx *)malloc(sizeof(cplx) * n), *Ap = (cplx *)malloc(sizeof(cplx) * n);
    double bn = vnorm(n, b);
    if (bn == 0.0) bn = 1.0;
    int it = 0, done = 0;
    while (!done) {
        op_apply(C, w, Ap);
        for (int i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
        double tr = vnorm(n, r) / bn;
        *relres = tr;
        if (tr <= tol || it >= maxit) break;
        for (int i = 0; i < n; ++i) z[i] = r[i] / D[i];
        for (int i = 0; i < n; ++i) pv[i] = z[i];
        double rz = 0.0;
        for (int i = 0; i < n; ++i) rz += creal(r[i] * z[i]);
        while (it < maxit) {
            op_apply(C, pv, Ap);
            double pAp = 0.0;
            for (int i = 0; i < n; ++i) pAp += creal(pv[i] * Ap[i]);
            double alpha = rz / pAp;
            for (int i = 0; i < n; ++i) { w[i] += alpha * pv[i]; r[i] -= alpha * Ap[i]; }
            ++it;
            if (vnorm(n, r) / bn <= tol) break; /* verified on the true residual above */
            for (int i = 0; i < n; ++i) z[i] = r[i] / D[i];
            double rz2 = 0.0;
            for (int i = 0; i < n; ++i) rz2 += creal(r[i] * z[i]);
            double beta = rz2 / rz;
            rz = rz2;
            for (int i = 0; i < n; ++i) pv[i] = z[i] + beta * pv[i];
        }
    }
    *iters = it;
    free(r); free(z); free(pv); free(Ap);
    return *relres <= tol ? 0 : 1;
}

static int solve_gmres(const op_ctx *C, const cplx *D, const cplx *b, cplx *w, double tol, int maxit, int restart,
                       int *iters, double *relres)
{
    int n = C->P->ndof, mr = restart;
    cplx *V = (cplx *)malloc(sizeof(cplx) * (size_t)n * (mr + 1));
    cplx *H = (cplx *)calloc((size_t)(mr + 1) * mr, sizeof(cplx));
    cplx *cs = (cplx *)malloc(sizeof(cplx) * mr), *sn = (cplx *)malloc(sizeof(cplx) * mr);
    cplx *g = (cplx *)malloc(sizeof(cplx) * (mr + 1)), *yv = (cplx *)malloc(sizeof(cplx) * mr);
    cplx *r = (cplx *)malloc(sizeof(cplx) * n), *t = (cplx *)malloc(sizeof(cplx) * n);
    double bn = vnorm(n, b);
    if (bn == 0.0) bn = 1.0;
    int it = 0;
    for (;;) {
        op_apply(C, w, t);
        for (int i = 0; i < n; ++i) r[i] = b[i] - t[i];
        double beta = vnorm(n, r);
        *relres = beta / bn;
        if (*relres <= tol || it >= maxit) break;
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int k = 0; k <= mr; ++k) g[k] = 0.0;
        g[0] = beta;
        int k;
        for (k = 0; k < mr && it < maxit; ++k, ++it) {
            cplx *vk = V + (size_t)k * n, *vn = V + (size_t)(k + 1) * n;
            for (int i = 0; i < n; ++i) t[i] = vk[i] / D[i]; /* right preconditioning */
            op_apply(C, t, vn);
            for (int j = 0; j <= k; ++j) {
                cplx *vj = V + (size_t)j * n;
                cplx hij = 0.0;
                for (int i = 0; i < n; ++i) hij += conj(vj[i]) * vn[i];
                H[j * mr + k] = hij;
                for (int i = 0; i < n; ++i) vn[i] -= hij * vj[i];
            }
            double hn = vnorm(n, vn);
            H[(k + 1) * mr + k] = hn;
            if (hn > 0.0)
                for (int i = 0; i < n; ++i) vn[i] /= hn;
            for (int j = 0; j < k; ++j) {
                cplx a = H[j * mr + k], bb = H[(j + 1) * mr + k];
                H[j * mr + k] = conj(cs[j]) * a + conj(sn[j]) * bb;
                H[(j + 1) * mr + k] = -sn[j] * a + cs[j] * bb;
            }
            cplx a = H[k * mr + k], bb = H[(k + 1) * mr + k];
            double den = sqrt(creal(a * conj(a)) + creal(bb * conj(bb)));
            cs[k] = a / den;
            sn[k] = bb / den;
            H[k * mr + k] = den;
            H[(k + 1) * mr + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = conj(cs[k]) * g[k];
            if (cabs(g[k + 1]) / bn <= tol) { ++k; ++it; break; }
        }
        for (int j = k - 1; j >= 0; --j) {
            cplx s = g[j];
            for (int l = j + 1; l < k; ++l) s -= H[j * mr + l] * yv[l];
            yv[j] = s / H[j * mr + j];
        }
        for (int i = 0; i < n; ++i) t[i] = 0.0;
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < n; ++i) t[i] += yv[j] * V[(size_t)j * n + i];
        for (int i = 0; i < n; ++i) w[i] += t[i] / D[i];
    }
    *iters = it;
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(t);
    return *relres <= tol ? 0 : 1;
}

/* solve T A T^T w = b; Adense NULL -> H2 operator.  Complex interleaved.     */
int or_solve(or_problem *P, const double *Adense, const double *bd, double *wd, double tol, int maxit, int restart,
             int32_t *iters, double *relres)
{
    op_ctx C = {P, (const cplx *)Adense};
    if (!Adense) or_h2_assemble(P, 0);
    cplx *D = (cplx *)malloc(sizeof(cplx) * P->ndof);
    or_jacobi_diag(P, Adense, (double *)D);
    int it = 0, rc;
    if (P->kernel == OR_LAPLACE)
        rc = solve_cg(&C, D, (const cplx *)bd, (cplx *)wd, tol, maxit, &it, relres);
    else
        rc = solve_gmres(&C, D, (const cplx *)bd, (cplx *)wd, tol, maxit, restart, &it, relres);
    *iters = it;
    free(D);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Potential by the representation formula (Sec. 3.1, eq. eq::repform):      */
/* u(x) = sum_E sum_q u*(x, F y_q) k(y_q) h^2 w_q mu_h(y_q), Gauss grhs.      */
/* ------------------------------------------------------------------------ */
void or_potential(const or_problem *P, const double *xsd, int64_t npts, const double *pts, double *ud)
{
    const cplx *xs = (const cplx *)xsd;
    cplx *u = (cplx *)ud;
    int g = P->grhs, p = P->p, pp = p + 1;
    double gx[64], gw[64];
    or_gauss(g, gx, gw);
    int64_t nq = (int64_t)P->nelem * g * g;
    double *Y = (double *)malloc(sizeof(double) * 3 * nq);
    cplx *c = (cplx *)malloc(sizeof(cplx) * nq);
    for (int E = 0; E < P->nelem; ++E)
        for (int j = 0; j < g; ++j)
            for (int i = 0; i < g; ++i) {
                int64_t k = (int64_t)E * g * g + j * g + i;
                int patch;
                double uu, vv, kap;
                elem_param(P, E, gx[i], gx[j], &patch, &uu, &vv);
                geom(P, patch, uu, vv, Y + 3 * k, &kap);
                cplx mu = 0.0;
                for (int r2 = 0; r2 < pp; ++r2)
                    for (int r1 = 0; r1 < pp; ++r1)
                        mu += xs[(size_t)E * P->nloc + r2 * pp + r1] * bernstein(p, r1, gx[i]) * bernstein(p, r2, gx[j]);
                c[k] = mu * kap * P->h * P->h * gw[i] * gw[j];
            }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < npts; ++x) {
        cplx s = 0.0;
        for (int64_t k = 0; k < nq; ++k) s += fundamental(P, pts + 3 * x, Y + 3 * k) * c[k];
        u[x] = s;
    }
    free(Y);
    free(c);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* All computed near-field element pairs (E <= F) with their classification:  */
/* rows (E, F, class, order), sorted by (E, F).  Returns the count; writes    */
/* when out != NULL.                                                           */
static int cmp_int4(const void *x, const void *y)
{
    const int32_t *a = (const int32_t *)x, *b = (const int32_t *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

int64_t or_near_pair_classes(or_problem *P, int32_t *out)
{
    build_near_csr(P);
    int64_t cnt = 0;
    for (int E = 0; E < P->nelem; ++E)
        for (int64_t k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k)
            if (P->nb_idx[k] >= E) ++cnt;
    if (!out) return cnt;
    int64_t t = 0;
    for (int E = 0; E < P->nelem; ++E)
        for (int64_t k = P->nb_ptr[E]; k < P->nb_ptr[E + 1]; ++k) {
            int F = P->nb_idx[k];
            if (F < E) continue;
            out[4 * t] = E;
            out[4 * t + 1] = F;
            t++;
        }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < cnt; ++i) {
        pair_info pi = classify(P, out[4 * i], out[4 * i + 1]);
        out[4 * i + 2] = pi.cls;
        out[4 * i + 3] = pi.order;
    }
    qsort(out, cnt, 4 * sizeof(int32_t), cmp_int4);
    return cnt;
}

/* Batch forms of or_pair_block_sym / or_coupling_block over a list, parallel */
/* over the list (used to time samples of a workload).  pairs: n x (E, F);    */
/* out: n blocks of nloc^2 complex values.                                    */
void or_pair_blocks(const or_problem *P, int64_t n, const int32_t *pairs, double *out)
{
    int nl = P->nloc;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) pair_block_sym(P, pairs[2 * i], pairs[2 * i + 1], (cplx *)out + i * nl * nl);
}

/* blocks: n x (level, tgt, src); out: n blocks of q^4 complex values */
void or_coupling_blocks(const or_problem *P, int64_t n, const int32_t *blocks, double *out)
{
    int64_t q4 = (int64_t)P->q * P->q * P->q * P->q;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i)
        or_coupling_block(P, blocks[3 * i], blocks[3 * i + 1], blocks[3 * i + 2], (cplx *)out + i * q4);
}
