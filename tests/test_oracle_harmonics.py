"""Spherical-harmonic pins of the oracle's dense Galerkin operator on the exact 6-patch unit sphere.

On the unit sphere the single-layer operator is diagonal in the spherical harmonics (Sec. 3.1,
eqs. fundament1 and fundament2): V Y_l^m = Y_l^m / (2l+1) for Laplace and V Y_l^m = lambda_l Y_l^m with
lambda_l = i k j_l(k) h_l^(1)(k) for Helmholtz (bilinear pairing, real basis).  These facts do not come
from the oracle, so they pin it:

* the Galerkin value b^T A^-1 b with b_i = <Y, b_i> approximates <V^-1 Y, Y> = 1/lambda_l (Y orthonormal);
* the Galerkin Rayleigh quotient of the L2 projection of Y tends to 1/(2l+1) (Laplace);
* the Galerkin density for data Y tends to Y / lambda_l in L2(Gamma) at rate h^(p+1) (Lemma
  cor::Approxcor, reading of the L2 rate as p+1).

The spherical harmonics come from scipy.special, the B-spline basis of S for the density and the mass
matrix from scipy.interpolate.BSpline (not the oracle's Cox-de Boor), and only the surface points and
measures F(x), kappa(x) are taken from the oracle's geometry (pinned separately: |F| = 1, area 4 pi).
A plausible mistake in the oracle's quadrature, kernel sign, T or right-hand side moves one of these.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.special import sph_harm_y, spherical_jn, spherical_yn

import oracle
from paper_1708_09162_amd import workloads as W

SPH = W.sphere_patches()
HARMONICS = [(1, 0), (2, 1), (3, -2)]  # (l, m): zonal and two tesseral ones off the patch axes


def real_sph_harm(l, m, X):
    """Real orthonormal spherical harmonic Y_l^m at the directions of the points X (n, 3)."""
    X = np.asarray(X, dtype=np.float64)
    r = np.linalg.norm(X, axis=1)
    theta = np.arccos(np.clip(X[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(X[:, 1], X[:, 0])
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    Y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (-1) ** m * (Y.real if m > 0 else Y.imag)


def eigenvalue(kind, l, k):
    if kind == "laplace":
        return 1.0 / (2 * l + 1)
    j, y = spherical_jn(l, k), spherical_yn(l, k)
    return 1j * k * j * (j + 1j * y)


_cache = {}


def system(kind, k, p, m):
    """(oracle problem, dense system matrix A = T A* T^T) on the sphere, Gauss order 8."""
    key = (kind, k, p, m)
    if key not in _cache:
        kw = dict(p=p, m=m, q=2, gauss_regular=8)
        if kind == "helmholtz":
            kw.update(kernel=oracle.HELMHOLTZ, wavenumber=k)
        P = oracle.Problem(SPH, **kw)
        _cache[key] = (P, P.dense_system())
    return _cache[key]


def surface_quadrature(p, m, ng=8):
    """Per patch: parameter points (u fastest), tensor Gauss weights and the tensor B-spline design matrix
    of S (columns j2*(2^m+p) + j1, the library's dof order)."""
    ne = 1 << m
    xg, wg = np.polynomial.legendre.leggauss(ng)
    xg, wg = (xg + 1) / 2, wg / 2
    t = np.concatenate([(e + xg) / ne for e in range(ne)])
    wt = np.concatenate([wg / ne] * ne)
    knots = np.concatenate([np.zeros(p + 1), np.arange(1, ne) / ne, np.ones(p + 1)])
    B = BSpline.design_matrix(t, knots, p).toarray()
    uu, vv = np.meshgrid(t, t, indexing="xy")
    uv = np.stack([uu.ravel(), vv.ravel()], axis=1)
    BB = np.einsum("vj,ui->vuji", B, B).reshape(len(t) ** 2, -1)
    return uv, np.outer(wt, wt).ravel(), BB


def density_l2_error(P, w, p, m, exact_fn):
    """||mu_h - exact||_L2(Gamma) / ||exact||, mu_h = sum_i w_i b_i."""
    uv, ww, BB = surface_quadrature(p, m)
    ns = BB.shape[1]
    e2 = n2 = 0.0
    for pt in range(6):
        g = P.geometry(pt, uv)
        mu = BB @ w[pt * ns:(pt + 1) * ns]
        ex = exact_fn(g[:, :3])
        e2 += np.sum(ww * g[:, 3] * np.abs(mu - ex) ** 2)
        n2 += np.sum(ww * g[:, 3] * np.abs(ex) ** 2)
    return math.sqrt(e2 / n2)


def mass_matrix(P, p, m):
    uv, ww, BB = surface_quadrature(p, m)
    ns = BB.shape[1]
    M = np.zeros((P.ndof, P.ndof))
    for pt in range(6):
        g = P.geometry(pt, uv)
        M[pt * ns:(pt + 1) * ns, pt * ns:(pt + 1) * ns] = BB.T @ (BB * (ww * g[:, 3])[:, None])
    return M


@pytest.mark.parametrize("p", [1, 2])
def test_laplace_inverse_eigenvalues(p):
    """b^T A^-1 b -> <V^-1 Y, Y> = 2l+1 for l = 1, 2, 3.  For l = 1 the error falls faster than h^(p+3): the
    energy-norm rate is h^(2p+3), reached only asymptotically on these coarse meshes."""
    for l, mq in HARMONICS:
        errs = []
        for m in (1, 2):
            P, A = system("laplace", 0.0, p, m)
            b = P.rhs(real_sph_harm(l, mq, P.rhs_points()))
            s = b @ np.linalg.solve(A, b)
            errs.append(abs(s / (2 * l + 1) - 1.0))
        assert errs[1] < errs[0] / 4 and errs[1] < 5e-4, (p, l, errs)
        if l == 1:
            assert math.log2(errs[0] / errs[1]) > p + 3, (p, errs)


@pytest.mark.parametrize("p", [1, 2])
def test_laplace_rayleigh_quotient_of_projection(p):
    """<V Pi Y, Pi Y> / <Pi Y, Pi Y> -> 1/(2l+1), Pi the L2 projection onto S (mass matrix from scipy's
    B-splines); <Pi Y, Pi Y> -> 1."""
    for l, mq in HARMONICS:
        errs = []
        for m in (1, 2):
            P, A = system("laplace", 0.0, p, m)
            b = P.rhs(real_sph_harm(l, mq, P.rhs_points()))
            c = np.linalg.solve(mass_matrix(P, p, m), b)
            errs.append(abs((c @ A @ c) / (c @ b) * (2 * l + 1) - 1.0))
            assert abs(c @ b - 1.0) < 0.06
        assert errs[1] < errs[0] / 4 and errs[1] < 2e-3, (p, l, errs)


@pytest.mark.parametrize("p", [1, 2])
def test_laplace_density_converges_to_scaled_harmonic(p):
    """Data Y_l^m: the density tends to (2l+1) Y_l^m in L2(Gamma), for l = 1 at rate h^(p+1) (higher l are
    still pre-asymptotic on 2x2 and 4x4 elements per patch and are only required to improve)."""
    for l, mq in HARMONICS:
        errs = []
        for m in (1, 2):
            P, A = system("laplace", 0.0, p, m)
            w = np.linalg.solve(A, P.rhs(real_sph_harm(l, mq, P.rhs_points())))
            errs.append(density_l2_error(P, w, p, m, lambda X: (2 * l + 1) * real_sph_harm(l, mq, X)))
        rate = math.log2(errs[0] / errs[1])
        assert (rate > p + 1 - 0.35) if l == 1 else (rate > 1.0), (p, l, errs, rate)
        assert errs[1] < 0.05


@pytest.mark.parametrize("k", [1.0, 2.0])
def test_helmholtz_inverse_eigenvalues(k):
    """b^T A^-1 b -> 1/lambda_l with lambda_l = i k j_l(k) h_l^(1)(k), l = 1, 2 (p = 1); the density tends to
    Y / lambda_l at rate h^2."""
    p = 1
    for l, mq in HARMONICS[:2]:
        lam = eigenvalue("helmholtz", l, k)
        errs, derr = [], []
        for m in (1, 2):
            P, A = system("helmholtz", k, p, m)
            b = P.rhs(real_sph_harm(l, mq, P.rhs_points()))
            w = np.linalg.solve(A, b)
            errs.append(abs((b @ w) * lam - 1.0))  # bilinear form: no conjugation
            derr.append(density_l2_error(P, w, p, m, lambda X: real_sph_harm(l, mq, X) / lam))
        assert errs[1] < errs[0] / 8 and errs[1] < 2e-4, (k, l, errs)
        assert math.log2(derr[0] / derr[1]) > p + 1 - 0.35 - (l > 1) * 0.6, (k, l, derr)
        # a conjugated kernel (outgoing/incoming mix-up) would converge to the conjugate eigenvalue instead
        assert abs((b @ w) * np.conj(lam) - 1.0) > 100 * errs[1]
