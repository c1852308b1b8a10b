"""Oracle pins on the paper's other geometries (Sec. 5): the Fichera cube (24 bilinear patches, an edge-2
cube with an indented corner) and the sphere with perturbed mappings (Sec. 5.2: every patch reparametrised
by a piecewise linear map with kinks, here at the dyadic points 1/4 and 3/4).

Facts that do not come from the oracle: the Fichera surface has area 24 and lies on the planes of its
faces; the perturbed sphere is the same point set (|F| = 1, area 4 pi, F(f(u), f(v)) reproduced) and the
single layer still maps the constant 1 to 1 on it; manufactured interior potentials (point charges outside
the domain, one of them inside the indentation) are harmonic, so the discrete potential must approach them.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1708_09162_amd import workloads as W


def _surface_samples(P, npatch, g=8, nsub=2):
    x, w = np.polynomial.legendre.leggauss(g)
    x, w = (x + 1) / 2, w / 2
    uv = np.array([[a, b] for b in x for a in x])
    ww = np.outer(w, w).reshape(-1)
    pts, area = [], 0.0
    for pt in range(npatch):
        for e2 in range(nsub):
            for e1 in range(nsub):
                G = P.geometry(pt, (uv + [e1, e2]) / nsub)
                pts.append(G[:, :3])
                area += np.sum(G[:, 3] * ww) / nsub ** 2
    return np.concatenate(pts), area


def test_fichera_geometry():
    F = W.fichera_patches()
    assert len(F) == 24
    P = oracle.Problem(F, p=0, m=0, q=1)
    pts, area = _surface_samples(P, 24)
    assert abs(area - 24.0) < 1e-12
    on_face = np.isclose(np.abs(pts), 1.0, atol=1e-14).any(axis=1)
    on_wall = (np.isclose(pts, 0.0, atol=1e-14) & (pts >= -1e-14).all(axis=1, keepdims=True)).any(axis=1)
    assert np.all(on_face | on_wall)
    assert not np.any((pts > 1e-12).all(axis=1) & ~on_wall)  # nothing inside the removed octant
    assert np.abs(pts).max() <= 1.0 + 1e-14


def test_fichera_dense_interior_problem():
    """Interior Laplace on the Fichera cube (p=0, 2x2 elements per patch, dense): symmetric positive
    definite Galerkin matrix; the potential of two exterior charges (one inside the indentation) is
    reproduced at interior points 0.15 away from the surface to the accuracy of this coarse mesh."""
    F = W.fichera_patches()
    P = oracle.Problem(F, p=0, m=1, q=2, gauss_regular=8, gauss_rhs=14)
    A = P.dense_system()
    assert np.array_equal(P.dense_super(), P.dense_super().T)
    np.linalg.cholesky(A)
    pos, q = np.array([[0.5, 0.5, 0.5], [2.0, -2.5, 1.5]]), np.array([1.0, -0.7])
    b = P.rhs(W.laplace_charge_field(P.rhs_points(), pos, q))
    w = np.linalg.solve(A, b)
    ev = W.fichera_interior_points(40, 2)
    err = np.abs(P.potential(P.apply_Tt(w), ev) - W.laplace_charge_field(ev, pos, q)).max()
    assert err < 5e-3


def test_perturbed_mapping_is_a_reparametrisation():
    S = W.sphere_patches()
    Pt = W.perturbed_mapping_patches(S)
    P0 = oracle.Problem(S, p=0, m=2, q=2)
    P1 = oracle.Problem(Pt, p=0, m=2, q=2)
    pts, area = _surface_samples(P1, 6, nsub=4)
    assert np.abs(np.linalg.norm(pts, axis=1) - 1.0).max() < 1e-15 * 8
    assert abs(area - 4 * math.pi) < 1e-12
    u = np.random.default_rng(3).random((64, 2))
    for pt in range(6):
        fu = np.stack([W.perturbation_map(u[:, 0]), W.perturbation_map(u[:, 1])], axis=1)
        assert np.abs(P1.geometry(pt, u)[:, :3] - P0.geometry(pt, fu)[:, :3]).max() < 1e-14
    # the kinks: one-sided derivatives of f differ at 1/4 and 3/4, f is continuous there
    for k in (0.25, 0.75):
        e = 1e-7
        left = (W.perturbation_map(k) - W.perturbation_map(k - e)) / e
        right = (W.perturbation_map(k + e) - W.perturbation_map(k)) / e
        assert abs(left - right) > 0.9


def test_perturbed_sphere_constant_density():
    """<V 1, 1> = 4 pi on the perturbed sphere as on the smooth one (the operator does not depend on the
    parametrisation; the partition of unity of S keeps the constant exactly)."""
    P = oracle.Problem(W.perturbed_mapping_patches(W.sphere_patches()), p=1, m=2, q=2, gauss_regular=8)
    one = np.ones(P.ndof)
    assert abs(one @ P.dense_system() @ one - 4 * math.pi) < 1e-8
