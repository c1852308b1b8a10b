"""Pins of the oracle's element-pair quadrature (Sec. 3.2 integrals, Sec. 4 item 4 rules).

Flat unit squares with the kernel 1/(4 pi |x-y|) and p = 0 (one Bernstein function per element):
  * coincident: closed form 4 asinh(1) - (4/3)(sqrt 2 - 1)
  * common edge (coplanar / perpendicular) and common vertex (coplanar, diagonal): reduced by
    difference variables to low-dimensional integrals evaluated here with mpmath, independently
    of the oracle's Duffy rules.
A plausible mistake in a region map, a Jacobian or an orientation frame breaks one of these.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1708_09162_amd import workloads as W

FOURPI = 4 * math.pi
SQ = W.flat_patch((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0))


def _tri(s):
    """density of s = a + b for a, b uniform on [0,1]"""
    return s if s <= 1 else 2 - s


def _edge_coplanar():
    # |x - y|^2 = (x1-y1)^2 + (x2+y2)^2; z = x1 - y1 has density (1-|z|), s = x2+y2 density tri(s)
    mp.mp.dps = 20
    f = lambda z, s: 2 * (1 - z) * _tri(s) / mp.sqrt(z * z + s * s)
    return float(mp.quad(f, [0, 1], [0, 1, 2]))


def _vertex_diagonal():
    mp.mp.dps = 20
    f = lambda a, b: _tri(a) * _tri(b) / mp.sqrt(a * a + b * b)
    return float(mp.quad(f, [0, 1, 2], [0, 1, 2]))


def _edge_perpendicular():
    # |x - y|^2 = (x1-y1)^2 + x2^2 + y2^2; inner square integral in polar coordinates
    mp.mp.dps = 20

    def inner(z):
        # int_0^1 int_0^1 (z^2 + a^2 + b^2)^(-1/2) da db, split by the diagonal, polar coordinates
        g = lambda th: mp.sqrt(z * z + 1 / mp.cos(th) ** 2) - abs(z)
        return 2 * mp.quad(g, [0, mp.pi / 4])

    return float(mp.quad(lambda z: 2 * (1 - z) * inner(z), [0, 1]))


@pytest.fixture(scope="module")
def pins():
    return {
        "coincident": 4 * math.asinh(1.0) - 4.0 / 3.0 * (math.sqrt(2) - 1),
        "edge": _edge_coplanar(),
        "vertex": _vertex_diagonal(),
        "perp": _edge_perpendicular(),
    }


def test_pin_values_sane(pins):
    # the survey's independently computed values agree with these reductions
    assert abs(pins["coincident"] - 2.97320959824738) < 1e-13
    assert abs(pins["edge"] - 1.11212868985) < 1e-10
    assert abs(pins["vertex"] - 0.748952218549) < 1e-11
    assert abs(pins["perp"] - 1.34889024636) < 1e-10


def _one(patches, E, F, gs):
    P = oracle.Problem(patches, p=0, m=0, q=1, gauss_singular=gs)
    return P.pair_block(E, F, symmetric=False)[0, 0] * FOURPI, P.pair_class(E, F)


def test_coincident(pins):
    errs = [abs(_one([SQ], 0, 0, g)[0] - pins["coincident"]) for g in (4, 6, 8, 12)]
    assert errs[-1] < 2e-13 * pins["coincident"]
    assert all(errs[i + 1] < errs[i] for i in range(2))


@pytest.mark.parametrize("variant", ["plain", "reversed_u", "swapped_uv", "second_first"])
def test_common_edge_coplanar(pins, variant):
    if variant == "plain":
        nb = W.flat_patch((1, 0, 0), (2, 0, 0), (1, 1, 0), (2, 1, 0))
    elif variant == "reversed_u":
        nb = W.flat_patch((2, 0, 0), (1, 0, 0), (2, 1, 0), (1, 1, 0))
    elif variant == "swapped_uv":
        nb = W.flat_patch((1, 0, 0), (1, 1, 0), (2, 0, 0), (2, 1, 0))
    else:
        nb = W.flat_patch((2, 1, 0), (1, 1, 0), (2, 0, 0), (1, 0, 0))
    patches = [SQ, nb] if variant != "second_first" else [nb, SQ]
    val, cls = _one(patches, 0, 1, 12)
    assert cls[0] == 2
    assert abs(val - pins["edge"]) < 1e-12 * pins["edge"]


def test_common_vertex(pins):
    for nb in (W.flat_patch((1, 1, 0), (2, 1, 0), (1, 2, 0), (2, 2, 0)),
               W.flat_patch((2, 2, 0), (1, 2, 0), (2, 1, 0), (1, 1, 0))):
        val, cls = _one([SQ, nb], 0, 1, 12)
        assert cls[0] == 3
        assert abs(val - pins["vertex"]) < 1e-12 * pins["vertex"]


def test_common_edge_perpendicular(pins):
    nb = W.flat_patch((0, 0, 0), (1, 0, 0), (0, 0, 1), (1, 0, 1))
    val, cls = _one([SQ, nb], 0, 1, 12)
    assert cls[0] == 2
    assert abs(val - pins["perp"]) < 1e-12 * pins["perp"]


def test_regular_pair_brute_force():
    """A regular pair of flat squares against an independent tensor Gauss sum in numpy."""
    nb = W.flat_patch((0.5, 3.0, 0.3), (1.5, 3.0, 0.3), (0.5, 4.0, 0.3), (1.5, 4.0, 0.3))
    P = oracle.Problem([SQ, nb], p=2, m=0, q=1, gauss_regular=10)
    cls = P.pair_class(0, 1)
    assert cls[0] == 0 and cls[1] == 10
    blk = P.pair_block(0, 1)
    t, w = np.polynomial.legendre.leggauss(30)
    t, w = (t + 1) / 2, w / 2
    B = np.array([[math.comb(2, r) * s ** r * (1 - s) ** (2 - r) for r in range(3)] for s in t])
    X = np.stack(np.meshgrid(t, t, indexing="xy"), -1).reshape(-1, 2)  # (u fastest)
    WX = np.outer(w, w).reshape(-1)
    phi = np.einsum("jb,ic->jibc", B, B).reshape(-1, 9)  # index r2*3+r1 with j=v, i=u
    x3 = np.c_[X, np.zeros(len(X))]
    y3 = np.c_[X[:, 0] + 0.5, X[:, 1] + 3.0, np.full(len(X), 0.3)]
    K = 1 / (FOURPI * np.linalg.norm(x3[:, None, :] - y3[None, :, :], axis=2))
    ref = phi.T @ (WX[:, None] * K * WX[None, :]) @ phi
    assert np.abs(blk - ref).max() < 1e-9 * np.abs(ref).max()


def test_symmetric_convention_sphere():
    """Blocks of (E,F) and (F,E) are exact transposes; identical blocks are symmetric."""
    P = oracle.Problem(W.sphere_patches(), p=1, m=1, q=1)
    for E, F in [(0, 1), (3, 9), (2, 2), (5, 20)]:
        a = P.pair_block(E, F)
        b = P.pair_block(F, E)
        assert np.array_equal(a, b.T)


def test_cross_patch_frames_align():
    """For touching pairs across patches, the canonical frames map the shared edge/corner to the
    same physical points (the interface compatibility of Sec. 2.2)."""
    P = oracle.Problem(W.sphere_patches(), p=0, m=2, q=1)
    ne = 4
    corner = [(0, 0), (1, 0), (1, 1), (0, 1)]
    rng = np.random.default_rng(0)
    n_edge = n_vert = 0
    for E in range(P.nelem):
        for F in range(E + 1, P.nelem):
            if E // 16 == F // 16:
                continue
            c = P.pair_class(E, F)
            if c[0] not in (2, 3):
                continue
            oE, aE, oF, aF = c[2], c[3], c[5], c[6]

            def pt(el, o, a, s):
                pt_, r = divmod(el, ne * ne)
                e2, e1 = divmod(r, ne)
                u = (e1 + corner[o][0] + s * (corner[a][0] - corner[o][0])) / ne
                v = (e2 + corner[o][1] + s * (corner[a][1] - corner[o][1])) / ne
                return P.geometry(pt_, [[u, v]])[0, :3]

            ss = rng.random(3) if c[0] == 2 else [0.0]
            for s in ss:
                assert np.linalg.norm(pt(E, oE, aE, s) - pt(F, oF, aF, s)) < 1e-14
            n_edge += c[0] == 2
            n_vert += c[0] == 3
    # 12 cube edges x 4 shared element edges; along each cube edge the pairs offset by one element share a vertex
    assert n_edge == 48
    assert n_vert == 12 * 2 * (ne - 1)
