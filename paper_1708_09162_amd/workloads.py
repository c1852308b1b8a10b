"""Seeded synthetic inputs: NURBS multipatch geometries and Dirichlet data.

This module holds no arithmetic of the boundary element method itself.  It
only produces *inputs*: NURBS control nets (the geometry description of
Section 2.2, eq. def::geom), seeded point sets and manufactured boundary data
of the kind used in Sections 5.1 and 5.3.  Both the CPU oracle and the HIP
path consume these, so nothing here may depend on either of them.

Geometries
----------
* ``sphere_patches()``: the unit sphere as 6 NURBS patches in a cube topology
  (Section 5).  Each patch is an *exact* rational Bezier patch of bidegree
  (4,4), obtained as the inverse stereographic projection of a planar
  rational biquadratic patch bounded by four circular arcs (the stereographic
  images of the great circles through the cube edges).  The composition of a
  bidegree-(2,2) rational map with the quadratic map sigma is bidegree (4,4),
  which matches the degree-4 patches named in Section 5.
* ``torus_patches()``: the torus with R=2, r=0.5 as 16 rational biquadratic
  patches, each a 90 degree by 90 degree piece (Section 5).
* ``flat_patch()`` / ``cube_patches()``: bilinear patches for tests.

Every patch is a dict with keys ``deg_u, deg_v, knots_u, knots_v, cpw`` where
``cpw`` has shape ``(n_v, n_u, 4)`` holding ``x, y, z, w`` (w > 0, control
points not premultiplied by w; u runs fastest in memory).
"""
from __future__ import annotations

import math
from math import comb

import numpy as np

__all__ = [
    "sphere_patches",
    "torus_patches",
    "flat_patch",
    "cube_patches",
    "perturbed_sphere_patches",
    "random_directions",
    "config_small_sphere",
    "config_sphere_h2",
    "config_torus_helmholtz",
    "interior_ball_points",
    "point_charges",
    "fichera_patches",
    "fichera_interior_points",
    "perturbation_map",
    "perturbed_mapping_patches",
]


# ---------------------------------------------------------------------------
# helpers for building control nets (geometric modelling, not the BEM method)
# ---------------------------------------------------------------------------
def _bezier_product(f: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Bernstein coefficients of the product of two tensor Bernstein polynomials.

    ``f`` has shape (a+1, b+1), ``g`` (c+1, d+1); the result has shape
    (a+c+1, b+d+1).  Uses B_i^a B_j^c = C(a,i)C(c,j)/C(a+c,i+j) B_{i+j}^{a+c}.
    """
    a, b = f.shape[0] - 1, f.shape[1] - 1
    c, d = g.shape[0] - 1, g.shape[1] - 1
    out = np.zeros((a + c + 1, b + d + 1))
    for i in range(a + 1):
        for j in range(b + 1):
            for k in range(c + 1):
                for l in range(d + 1):
                    cu = comb(a, i) * comb(c, k) / comb(a + c, i + k)
                    cv = comb(b, j) * comb(d, l) / comb(b + d, j + l)
                    out[i + k, j + l] += f[i, j] * g[k, l] * cu * cv
    return out


def _bezier_knots(deg: int) -> np.ndarray:
    return np.array([0.0] * (deg + 1) + [1.0] * (deg + 1))


def _patch(deg_u, deg_v, knots_u, knots_v, cpw) -> dict:
    cpw = np.ascontiguousarray(cpw, dtype=np.float64)
    assert cpw.ndim == 3 and cpw.shape[2] == 4
    return {
        "deg_u": int(deg_u),
        "deg_v": int(deg_v),
        "knots_u": np.ascontiguousarray(knots_u, dtype=np.float64),
        "knots_v": np.ascontiguousarray(knots_v, dtype=np.float64),
        "cpw": cpw,
    }


def _rotate_patch(patch: dict, R: np.ndarray) -> dict:
    cpw = patch["cpw"].copy()
    cpw[..., :3] = cpw[..., :3] @ R.T
    return _patch(patch["deg_u"], patch["deg_v"], patch["knots_u"], patch["knots_v"], cpw)


# ---------------------------------------------------------------------------
# unit sphere, 6 exact rational patches of bidegree (4,4)
# ---------------------------------------------------------------------------
def _sphere_top_patch() -> dict:
    """Patch covering the cap {|x| <= z, |y| <= z} of the unit sphere."""
    s3 = math.sqrt(3.0)
    c = (s3 - 1.0) / 2.0            # corner of the curvilinear square (cube corner image)
    t = 2.0 * s3 - 3.0              # tangent intersection of the 30 degree arcs
    we = math.cos(math.pi / 12.0)   # conic weight of a 30 degree circular arc
    wc = we * we                    # centre weight
    # planar control net: index [i][j], i along u (first plane coordinate a),
    # j along v (second coordinate b)
    pos = np.zeros((3, 3, 2))
    wgt = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            ci, cj = i - 1, j - 1
            if ci != 0 and cj != 0:
                pos[i, j] = (ci * c, cj * c)
                wgt[i, j] = 1.0
            elif ci == 0 and cj == 0:
                pos[i, j] = (0.0, 0.0)
                wgt[i, j] = wc
            elif ci == 0:
                pos[i, j] = (0.0, cj * t)
                wgt[i, j] = we
            else:
                pos[i, j] = (ci * t, 0.0)
                wgt[i, j] = we
    A = pos[..., 0] * wgt            # homogeneous planar coordinates
    B = pos[..., 1] * wgt
    W = wgt
    AW = _bezier_product(A, W)
    BW = _bezier_product(B, W)
    WW = _bezier_product(W, W)
    AA = _bezier_product(A, A)
    BB = _bezier_product(B, B)
    X = 2.0 * AW
    Y = 2.0 * BW
    Z = WW - AA - BB
    H = WW + AA + BB
    if not np.all(H > 0):
        raise RuntimeError("sphere construction produced a non-positive weight")
    # cpw layout (n_v, n_u, 4): [j][i]
    cpw = np.zeros((5, 5, 4))
    for i in range(5):
        for j in range(5):
            h = H[i, j]
            cpw[j, i] = (X[i, j] / h, Y[i, j] / h, Z[i, j] / h, h)
    return _patch(4, 4, _bezier_knots(4), _bezier_knots(4), cpw)


_FACE_ROTATIONS = {
    "+z": np.eye(3),
    "-z": np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, -1.0]]),
    "+x": np.array([[0.0, 0, 1.0], [0, 1.0, 0], [-1.0, 0, 0]]),
    "-x": np.array([[0.0, 0, -1.0], [0, 1.0, 0], [1.0, 0, 0]]),
    "+y": np.array([[1.0, 0, 0], [0, 0, 1.0], [0, -1.0, 0]]),
    "-y": np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]]),
}


def sphere_patches(radius: float = 1.0) -> list[dict]:
    """Exact sphere of the given radius as 6 rational bidegree-(4,4) patches."""
    top = _sphere_top_patch()
    out = []
    for key in ("+z", "-z", "+x", "-x", "+y", "-y"):
        p = _rotate_patch(top, _FACE_ROTATIONS[key])
        p["cpw"][..., :3] *= radius
        out.append(p)
    return out


def perturbed_sphere_patches(amplitude: float, seed: int, max_degree: int = 6) -> list[dict]:
    """Sphere with control points moved radially, c -> c (1 + amplitude rho(c/|c|)).

    rho is a seeded random combination of real spherical-harmonic-like
    polynomials of degree <= max_degree (here: random homogeneous polynomials
    restricted to the sphere), normalised so max|rho| = 1 on a sample.  The
    result is still an exact NURBS description of a smooth closed surface.
    """
    rng = np.random.default_rng(seed)
    terms = []
    for deg in range(1, max_degree + 1):
        for _ in range(2 * deg + 1):
            e = rng.integers(0, deg + 1, size=2)
            a = min(int(e[0]), deg)
            b = min(int(e[1]), deg - a)
            terms.append((a, b, deg - a - b, rng.standard_normal()))

    def rho(v):
        v = v / np.linalg.norm(v, axis=-1, keepdims=True)
        s = 0.0
        for a, b, c, coef in terms:
            s = s + coef * v[..., 0] ** a * v[..., 1] ** b * v[..., 2] ** c
        return s

    sample = random_directions(4096, seed + 7919)
    scale = np.max(np.abs(rho(sample)))
    out = []
    for p in sphere_patches():
        cpw = p["cpw"].copy()
        pts = cpw[..., :3]
        fac = 1.0 + amplitude * rho(pts) / scale
        cpw[..., :3] = pts * fac[..., None]
        out.append(_patch(p["deg_u"], p["deg_v"], p["knots_u"], p["knots_v"], cpw))
    return out


# ---------------------------------------------------------------------------
# torus, 16 rational biquadratic patches
# ---------------------------------------------------------------------------
def _quarter_arc(a0: float):
    """Control points and weights of the unit-circle arc [a0, a0 + pi/2]."""
    c0, s0 = math.cos(a0), math.sin(a0)
    c2, s2 = math.cos(a0 + math.pi / 2), math.sin(a0 + math.pi / 2)
    pts = np.array([[c0, s0], [c0 + c2, s0 + s2], [c2, s2]])
    w = np.array([1.0, math.sqrt(0.5), 1.0])
    return pts, w


def torus_patches(R: float = 2.0, r: float = 0.5) -> list[dict]:
    """Torus around the z axis; u runs along the big circle, v around the tube."""
    out = []
    for i in range(4):            # toroidal quarter
        Q, wq = _quarter_arc(i * math.pi / 2)
        for j in range(4):        # poloidal quarter
            C, wcirc = _quarter_arc(j * math.pi / 2)
            cpw = np.zeros((3, 3, 4))
            for b in range(3):    # v index (tube)
                rho = R + r * C[b, 0]
                z = r * C[b, 1]
                for a in range(3):  # u index
                    cpw[b, a] = (rho * Q[a, 0], rho * Q[a, 1], z, wq[a] * wcirc[b])
            out.append(_patch(2, 2, _bezier_knots(2), _bezier_knots(2), cpw))
    return out


# ---------------------------------------------------------------------------
# flat test patches
# ---------------------------------------------------------------------------
def flat_patch(p00, p10, p01, p11) -> dict:
    """Bilinear patch with corners F(0,0)=p00, F(1,0)=p10, F(0,1)=p01, F(1,1)=p11."""
    cpw = np.zeros((2, 2, 4))
    cpw[0, 0, :3], cpw[0, 1, :3] = p00, p10
    cpw[1, 0, :3], cpw[1, 1, :3] = p01, p11
    cpw[..., 3] = 1.0
    return _patch(1, 1, _bezier_knots(1), _bezier_knots(1), cpw)


def cube_patches(edge: float = 2.0) -> list[dict]:
    """Surface of the cube [-edge/2, edge/2]^3 as 6 bilinear patches (outward normals)."""
    h = edge / 2.0
    out = []
    for key in ("+z", "-z", "+x", "-x", "+y", "-y"):
        R = _FACE_ROTATIONS[key]
        corners = [np.array(c) for c in ((-h, -h, h), (h, -h, h), (-h, h, h), (h, h, h))]
        out.append(flat_patch(*[R @ c for c in corners]))
    return out


def fichera_patches() -> list[dict]:
    """The Fichera cube of Section 5: the cube [-1,1]^3 (edge length 2) with the corner octant (0,1]^3
    removed, as 24 bilinear unit squares (outward normals): the four quarters of each cube face, less the
    three that bound the removed octant, plus the three walls of the indentation (planes x, y, z = 0)."""
    squares = []
    for axis in range(3):
        for side in (-1.0, 1.0):
            for a0 in (-1.0, 0.0):
                for b0 in (-1.0, 0.0):
                    if side == 1.0 and a0 == 0.0 and b0 == 0.0:
                        continue  # this quarter bounds the removed octant
                    squares.append((axis, side, a0, b0, side))
    for axis in range(3):
        squares.append((axis, 0.0, 0.0, 0.0, 1.0))  # indentation wall, outward normal +e_axis
    out = []
    for axis, c, a0, b0, sgn in squares:
        i, j = (axis + 1) % 3, (axis + 2) % 3  # e_i x e_j = e_axis

        def pt(u, v, axis=axis, c=c, a0=a0, b0=b0, i=i, j=j):
            p = np.zeros(3)
            p[axis], p[i], p[j] = c, a0 + u, b0 + v
            return p

        if sgn > 0:
            out.append(flat_patch(pt(0, 0), pt(1, 0), pt(0, 1), pt(1, 1)))
        else:  # parameters exchanged: the normal flips to -e_axis
            out.append(flat_patch(pt(0, 0), pt(0, 1), pt(1, 0), pt(1, 1)))
    return out


def fichera_interior_points(n: int, seed: int, margin: float = 0.15) -> np.ndarray:
    """n seeded points inside the Fichera cube at least `margin` from its surface (Section 5.1 keeps
    evaluation points 0.15 away from the boundary)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(-1.0 + margin, 1.0 - margin, 3)
        if np.all(p > -margin):  # inside, or too close to, the removed octant
            continue
        pts.append(p)
    return np.array(pts)


def perturbation_map(x):
    """Piecewise linear, monotone map of [0,1] onto itself with kinks at 1/4 and 3/4 (slopes 1/2, 3/2,
    1/2): continuous with a discontinuous derivative, so it lies in H^1 but not in H^2, like the map of
    Section 5.2 (whose kinks at 0.3 and 0.7 are moved to the dyadic points 1/4 and 3/4 here, element
    boundaries of every mesh with m >= 2)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= 0.25, 0.5 * x, np.where(x < 0.75, 1.5 * x - 0.25, 0.5 * (x + 1.0)))


def _subdivide_bezier_1d(P: np.ndarray, t: float):
    """de Casteljau split of a Bezier curve (control points along axis 0, homogeneous) at t."""
    P = P.copy()
    n = P.shape[0] - 1
    left, right = [P[0].copy()], [P[n].copy()]
    for r in range(1, n + 1):
        P = (1 - t) * P[:-1] + t * P[1:]
        left.append(P[0].copy())
        right.append(P[-1].copy())
    return np.array(left), np.array(right[::-1])


def _reparametrise_bezier_1d(P: np.ndarray, a: float, b: float) -> np.ndarray:
    """Control points of the Bezier curve restricted to [a, b] (homogeneous points along axis 0)."""
    _, R = _subdivide_bezier_1d(P, a)
    if a < 1.0:
        L, _ = _subdivide_bezier_1d(R, (b - a) / (1.0 - a))
    else:
        L = R
    return L


def perturbed_mapping_patches(patches: list[dict]) -> list[dict]:
    """Each single-piece rational Bezier patch F composed with the perturbation map in both parameters,
    F(f(u), f(v)) (Section 5.2): the same surface, parametrised with kinks at u, v = 1/4 and 3/4.  The
    result is a NURBS patch of the same degrees with knots of full multiplicity at 1/4 and 3/4 (one
    Bezier piece per linear piece of f, obtained by de Casteljau subdivision)."""
    breaks = [0.0, 0.25, 0.75, 1.0]
    out = []
    for p in patches:
        du, dv = p["deg_u"], p["deg_v"]
        cpw = np.asarray(p["cpw"], dtype=np.float64)
        if cpw.shape[1] != du + 1 or cpw.shape[0] != dv + 1:
            raise ValueError("perturbed_mapping_patches expects single Bezier patches")
        H = cpw.copy()
        H[..., :3] *= H[..., 3:4]  # homogeneous (x w, y w, z w, w)

        def pieces_1d(Q, deg):
            segs = []
            for k in range(3):
                a, b = perturbation_map(breaks[k]), perturbation_map(breaks[k + 1])
                seg = _reparametrise_bezier_1d(Q, float(a), float(b))
                segs.append(seg if k == 0 else seg[1:])
            return np.concatenate(segs, axis=0)

        # along u (axis 1), then along v (axis 0)
        Hu = np.stack([pieces_1d(H[j], du) for j in range(H.shape[0])], axis=0)
        Hv = np.stack([pieces_1d(Hu[:, i], dv) for i in range(Hu.shape[1])], axis=1)
        C = Hv.copy()
        C[..., :3] /= C[..., 3:4]
        ku = np.array([0.0] * (du + 1) + [0.25] * du + [0.75] * du + [1.0] * (du + 1))
        kv = np.array([0.0] * (dv + 1) + [0.25] * dv + [0.75] * dv + [1.0] * (dv + 1))
        out.append(_patch(du, dv, ku, kv, C))
    return out


# ---------------------------------------------------------------------------
# seeded point sets and data
# ---------------------------------------------------------------------------
def random_directions(n: int, seed: int) -> np.ndarray:
    """n unit vectors: normalised standard normals from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def interior_ball_points(n: int, seed: int, radius: float = 0.85) -> np.ndarray:
    """n points uniform in the ball of the given radius (seeded)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = radius * rng.random(n) ** (1.0 / 3.0)
    return d * rad[:, None]


def point_charges(n: int, seed: int, rmin: float = 1.5, rmax: float = 3.0):
    """n exterior charges: positions at radius U[rmin,rmax] and strengths U[-1,1]."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = rng.uniform(rmin, rmax, n)
    q = rng.uniform(-1.0, 1.0, n)
    return d * rad[:, None], q


def laplace_charge_field(points: np.ndarray, pos: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Harmonic field sum_i q_i / (4 pi |x - x_i|) at the given points (data, not the method)."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    for x0, c in zip(pos, q):
        out += c / (4.0 * math.pi * np.linalg.norm(pts - x0, axis=1))
    return out


def helmholtz_point_source(points: np.ndarray, v, kappa: float) -> np.ndarray:
    """exp(i kappa |x - v|) / |x - v| at the given points (Section 5.3 data family)."""
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    d = np.linalg.norm(pts - np.asarray(v, dtype=np.float64), axis=1)
    return np.exp(1j * kappa * d) / d


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------
def config_small_sphere() -> dict:
    """Laplace interior Dirichlet on the 6-patch unit sphere, p=1, 4x4 elements per patch,
    Gauss order 6, dense (every element pair in the near field); data = 1/|x - x0|
    with x0 seeded at radius 2; 100 seeded interior evaluation points."""
    x0 = 2.0 * random_directions(1, 1)[0]
    return {
        "name": "laplace_sphere_p1_m2_dense",
        "patches": sphere_patches(),
        "kernel": 0, "wavenumber": 0.0,
        "p": 1, "m": 2, "q": 8, "eta": 1.6, "gauss_regular": 6,
        "dense": True,
        "source": x0,
        "eval_points": interior_ball_points(100, 1),
    }


def config_sphere_h2() -> dict:
    """Laplace on the 6-patch unit sphere, p=3, 32x32 elements per patch (m=5), H2 with
    q=8 Chebyshev nodes per parametric direction, eta=1.6, Gauss order 6; data from 4
    seeded exterior point charges."""
    pos, q = point_charges(4, 2)
    return {
        "name": "laplace_sphere_p3_m5_q8",
        "patches": sphere_patches(),
        "kernel": 0, "wavenumber": 0.0,
        "p": 3, "m": 5, "q": 8, "eta": 1.6, "gauss_regular": 6,
        "dense": False,
        "charges": (pos, q),
        "eval_points": interior_ball_points(100, 2),
    }


def config_torus_helmholtz() -> dict:
    """Helmholtz exterior on the 16-patch torus (R=2, r=0.5), p=2, 64x64 elements per
    patch (m=6), kappa=8, q=10; plane wave with seeded unit direction; potential on a
    64x64 grid of the plane z=1, x,y in [-4,4]."""
    d = random_directions(1, 3)[0]
    xs = np.linspace(-4.0, 4.0, 64)
    gx, gy = np.meshgrid(xs, xs, indexing="xy")
    grid = np.stack([gx.ravel(), gy.ravel(), np.ones(gx.size)], axis=1)
    return {
        "name": "helmholtz_torus_p2_m6_q10_k8",
        "patches": torus_patches(),
        "kernel": 1, "wavenumber": 8.0,
        "p": 2, "m": 6, "q": 10, "eta": 1.6, "gauss_regular": 6,
        "dense": False,
        "direction": d,
        "eval_points": grid,
    }


def config_learned_preconditioner() -> dict:
    """Laplace on the radially perturbed sphere (amplitude 0.1, spherical-harmonic degree <= 6,
    seed 5), p=2, 128x128 elements per patch (m=7), q=8; 2000 training vectors x ~ N(0, 1)
    (seed 5); right-hand side from 4 exterior point charges (seed 2)."""
    return {
        "name": "laplace_perturbed_sphere_p2_m7_q8",
        "patches": perturbed_sphere_patches(0.1, 5),
        "p": 2, "m": 7, "q": 8, "eta": 1.6, "gauss_regular": 6,
        "n_pairs": 2000, "pair_seed": 5, "charges": (4, 2),
    }


CNN_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 1)]


def cnn_initial_weights(seed: int, last_scale: float = 0.0) -> np.ndarray:
    """Seeded initial weights of the preconditioner network, layer after layer, each
    [c_out][c_in][3][3] (FP32): normal with standard deviation sqrt(2 / (9 c_in)) for the
    first four layers, last layer normal * last_scale (zero by default)."""
    rng = np.random.default_rng(seed)
    out = []
    for l, (ci, co) in enumerate(CNN_LAYERS):
        std = np.sqrt(2.0 / (9 * ci)) if l < len(CNN_LAYERS) - 1 else last_scale
        out.append(rng.standard_normal(9 * ci * co) * std)
    return np.concatenate(out).astype(np.float32)


def training_vectors(n_pairs: int, n: int, seed: int) -> np.ndarray:
    """n_pairs seeded standard normal coefficient vectors of length n (FP64)."""
    return np.random.default_rng(seed).standard_normal((n_pairs, n))


def _near_sphere_resonance(kappa: float, lmax: int = 19, gap: float = 0.05) -> bool:
    """True when kappa lies within `gap` of a zero of a spherical Bessel function j_l, l <= lmax (the interior
    Dirichlet eigenvalues of the unit sphere, where the single-layer operator is singular)."""
    from scipy.special import spherical_jn

    xs = np.linspace(max(kappa - gap, 1e-6), kappa + gap, 41)
    for l in range(lmax + 1):
        v = spherical_jn(l, xs)
        if np.any(np.sign(v[1:]) != np.sign(v[:-1])) or np.any(v == 0.0):
            return True
    return False


def config_batched(n: int = 128, seed: int = 4) -> list[dict]:
    """n independent problems (seed + i each): unit sphere or 16-patch torus, 2^m x 2^m elements per patch
    with m in {2,3,4,5}, degree p in {1,2,3}, q = 6; Laplace (data from 4 exterior point charges) or
    Helmholtz with kappa uniform in [1, 16] (data from a point source inside: sphere radius <= 0.5, torus
    tube centre line; kappa redrawn near sphere resonances); 1 to 8 right-hand sides each (n_rhs; the
    first from the fields above, the others in more_rhs)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed + i)
        torus = bool(rng.integers(0, 2))
        m = int(rng.integers(2, 6))
        p = int(rng.integers(1, 4))
        helm = bool(rng.integers(0, 2))
        d = {"geometry": "torus" if torus else "sphere", "m": m, "p": p, "q": 6, "eta": 1.6, "gauss_regular": 6,
             "kernel": 1 if helm else 0, "wavenumber": 0.0, "seed": seed + i}
        if helm:
            k = float(rng.uniform(1.0, 16.0))
            while not torus and _near_sphere_resonance(k):
                k = float(rng.uniform(1.0, 16.0))
            d["wavenumber"] = k
            if torus:
                a = float(rng.uniform(0.0, 2.0 * np.pi))
                d["source"] = np.array([2.0 * np.cos(a), 2.0 * np.sin(a), 0.0])
            else:
                v = rng.standard_normal(3)
                d["source"] = v / np.linalg.norm(v) * float(rng.uniform(0.0, 0.5))
        else:
            d["charges"] = point_charges(4, seed + i, rmin=3.5 if torus else 1.5, rmax=5.0 if torus else 3.0)
        # further right-hand sides of the same problem (1..8 in all): other charges or sources
        d["n_rhs"] = int(rng.integers(1, 9))
        d["more_rhs"] = []
        for r in range(1, d["n_rhs"]):
            rr = np.random.default_rng((seed + i, r))
            if helm and torus:
                a = float(rr.uniform(0.0, 2.0 * np.pi))
                d["more_rhs"].append({"source": np.array([2.0 * np.cos(a), 2.0 * np.sin(a), 0.0])})
            elif helm:
                v = rr.standard_normal(3)
                d["more_rhs"].append({"source": v / np.linalg.norm(v) * float(rr.uniform(0.0, 0.5))})
            else:
                d["more_rhs"].append({"charges": point_charges(4, 100000 * (seed + i) + r, rmin=3.5 if torus else 1.5,
                                                               rmax=5.0 if torus else 3.0)})
        out.append(d)
    return out
