"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark may use this package.  The product path (the HIP library and its
binding) never imports it and shares no code with it.

Vectors are numpy arrays.  S* ("superspace", Sec. 4.3) vectors use the
element-major order a = E*(p+1)^2 + r2*(p+1) + r1 with
E = patch*4^m + e2*2^m + e1; S vectors use patch*(2^m+p)^2 + j2*(2^m+p) + j1.
Complex quantities are complex128; for Laplace the real part is returned.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LAPLACE, HELMHOLTZ = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_native = None  # path of a build for this host's CPU (use_native_build), used instead of _LIB


def use_native_build() -> str:
    """Compiles the oracle for the CPU of this host (-O3 -march=native) into a temporary directory and
    loads that build from now on (for timing).  The default build targets x86-64-v3 so that it runs on
    any host it is copied to.  Must be called before the oracle is first used in the process."""
    import tempfile

    global _native
    if _lib is not None:
        raise RuntimeError("the oracle is already loaded")
    out = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle.so")
    subprocess.run(["gcc", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-std=gnu11", _SRC, "-o", out, "-lm"], check=True)
    _native = out
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _native is None and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        build(force=True)
    lib = C.CDLL(_native or _LIB)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    lib.or_create.restype = P
    lib.or_create.argtypes = [C.c_int, ip, ip, dp, dp, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                              C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.or_destroy.argtypes = [P]
    lib.or_info.argtypes = [P, lp]
    lib.or_export_partition.argtypes = [P, ip, ip]
    lib.or_T1.argtypes = [P, dp]
    lib.or_chebyshev_nodes.argtypes = [P, dp]
    lib.or_geometry.argtypes = [P, C.c_int, C.c_int, dp, dp]
    lib.or_pair_class.argtypes = [P, C.c_int, C.c_int, ip]
    lib.or_pair_block_sym.argtypes = [P, C.c_int, C.c_int, dp]
    lib.or_pair_block.argtypes = [P, C.c_int, C.c_int, dp]
    lib.or_apply_T.argtypes = [P, C.c_int, dp, dp]
    lib.or_apply_Tt.argtypes = [P, C.c_int, dp, dp]
    lib.or_dense_assemble.argtypes = [P, dp]
    lib.or_rhs_points.argtypes = [P, dp]
    lib.or_rhs.argtypes = [P, dp, dp]
    lib.or_h2_assemble.argtypes = [P, C.c_int]
    lib.or_h2_matvec_super.argtypes = [P, dp, dp]
    lib.or_h2_matvec_rows.argtypes = [P, dp, C.c_int, ip, dp]
    lib.or_coupling_block.argtypes = [P, C.c_int, C.c_int, C.c_int, dp]
    lib.or_matvec.argtypes = [P, dp, dp, dp]
    lib.or_jacobi_diag.argtypes = [P, dp, dp]
    lib.or_solve.restype = C.c_int
    lib.or_solve.argtypes = [P, dp, dp, dp, C.c_double, C.c_int, C.c_int, ip, dp]
    lib.or_potential.argtypes = [P, dp, C.c_int64, dp, dp]
    lib.or_pair_blocks.argtypes = [P, C.c_int64, ip, dp]
    lib.or_coupling_blocks.argtypes = [P, C.c_int64, ip, dp]
    lib.or_near_pair_classes.restype = C.c_int64
    lib.or_near_pair_classes.argtypes = [P, ip]
    lib.or_gauss.restype = C.c_int
    lib.or_gauss.argtypes = [C.c_int, dp, dp]
    lib.or_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def gauss(n: int):
    """Gauss-Legendre nodes and weights on [0,1] (ascending)."""
    lib = _load()
    x = np.zeros(n)
    w = np.zeros(n)
    if lib.or_gauss(n, _d(x), _d(w)) != 0:
        raise ValueError("order out of range")
    return x, w


def num_threads() -> int:
    return int(_load().or_num_threads())


def _flatten_patches(patches):
    deg, ncp, knots, cpw = [], [], [], []
    for p in patches:
        cp = np.asarray(p["cpw"], dtype=np.float64)
        nv, nu = cp.shape[0], cp.shape[1]
        deg += [p["deg_u"], p["deg_v"]]
        ncp += [nu, nv]
        knots.append(np.asarray(p["knots_u"], dtype=np.float64))
        knots.append(np.asarray(p["knots_v"], dtype=np.float64))
        cpw.append(cp.reshape(-1))
    return (np.array(deg, dtype=np.int32), np.array(ncp, dtype=np.int32),
            np.ascontiguousarray(np.concatenate(knots)), np.ascontiguousarray(np.concatenate(cpw)))


class Problem:
    """One discretised single-layer problem (geometry + parameters)."""

    def __init__(self, patches, *, kernel=LAPLACE, wavenumber=0.0, p=1, m=2, q=8, eta=1.6, leaf_depth=-1,
                 gauss_regular=6, gauss_singular=-1, gauss_rhs=-1, threads=0, kappa_diam=0.0):
        lib = _load()
        self._keep = _flatten_patches(patches)
        deg, ncp, knots, cpw = self._keep
        self._h = lib.or_create(len(patches), _i(deg), _i(ncp), _d(knots), _d(cpw), int(kernel), float(wavenumber),
                                int(p), int(m), int(q), float(eta), float(kappa_diam), int(leaf_depth),
                                int(gauss_regular),
                                int(gauss_singular), int(gauss_rhs), int(threads))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.kernel = kernel
        self.p, self.m, self.q = p, m, q
        info = np.zeros(16, dtype=np.int64)
        lib.or_info(self._h, info.ctypes.data_as(C.POINTER(C.c_int64)))
        (self.ndof, self.nsup, self.nelem, self.nloc, self.L, self.nnear, self.nfar, self.nrhs,
         self.gs, self.grhs, self.ns1) = [int(v) for v in info[:11]]
        self._dense = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().or_destroy(h)
            self._h = None

    # ---- helpers -------------------------------------------------------
    def _out(self, z):
        return z.real.copy() if self.kernel == LAPLACE else z

    @staticmethod
    def _c(v):
        return np.ascontiguousarray(np.asarray(v, dtype=np.complex128))

    # ---- structure -----------------------------------------------------
    def partition(self):
        """(near, far): near (n,2) leaf-pair ids at level L; far (n,3) = (level, tgt, src)."""
        near = np.zeros((self.nnear, 2), dtype=np.int32)
        far = np.zeros((self.nfar, 3), dtype=np.int32)
        _load().or_export_partition(self._h, _i(near), _i(far))
        return near, far

    def T1(self):
        out = np.zeros((self.ns1, (1 << self.m) * (self.p + 1)))
        _load().or_T1(self._h, _d(out))
        return out

    def chebyshev_nodes(self):
        out = np.zeros(self.q)
        _load().or_chebyshev_nodes(self._h, _d(out))
        return out

    def geometry(self, patch: int, uv):
        uv = np.ascontiguousarray(np.asarray(uv, dtype=np.float64).reshape(-1, 2))
        out = np.zeros((uv.shape[0], 4))
        _load().or_geometry(self._h, int(patch), uv.shape[0], _d(uv), _d(out))
        return out

    def pair_class(self, E: int, F: int):
        out = np.zeros(8, dtype=np.int32)
        _load().or_pair_class(self._h, int(E), int(F), _i(out))
        return out

    def near_pair_classes(self):
        """(n, 4) int32 rows (E, F, class, order) of the near-field pairs E <= F, sorted."""
        lib = _load()
        n = int(lib.or_near_pair_classes(self._h, None))
        out = np.zeros((n, 4), dtype=np.int32)
        lib.or_near_pair_classes(self._h, _i(out))
        return out

    def pair_block(self, E: int, F: int, symmetric=True):
        out = np.zeros((self.nloc, self.nloc), dtype=np.complex128)
        fn = _load().or_pair_block_sym if symmetric else _load().or_pair_block
        fn(self._h, int(E), int(F), out.ctypes.data_as(C.POINTER(C.c_double)))
        return self._out(out)

    def pair_blocks(self, pairs):
        """Blocks of a list of element pairs (n, 2), symmetric convention, computed in parallel."""
        pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = np.zeros((len(pairs), self.nloc, self.nloc), dtype=np.complex128)
        _load().or_pair_blocks(self._h, len(pairs), _i(pairs), _d(out.view(np.float64)))
        return self._out(out)

    def coupling_blocks(self, blocks):
        """Coupling blocks of a list of far pairs (n, 3) = (level, tgt, src), computed in parallel."""
        blocks = np.ascontiguousarray(np.asarray(blocks, dtype=np.int32).reshape(-1, 3))
        q2 = self.q * self.q
        out = np.zeros((len(blocks), q2, q2), dtype=np.complex128)
        _load().or_coupling_blocks(self._h, len(blocks), _i(blocks), _d(out.view(np.float64)))
        return self._out(out)

    def coupling_block(self, level: int, tgt: int, src: int):
        q2 = self.q * self.q
        out = np.zeros((q2, q2), dtype=np.complex128)
        _load().or_coupling_block(self._h, int(level), int(tgt), int(src), out.ctypes.data_as(C.POINTER(C.c_double)))
        return self._out(out)

    # ---- operators -----------------------------------------------------
    def apply_T(self, xs):
        xs = self._c(xs)
        y = np.zeros(self.ndof, dtype=np.complex128)
        _load().or_apply_T(self._h, 2, _d(xs.view(np.float64)), _d(y.view(np.float64)))
        return self._out(y)

    def apply_Tt(self, w):
        w = self._c(w)
        xs = np.zeros(self.nsup, dtype=np.complex128)
        _load().or_apply_Tt(self._h, 2, _d(w.view(np.float64)), _d(xs.view(np.float64)))
        return self._out(xs)

    def dense_super(self):
        """Dense Galerkin matrix A* over S* (nsup x nsup), complex128 internally."""
        if self._dense is None:
            A = np.zeros((self.nsup, self.nsup), dtype=np.complex128)
            _load().or_dense_assemble(self._h, _d(A.view(np.float64)))
            self._dense = A
        return self._out(self._dense)

    def dense_system(self):
        """A = T A* T^T (ndof x ndof)."""
        self.dense_super()
        A = self._dense
        T = self.T_matrix()
        return self._out(T @ A @ T.T)

    def T_matrix(self):
        """Dense T (ndof x nsup): per patch the tensor product T1 (x) T1 (Sec. 4.3)."""
        T1r = self.T1().reshape(self.ns1, 1 << self.m, self.p + 1)
        ne, pp, ns1 = 1 << self.m, self.p + 1, self.ns1
        npatch = self.nelem // (ne * ne)
        T = np.zeros((self.ndof, self.nsup))
        for pt in range(npatch):
            for j2 in range(ns1):
                for j1 in range(ns1):
                    row = pt * ns1 * ns1 + j2 * ns1 + j1
                    for e2 in range(ne):
                        for e1 in range(ne):
                            col = (pt * ne * ne + e2 * ne + e1) * pp * pp
                            T[row, col:col + pp * pp] = np.outer(T1r[j2, e2], T1r[j1, e1]).reshape(-1)
        return T

    def rhs_points(self):
        out = np.zeros((self.nrhs, 3))
        _load().or_rhs_points(self._h, _d(out))
        return out

    def rhs_super(self, gvals):
        g = self._c(gvals)
        out = np.zeros(self.nsup, dtype=np.complex128)
        _load().or_rhs(self._h, _d(g.view(np.float64)), _d(out.view(np.float64)))
        return self._out(out)

    def rhs(self, gvals):
        """b = T g* (Sec. 4.3)."""
        return self.apply_T(self.rhs_super(gvals))

    def h2_assemble(self, store_coupling=False):
        _load().or_h2_assemble(self._h, int(bool(store_coupling)))

    def h2_matvec_super(self, xs):
        xs = self._c(xs)
        y = np.zeros(self.nsup, dtype=np.complex128)
        _load().or_h2_matvec_super(self._h, _d(xs.view(np.float64)), _d(y.view(np.float64)))
        return self._out(y)

    def h2_matvec_rows(self, xs, leaves):
        xs = self._c(xs)
        leaves = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32))
        per = 1 << (2 * (self.m - self.L))
        out = np.zeros(len(leaves) * per * self.nloc, dtype=np.complex128)
        _load().or_h2_matvec_rows(self._h, _d(xs.view(np.float64)), len(leaves), _i(leaves), _d(out.view(np.float64)))
        return self._out(out.reshape(len(leaves), per, self.nloc))

    def matvec(self, w, dense=False):
        w = self._c(w)
        y = np.zeros(self.ndof, dtype=np.complex128)
        A = None
        if dense:
            self.dense_super()
            A = self._dense
        _load().or_matvec(self._h, _d(A.view(np.float64)) if A is not None else None,
                          _d(w.view(np.float64)), _d(y.view(np.float64)))
        return self._out(y)

    def jacobi_diag(self, dense=False):
        D = np.zeros(self.ndof, dtype=np.complex128)
        A = None
        if dense:
            self.dense_super()
            A = self._dense
        _load().or_jacobi_diag(self._h, _d(A.view(np.float64)) if A is not None else None, _d(D.view(np.float64)))
        return self._out(D)

    def solve(self, b, dense=False, tol=1e-8, maxit=2000, restart=100, w0=None):
        """Jacobi-preconditioned CG (Laplace) / GMRES (Helmholtz); returns (w, iters, relres)."""
        b = self._c(b)
        w = self._c(w0) if w0 is not None else np.zeros(self.ndof, dtype=np.complex128)
        A = None
        if dense:
            self.dense_super()
            A = self._dense
        it = np.zeros(1, dtype=np.int32)
        rr = np.zeros(1)
        _load().or_solve(self._h, _d(A.view(np.float64)) if A is not None else None, _d(b.view(np.float64)),
                         _d(w.view(np.float64)), float(tol), int(maxit), int(restart), _i(it), _d(rr))
        return self._out(w), int(it[0]), float(rr[0])

    def potential(self, xs, points):
        xs = self._c(xs)
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
        u = np.zeros(pts.shape[0], dtype=np.complex128)
        _load().or_potential(self._h, _d(xs.view(np.float64)), pts.shape[0], _d(pts), _d(u.view(np.float64)))
        return self._out(u)


def timed(fn, *a, **k):
    t0 = time.perf_counter()
    r = fn(*a, **k)
    return r, time.perf_counter() - t0
