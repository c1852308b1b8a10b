"""Thin ctypes binding of libigabem (declared in include/igabem.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device vectors are torch tensors on the GPU (float64, or complex128
for Helmholtz); the operator runs on the torch stream that is current when it
is created.  There is no CPU fallback: if the shared library is missing or
cannot be loaded, importing this module raises.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigabem.so")

IGB_OK = 0
IGB_ENOT_CONVERGED = 1
IGB_EINVAL = -1
IGB_EHIP = -2
IGB_ENOMEM = -3
IGB_EUNSUPPORTED = -4
IGB_LAPLACE = 0
IGB_HELMHOLTZ = 1
IGB_DENSE = 0
IGB_H2_STORED = 1
IGB_H2_ONTHEFLY = 2
IGB_FP64 = 0
IGB_FP32 = 1

EXPORTED = [
    "igb_last_error", "igb_geometry_create", "igb_geometry_destroy", "igb_operator_create",
    "igb_operator_destroy", "igb_operator_info", "igb_rhs_points", "igb_rhs_assemble", "igb_matvec",
    "igb_matvec_super", "igb_apply_Tt", "igb_apply_T", "igb_jacobi_diag", "igb_solve", "igb_potential",
    "igb_export_partition", "igb_export_pair_classes", "igb_export_near_block", "igb_export_coupling_block",
    "igb_plan_create", "igb_plan_destroy", "igb_plan_info", "igb_plan_export_partition",
    "igb_plan_export_pair_classes", "igb_matvec_profile", "igb_release_cached_memory",
    "igb_cnn_create", "igb_cnn_destroy", "igb_cnn_get_weights", "igb_cnn_forward", "igb_cnn_gradient",
    "igb_cnn_training_pairs", "igb_cnn_train", "igb_cnn_train_operator", "igb_solve_fgmres", "igb_solve_many",
    "igb_potential_noalloc", "igb_solve_fgmres_select", "igb_potential_h2",
]
IGB_CNN_NUM_WEIGHTS = 28224
IGB_CNN_RELU = 0
IGB_CNN_LINEAR = 1
CNN_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 32), (32, 1)]  # (c_in, c_out) of each 3x3 convolution
IGB_PROFILE_SEPARATE = 1
STAGES = ["upward", "coupling", "coupling_gather", "near_gemv", "near_gather", "downward"]


class igb_nurbs_patch(C.Structure):
    _fields_ = [("deg_u", C.c_int32), ("deg_v", C.c_int32), ("n_u", C.c_int32), ("n_v", C.c_int32),
                ("knots_u", C.POINTER(C.c_double)), ("knots_v", C.POINTER(C.c_double)),
                ("cpw", C.POINTER(C.c_double))]


class igb_params(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("wavenumber", C.c_double), ("p", C.c_int32), ("m", C.c_int32),
                ("q", C.c_int32), ("eta", C.c_double), ("leaf_depth", C.c_int32), ("gauss_regular", C.c_int32),
                ("gauss_singular", C.c_int32), ("gauss_rhs", C.c_int32), ("mode", C.c_int32),
                ("far_precision", C.c_int32), ("kappa_diam", C.c_double)]


class igb_info(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_dof_super", C.c_int64), ("n_elements", C.c_int64),
                ("n_rhs_points", C.c_int64), ("leaf_level", C.c_int32), ("gauss_singular", C.c_int32),
                ("gauss_rhs", C.c_int32), ("layout_flags", C.c_int32), ("n_near_blocks", C.c_int64),
                ("n_far_blocks", C.c_int64), ("n_pairs", C.c_int64 * 4), ("near_bytes", C.c_int64),
                ("coupling_bytes", C.c_int64), ("matvec_bytes", C.c_int64), ("setup_seconds", C.c_double),
                ("assembly_seconds", C.c_double), ("quad_points_regular", C.c_int64),
                ("quad_points_touching", C.c_int64), ("quad_regular_ms", C.c_double),
                ("quad_touching_ms", C.c_double)]


class igb_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double),
                ("fallback", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libigabem.so not built at {LIB_PATH}; run paper_1708_09162_amd/build.py")
    # torch first: its HIP runtime is then the one libigabem.so binds to (same soname).  Loaded the
    # other way round, the process would hold two HIP runtimes and the second one sees no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip, fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_float)
    sig = {
        "igb_last_error": (C.c_char_p, []),
        "igb_geometry_create": (C.c_int32, [C.c_int32, C.POINTER(igb_nurbs_patch), C.POINTER(vp)]),
        "igb_geometry_destroy": (None, [vp]),
        "igb_operator_create": (C.c_int32, [vp, C.POINTER(igb_params), vp, C.POINTER(vp)]),
        "igb_operator_destroy": (None, [vp]),
        "igb_operator_info": (C.c_int32, [vp, C.POINTER(igb_info)]),
        "igb_rhs_points": (C.c_int32, [vp, vp]),
        "igb_rhs_assemble": (C.c_int32, [vp, vp, vp]),
        "igb_matvec": (C.c_int32, [vp, vp, vp]),
        "igb_matvec_super": (C.c_int32, [vp, vp, vp]),
        "igb_apply_Tt": (C.c_int32, [vp, vp, vp]),
        "igb_apply_T": (C.c_int32, [vp, vp, vp]),
        "igb_jacobi_diag": (C.c_int32, [vp, vp]),
        "igb_solve": (C.c_int32, [vp, vp, vp, C.c_double, C.c_int32, C.c_int32, C.POINTER(igb_solve_info)]),
        "igb_potential": (C.c_int32, [vp, vp, C.c_int64, vp, vp]),
        "igb_potential_noalloc": (C.c_int32, [vp, vp, C.c_int64, vp, vp]),
        "igb_potential_h2": (C.c_int32, [vp, vp, C.c_int64, vp, vp]),
        "igb_export_partition": (C.c_int32, [vp, ip, ip]),
        "igb_export_pair_classes": (C.c_int32, [vp, ip]),
        "igb_export_near_block": (C.c_int32, [vp, C.c_int32, C.c_int32, dp]),
        "igb_export_coupling_block": (C.c_int32, [vp, C.c_int32, C.c_int32, C.c_int32, dp]),
        "igb_matvec_profile": (C.c_int32, [vp, C.c_int32, C.c_int32, dp]),
        "igb_plan_create": (C.c_int32, [vp, C.POINTER(igb_params), C.POINTER(vp)]),
        "igb_plan_destroy": (None, [vp]),
        "igb_plan_info": (C.c_int32, [vp, C.POINTER(igb_info)]),
        "igb_plan_export_partition": (C.c_int32, [vp, ip, ip]),
        "igb_plan_export_pair_classes": (C.c_int32, [vp, ip]),
        "igb_release_cached_memory": (C.c_int32, []),
        "igb_cnn_create": (C.c_int32, [fp, C.c_int32, vp, C.POINTER(vp)]),
        "igb_cnn_destroy": (None, [vp]),
        "igb_cnn_get_weights": (C.c_int32, [vp, fp]),
        "igb_cnn_forward": (C.c_int32, [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp]),
        "igb_cnn_gradient": (C.c_int32, [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, dp, fp]),
        "igb_cnn_training_pairs": (C.c_int32, [vp, vp, C.c_int64, vp, vp]),
        "igb_cnn_train": (C.c_int32, [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_float, dp]),
        "igb_solve_many": (C.c_int32, [C.c_int32, vp, vp, vp, C.c_double, C.c_int32, C.c_int32,
                                       C.POINTER(igb_solve_info)]),
        "igb_cnn_train_operator": (C.c_int32, [vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_float, dp]),
        "igb_solve_fgmres": (C.c_int32, [vp, vp, vp, vp, C.c_double, C.c_int32, C.c_int32,
                                         C.POINTER(igb_solve_info)]),
        "igb_solve_fgmres_select": (C.c_int32, [vp, vp, C.c_int32, vp, vp, vp, C.c_double, C.c_int32, C.c_int32,
                                                C.POINTER(C.c_int32), C.POINTER(igb_solve_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


class IgbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libigabem status {status}: {msg}")
        self.status = status


def igb_last_error() -> str:
    return (_lib.igb_last_error() or b"").decode()


def _check(status: int, allow=(IGB_OK,)):
    if status not in allow:
        raise IgbError(status, igb_last_error())
    return status


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# same-name wrappers of the C entry points
# ---------------------------------------------------------------------------
def igb_geometry_create(patches) -> C.c_void_p:
    """patches: list of dicts with deg_u, deg_v, knots_u, knots_v, cpw (n_v, n_u, 4)."""
    keep, arr = [], (igb_nurbs_patch * len(patches))()
    for i, p in enumerate(patches):
        cpw = np.ascontiguousarray(p["cpw"], dtype=np.float64)
        ku = np.ascontiguousarray(p["knots_u"], dtype=np.float64)
        kv = np.ascontiguousarray(p["knots_v"], dtype=np.float64)
        keep += [cpw, ku, kv]
        arr[i] = igb_nurbs_patch(int(p["deg_u"]), int(p["deg_v"]), cpw.shape[1], cpw.shape[0],
                                 ku.ctypes.data_as(C.POINTER(C.c_double)), kv.ctypes.data_as(C.POINTER(C.c_double)),
                                 cpw.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    _check(_lib.igb_geometry_create(len(patches), arr, C.byref(h)))
    return h


def igb_geometry_destroy(h):
    _lib.igb_geometry_destroy(h)


def igb_operator_create(geo, prm: igb_params, stream) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.igb_operator_create(geo, C.byref(prm), C.c_void_p(stream), C.byref(h)))
    return h


def igb_operator_destroy(h):
    _lib.igb_operator_destroy(h)


def igb_release_cached_memory() -> None:
    """Frees the device buffers the library keeps for reuse by later operators."""
    _check(_lib.igb_release_cached_memory())


def igb_operator_info(op) -> igb_info:
    out = igb_info()
    _check(_lib.igb_operator_info(op, C.byref(out)))
    return out


def igb_rhs_points(op, xyz):
    _check(_lib.igb_rhs_points(op, _ptr(xyz)))


def igb_rhs_assemble(op, g, b):
    _check(_lib.igb_rhs_assemble(op, _ptr(g), _ptr(b)))


def igb_matvec(op, x, y):
    _check(_lib.igb_matvec(op, _ptr(x), _ptr(y)))


def igb_matvec_super(op, xs, ys):
    _check(_lib.igb_matvec_super(op, _ptr(xs), _ptr(ys)))


def igb_apply_Tt(op, w, xs):
    _check(_lib.igb_apply_Tt(op, _ptr(w), _ptr(xs)))


def igb_apply_T(op, ys, y):
    _check(_lib.igb_apply_T(op, _ptr(ys), _ptr(y)))


def igb_jacobi_diag(op, d):
    _check(_lib.igb_jacobi_diag(op, _ptr(d)))


def igb_solve(op, b, w, rel_tol, max_iter, restart) -> igb_solve_info:
    info = igb_solve_info()
    _check(_lib.igb_solve(op, _ptr(b), _ptr(w), float(rel_tol), int(max_iter), int(restart), C.byref(info)),
           allow=(IGB_OK, IGB_ENOT_CONVERGED))
    return info


def igb_solve_fgmres(op, net, b, w, rel_tol, max_iter, restart) -> igb_solve_info:
    info = igb_solve_info()
    _check(_lib.igb_solve_fgmres(op, net, _ptr(b), _ptr(w), float(rel_tol), int(max_iter), int(restart),
                                 C.byref(info)), allow=(IGB_OK, IGB_ENOT_CONVERGED))
    return info


def igb_solve_fgmres_select(op, nets, v, b, w, rel_tol, max_iter, restart):
    """Returns (index of the kept network or -1 for Jacobi, info of the final solve)."""
    n = len(nets)
    arr = (C.c_void_p * max(n, 1))(*[x.value if isinstance(x, C.c_void_p) else x for x in nets])
    chosen, info = C.c_int32(-2), igb_solve_info()
    _check(_lib.igb_solve_fgmres_select(op, arr, n, _ptr(v), _ptr(b), _ptr(w), float(rel_tol), int(max_iter),
                                        int(restart), C.byref(chosen), C.byref(info)),
           allow=(IGB_OK, IGB_ENOT_CONVERGED))
    return chosen.value, info


def igb_solve_many(ops, bs, ws, rel_tol, max_iter, restart):
    n = len(ops)
    arr = lambda xs: (C.c_void_p * max(n, 1))(*xs)
    infos = (igb_solve_info * max(n, 1))()
    _check(_lib.igb_solve_many(n, arr([o.value for o in ops]), arr([t.data_ptr() for t in bs]),
                               arr([t.data_ptr() for t in ws]), float(rel_tol), int(max_iter), int(restart), infos),
           allow=(IGB_OK, IGB_ENOT_CONVERGED))
    return [infos[i] for i in range(n)]


def solve_many(operators, bs, tol=1e-8, max_iter=1000, restart=300):
    """Solves the systems of several operators at once (igb_solve_many); returns (densities, infos).  An
    operator may appear several times (several right-hand sides, solved in list order).  Instances overlap
    on the GPU when each operator was created with its own stream."""
    ws = [op._vec(op.info.n_dof) for op in operators]
    bs = [op._in(b, op.info.n_dof) for op, b in zip(operators, bs)]
    for op in {id(o): o for o in operators}.values():
        op.torch.cuda.synchronize(op.device)
    infos = igb_solve_many([op.h for op in operators], bs, ws, tol, max_iter, restart)
    return ws, infos


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def igb_cnn_create(weights, activation, stream) -> C.c_void_p:
    w = np.ascontiguousarray(weights, dtype=np.float32).reshape(-1)
    if w.size != IGB_CNN_NUM_WEIGHTS:
        raise ValueError(f"expected {IGB_CNN_NUM_WEIGHTS} weights, got {w.size}")
    h = C.c_void_p()
    _check(_lib.igb_cnn_create(_fptr(w), int(activation), C.c_void_p(stream), C.byref(h)))
    return h


def igb_cnn_get_weights(net):
    out = np.zeros(IGB_CNN_NUM_WEIGHTS, dtype=np.float32)
    _check(_lib.igb_cnn_get_weights(net, _fptr(out)))
    return out


def igb_cnn_forward(net, x, n_img, h, w, out):
    _check(_lib.igb_cnn_forward(net, _ptr(x), int(n_img), int(h), int(w), _ptr(out)))


def igb_cnn_gradient(net, x, target, n_img, h, w):
    loss = C.c_double()
    grad = np.zeros(IGB_CNN_NUM_WEIGHTS, dtype=np.float32)
    _check(_lib.igb_cnn_gradient(net, _ptr(x), _ptr(target), int(n_img), int(h), int(w), C.byref(loss),
                                 _fptr(grad)))
    return loss.value, grad


def igb_cnn_training_pairs(op, x, n_pairs, y32, x32):
    _check(_lib.igb_cnn_training_pairs(op, _ptr(x), int(n_pairs), _ptr(y32), _ptr(x32)))


def igb_cnn_train(net, y32, x32, n_pairs, imgs_per_pair, h, w, epochs, batch, lr):
    losses = np.zeros(max(int(epochs), 1), dtype=np.float64)
    _check(_lib.igb_cnn_train(net, _ptr(y32), _ptr(x32), int(n_pairs), int(imgs_per_pair), int(h), int(w),
                              int(epochs), int(batch), float(lr), losses.ctypes.data_as(C.POINTER(C.c_double))))
    return losses[:int(epochs)]


def igb_cnn_train_operator(net, op, y32, x32, n_pairs, epochs, batch, lr):
    losses = np.zeros(max(int(epochs), 1), dtype=np.float64)
    _check(_lib.igb_cnn_train_operator(net, op, _ptr(y32), _ptr(x32), int(n_pairs), int(epochs), int(batch),
                                       float(lr), losses.ctypes.data_as(C.POINTER(C.c_double))))
    return losses[:int(epochs)]


def igb_potential(op, w, xyz, u):
    n = xyz.shape[0]
    _check(_lib.igb_potential(op, _ptr(w), int(n), _ptr(xyz) if n else None, _ptr(u) if n else None))


def igb_potential_noalloc(op, w, xyz, u):
    n = xyz.shape[0]
    _check(_lib.igb_potential_noalloc(op, _ptr(w), int(n), _ptr(xyz) if n else None, _ptr(u) if n else None))


def igb_potential_h2(op, w, xyz, u):
    n = xyz.shape[0]
    _check(_lib.igb_potential_h2(op, _ptr(w), int(n), _ptr(xyz) if n else None, _ptr(u) if n else None))


def igb_export_partition(op, info: igb_info):
    near = np.zeros((info.n_near_blocks, 2), dtype=np.int32)
    far = np.zeros((info.n_far_blocks, 3), dtype=np.int32)
    _check(_lib.igb_export_partition(op, near.ctypes.data_as(C.POINTER(C.c_int32)),
                                     far.ctypes.data_as(C.POINTER(C.c_int32))))
    return near, far


def igb_export_pair_classes(op, info: igb_info):
    n = int(sum(info.n_pairs))
    out = np.zeros((n, 4), dtype=np.int32)
    _check(_lib.igb_export_pair_classes(op, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def igb_export_near_block(op, E, F, nloc, cplx):
    out = np.zeros((nloc, nloc, 2 if cplx else 1))
    _check(_lib.igb_export_near_block(op, int(E), int(F), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out[..., 0] + 1j * out[..., 1] if cplx else out[..., 0]


def igb_export_coupling_block(op, level, tgt, src, q2, cplx):
    out = np.zeros((q2, q2, 2 if cplx else 1))
    _check(_lib.igb_export_coupling_block(op, int(level), int(tgt), int(src),
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
    return out[..., 0] + 1j * out[..., 1] if cplx else out[..., 0]


def igb_matvec_profile(op, reps, flags=0):
    out = np.zeros(len(STAGES))
    _check(_lib.igb_matvec_profile(op, int(reps), int(flags), out.ctypes.data_as(C.POINTER(C.c_double))))
    return dict(zip(STAGES, out.tolist()))


def make_params(*, kernel=IGB_LAPLACE, wavenumber=0.0, p=1, m=2, q=8, eta=1.6, leaf_depth=-1, gauss_regular=6,
                gauss_singular=-1, gauss_rhs=-1, mode=IGB_H2_STORED, far_precision=IGB_FP64,
                kappa_diam=0.0) -> igb_params:
    return igb_params(int(kernel), float(wavenumber), int(p), int(m), int(q), float(eta), int(leaf_depth),
                      int(gauss_regular), int(gauss_singular), int(gauss_rhs), int(mode), int(far_precision),
                      float(kappa_diam))


def igb_plan_create(geo, prm: igb_params):
    h = C.c_void_p()
    _check(_lib.igb_plan_create(geo, C.byref(prm), C.byref(h)))
    return h


def igb_plan_destroy(h):
    _lib.igb_plan_destroy(h)


def igb_plan_info(plan) -> igb_info:
    out = igb_info()
    _check(_lib.igb_plan_info(plan, C.byref(out)))
    return out


def igb_plan_export_partition(plan, info: igb_info):
    near = np.zeros((info.n_near_blocks, 2), dtype=np.int32)
    far = np.zeros((info.n_far_blocks, 3), dtype=np.int32)
    _check(_lib.igb_plan_export_partition(plan, near.ctypes.data_as(C.POINTER(C.c_int32)),
                                          far.ctypes.data_as(C.POINTER(C.c_int32))))
    return near, far


def igb_plan_export_pair_classes(plan, info: igb_info):
    out = np.zeros((int(sum(info.n_pairs)), 4), dtype=np.int32)
    _check(_lib.igb_plan_export_pair_classes(plan, out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


class Plan:
    """Host-only plan: partition and pair classification without GPU work."""

    def __init__(self, geometry: "Geometry", **params):
        self.geometry = geometry
        self.h = igb_plan_create(geometry.h, make_params(**params))
        self.info = igb_plan_info(self.h)

    def __del__(self, _destroy=_lib.igb_plan_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def partition(self):
        return igb_plan_export_partition(self.h, self.info)

    def pair_classes(self):
        return igb_plan_export_pair_classes(self.h, self.info)


# ---------------------------------------------------------------------------
# convenience objects (still only marshalling)
# ---------------------------------------------------------------------------
class Geometry:
    def __init__(self, patches):
        self.h = igb_geometry_create(patches)

    # the destroy routine is bound at definition time: module globals may already be gone when an
    # object is collected at interpreter shutdown
    def __del__(self, _destroy=_lib.igb_geometry_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class _StreamOrdered:
    """Orders the object's HIP stream against torch's current stream around each library call.

    Inputs and zero-filled outputs are made on the current stream; the library works on the object's
    stream.  Before a call the object's stream waits for the current one, and after it the current stream
    waits for the object's, so results can be used on the current stream without a host synchronisation
    and temporaries freed on the current stream are not reused before the library is done with them."""

    @contextlib.contextmanager
    def _ordered(self):
        cur = self.torch.cuda.current_stream(self.device)
        other = cur.cuda_stream != self.stream.cuda_stream
        if other:
            self.stream.wait_stream(cur)
        try:
            yield
        finally:
            if other:
                cur.wait_stream(self.stream)


class Operator(_StreamOrdered):
    """An assembled single-layer operator on the current torch CUDA (HIP) stream."""

    def __init__(self, geometry: Geometry, *, kernel=IGB_LAPLACE, wavenumber=0.0, p=1, m=2, q=8, eta=1.6,
                 leaf_depth=-1, gauss_regular=6, gauss_singular=-1, gauss_rhs=-1, mode=IGB_H2_STORED,
                 far_precision=IGB_FP64, kappa_diam=0.0, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.geometry = geometry
        prm = make_params(kernel=kernel, wavenumber=wavenumber, p=p, m=m, q=q, eta=eta, leaf_depth=leaf_depth,
                          gauss_regular=gauss_regular, gauss_singular=gauss_singular, gauss_rhs=gauss_rhs, mode=mode,
                          far_precision=far_precision, kappa_diam=kappa_diam)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.h = igb_operator_create(geometry.h, prm, self.stream.cuda_stream)
        self.info = igb_operator_info(self.h)
        self.cplx = kernel == IGB_HELMHOLTZ
        self.dtype = torch.complex128 if self.cplx else torch.float64
        self.p, self.q, self.m = p, q, m

    def __del__(self, _destroy=_lib.igb_operator_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def _vec(self, n):
        return self.torch.zeros(int(n), dtype=self.dtype, device=self.device)

    def _in(self, t, n):
        t = t.to(device=self.device, dtype=self.dtype).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def rhs_points(self):
        xyz = self.torch.zeros((self.info.n_rhs_points, 3), dtype=self.torch.float64, device=self.device)
        with self._ordered():
            igb_rhs_points(self.h, xyz)
        return xyz

    def rhs(self, g):
        b, g = self._vec(self.info.n_dof), self._in(g, self.info.n_rhs_points)
        with self._ordered():
            igb_rhs_assemble(self.h, g, b)
        return b

    def matvec(self, x):
        y, x = self._vec(self.info.n_dof), self._in(x, self.info.n_dof)
        with self._ordered():
            igb_matvec(self.h, x, y)
        return y

    def matvec_super(self, xs):
        ys, xs = self._vec(self.info.n_dof_super), self._in(xs, self.info.n_dof_super)
        with self._ordered():
            igb_matvec_super(self.h, xs, ys)
        return ys

    def apply_Tt(self, w):
        xs, w = self._vec(self.info.n_dof_super), self._in(w, self.info.n_dof)
        with self._ordered():
            igb_apply_Tt(self.h, w, xs)
        return xs

    def apply_T(self, ys):
        y, ys = self._vec(self.info.n_dof), self._in(ys, self.info.n_dof_super)
        with self._ordered():
            igb_apply_T(self.h, ys, y)
        return y

    def jacobi_diag(self):
        d = self._vec(self.info.n_dof)
        with self._ordered():
            igb_jacobi_diag(self.h, d)
        return d

    def solve(self, b, w0=None, tol=1e-8, max_iter=1000, restart=300):
        w = self._vec(self.info.n_dof) if w0 is None else self._in(w0, self.info.n_dof).clone()
        b = self._in(b, self.info.n_dof)
        with self._ordered():
            info = igb_solve(self.h, b, w, tol, max_iter, restart)
        return w, info

    def solve_fgmres(self, b, net=None, w0=None, tol=1e-8, max_iter=1000, restart=100):
        """Flexible GMRES with the network preconditioner `net` (a CNN), or Jacobi when net is None."""
        w = self._vec(self.info.n_dof) if w0 is None else self._in(w0, self.info.n_dof).clone()
        b = self._in(b, self.info.n_dof)
        with self._ordered():
            info = igb_solve_fgmres(self.h, net.h if net is not None else None, b, w, tol, max_iter, restart)
        return w, info

    def solve_fgmres_select(self, nets, v, b, w0=None, tol=1e-8, max_iter=1000, restart=100):
        """Keeps the network (or Jacobi) with the fewest flexible-GMRES steps on the validation right-hand side
        v, then solves for b with it (igb_solve_fgmres_select); returns (w, kept index or -1, info)."""
        w = self._vec(self.info.n_dof) if w0 is None else self._in(w0, self.info.n_dof).clone()
        b = self._in(b, self.info.n_dof)
        v = self._in(v, self.info.n_dof)
        with self._ordered():
            chosen, info = igb_solve_fgmres_select(self.h, [x.h for x in nets], v, b, w, tol, max_iter, restart)
        return w, chosen, info

    @property
    def grid(self):
        """(patches, side): a vector of S is `patches` coefficient grids of side x side."""
        side = (1 << self.m) + self.p
        return self.info.n_dof // (side * side), side

    def training_pairs(self, x):
        """(D^-1 A x_s, x_s) in FP32 for the rows x_s of x (n_pairs x n_dof, FP64)."""
        x = x.to(device=self.device, dtype=self.torch.float64).contiguous()
        n_pairs = x.shape[0]
        if x.numel() != n_pairs * self.info.n_dof:
            raise ValueError("x must be n_pairs x n_dof")
        y32 = self.torch.empty((n_pairs, self.info.n_dof), dtype=self.torch.float32, device=self.device)
        x32 = self.torch.empty_like(y32)
        with self._ordered():
            igb_cnn_training_pairs(self.h, x, n_pairs, y32, x32)
        return y32, x32

    def potential(self, w, points):
        pts = self.torch.as_tensor(points, dtype=self.torch.float64).to(self.device).reshape(-1, 3).contiguous()
        u, w = self._vec(pts.shape[0]), self._in(w, self.info.n_dof)
        with self._ordered():
            igb_potential(self.h, w, pts, u)
        return u

    def potential_h2(self, w, points):
        """Potential with the far field interpolated at the clusters' Chebyshev nodes (igb_potential_h2)."""
        pts = self.torch.as_tensor(points, dtype=self.torch.float64).to(self.device).reshape(-1, 3).contiguous()
        u, w = self._vec(pts.shape[0]), self._in(w, self.info.n_dof)
        with self._ordered():
            igb_potential_h2(self.h, w, pts, u)
        return u

    def potential_noalloc(self, w, points, out):
        """Potential into the preallocated `out` without any device allocation by the library
        (igb_potential_noalloc; asynchronous on the operator's stream)."""
        pts = self.torch.as_tensor(points, dtype=self.torch.float64).to(self.device).reshape(-1, 3).contiguous()
        w = self._in(w, self.info.n_dof)
        if out.numel() != pts.shape[0] or out.dtype != self.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous vector of n_pts values of the operator's dtype")
        with self._ordered():
            igb_potential_noalloc(self.h, w, pts, out)
        return out

    def profile(self, reps=10, separate=False):
        """Mean milliseconds per matvec stage, from HIP events on the operator's stream; with
        separate=True the far- and near-field products run as separate launches."""
        return igb_matvec_profile(self.h, reps, IGB_PROFILE_SEPARATE if separate else 0)

    def partition(self):
        return igb_export_partition(self.h, self.info)

    def pair_classes(self):
        return igb_export_pair_classes(self.h, self.info)

    def near_block(self, E, F):
        return igb_export_near_block(self.h, E, F, (self.p + 1) ** 2, self.cplx)

    def coupling_block(self, level, tgt, src):
        return igb_export_coupling_block(self.h, level, tgt, src, self.q * self.q, self.cplx)


class CNN(_StreamOrdered):
    """The learned preconditioner's network on the current torch CUDA (HIP) stream."""

    def __init__(self, weights, activation=IGB_CNN_RELU, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.activation = activation
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.h = igb_cnn_create(weights, activation, self.stream.cuda_stream)

    def __del__(self, _destroy=_lib.igb_cnn_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def _f32(self, t):
        return t.to(device=self.device, dtype=self.torch.float32).contiguous()

    def weights(self):
        return igb_cnn_get_weights(self.h)

    def forward(self, x, n_img, h, w):
        """x + f(x) for n_img images of h x w."""
        x = self._f32(x)
        out = self.torch.empty_like(x)
        with self._ordered():
            igb_cnn_forward(self.h, x, n_img, h, w, out)
        return out

    def gradient(self, x, target, n_img, h, w):
        """(loss, gradient with respect to the weights) of one batch."""
        x, target = self._f32(x), self._f32(target)
        with self._ordered():
            return igb_cnn_gradient(self.h, x, target, n_img, h, w)

    def train(self, y32, x32, imgs_per_pair, h, w, epochs=5, batch=16, lr=1e-3):
        """Adam over the (y, x) pairs (rows of y32, x32); returns the mean loss of each epoch."""
        y32, x32 = self._f32(y32), self._f32(x32)
        with self._ordered():
            return igb_cnn_train(self.h, y32, x32, y32.shape[0], imgs_per_pair, h, w, epochs, batch, lr)

    def train_operator(self, op, y32, x32, epochs=5, batch=16, lr=1e-3):
        """Adam on the preconditioned residual |D^-1 A (M(y) - x)|^2 of operator `op` over the pairs."""
        y32, x32 = self._f32(y32), self._f32(x32)
        with self._ordered(), op._ordered():
            return igb_cnn_train_operator(self.h, op.h, y32, x32, y32.shape[0], epochs, batch, lr)
