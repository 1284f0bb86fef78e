"""Thin ctypes binding of libstokesreg.so (C ABI in include/stokesreg.h).

Argument marshalling only: torch supplies device memory and the stream; every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: if the library is not built, or no GPU
is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstokesreg.so")

SR_OK, SR_EINVAL, SR_ENOMEM, SR_ENODEV, SR_ESTATE, SR_EHIP, SR_ENOCONV, SR_ENEAR = 0, -1, -2, -3, -4, -5, -6, -7
SR_SL, SR_DL, SR_HOST = 1, 2, 16
SR_FP64, SR_MIXED = 0, 1
SR_DIRECT, SR_TREE = 0, 1
_NAMES = {0: "SR_OK", -1: "SR_EINVAL", -2: "SR_ENOMEM", -3: "SR_ENODEV", -4: "SR_ESTATE", -5: "SR_EHIP",
          -6: "SR_ENOCONV", -7: "SR_ENEAR"}

# every symbol the header declares; the CPU test-suite checks that the library exports each one
EXPORTS = ("sr_default_params", "sr_create", "sr_destroy", "sr_set_params", "sr_set_surface", "sr_set_density",
           "sr_eval", "sr_eval_far", "sr_eval_noalloc", "sr_check", "sr_max_targets", "sr_near_table", "sr_set_profiling", "sr_get_profile", "sr_tree_work", "sr_rigid_create", "sr_rigid_destroy",
           "sr_rigid_set_params", "sr_rigid_set_spheres", "sr_rigid_rhs", "sr_rigid_matvec", "sr_rigid_solve",
           "sr_rigid_solve_refined", "sr_rigid_set_operator", "sr_rigid_single_layer", "sr_rigid_velocity", "sr_rigid_last_error", "sr_prolong_create",
           "sr_prolong_apply", "sr_prolong_destroy", "sr_mlp_num_params", "sr_mlp_create", "sr_mlp_destroy",
           "sr_mlp_set_options", "sr_mlp_set_params", "sr_mlp_get_params", "sr_mlp_set_output_scale",
           "sr_mlp_fit_output_scale", "sr_mlp_get_output_scale", "sr_mlp_forward", "sr_mlp_predict",
           "sr_mlp_gradients", "sr_mlp_train_step", "sr_mlp_set_profiling", "sr_mlp_get_profile",
           "sr_mlp_gemm_test", "sr_mlp_last_error", "sr_last_error",
           "sr_version")
SR_PHASE_FAR, SR_PHASE_NEAR, SR_NPHASES = 0, 1, 2


class SrParams(C.Structure):
    _fields_ = [("h", C.c_double), ("rho", C.c_double * 3), ("cutoff", C.c_double), ("precision", C.c_int),
                ("far_method", C.c_int), ("tree_degree", C.c_int), ("tree_theta", C.c_double),
                ("tree_leaf", C.c_int), ("surface_sharp", C.c_int), ("sharp_rho", C.c_double)]


class SrError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libstokesreg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() (hipcc, gfx950) first")
    L = C.CDLL(path)
    vp, d, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int64
    L.sr_default_params.argtypes = [C.POINTER(SrParams)]
    L.sr_default_params.restype = None
    L.sr_create.argtypes = [C.POINTER(vp), C.c_int]
    L.sr_destroy.argtypes = [vp]
    L.sr_set_params.argtypes = [vp, C.POINTER(SrParams)]
    L.sr_set_surface.argtypes = [vp, i64, vp, vp, vp, vp]
    L.sr_set_density.argtypes = [vp, C.c_int, vp, vp]
    L.sr_eval.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.sr_eval_far.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp]
    L.sr_eval_noalloc.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.sr_check.argtypes = [vp, vp]
    L.sr_max_targets.argtypes = []
    L.sr_max_targets.restype = i64
    L.sr_near_table.argtypes = [d, C.c_double, C.c_double, d, i64, d]
    L.sr_set_profiling.argtypes = [vp, C.c_int]
    L.sr_get_profile.argtypes = [vp, d, C.POINTER(C.c_int64)]
    L.sr_tree_work.argtypes = [vp, i64, vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.sr_rigid_create.argtypes = [C.POINTER(vp), C.c_int]
    L.sr_rigid_destroy.argtypes = [vp]
    L.sr_rigid_set_params.argtypes = [vp, C.POINTER(SrParams)]
    L.sr_rigid_set_spheres.argtypes = [vp, C.c_int, d, d, C.POINTER(C.c_int64), vp, vp, vp, vp]
    L.sr_rigid_rhs.argtypes = [vp, d, vp, vp]
    L.sr_rigid_matvec.argtypes = [vp, vp, vp, vp]
    L.sr_rigid_solve.argtypes = [vp, vp, vp, C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                                 C.POINTER(C.c_double), vp]
    L.sr_rigid_solve_refined.argtypes = [vp, vp, vp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
                                         C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double), vp]
    L.sr_rigid_set_operator.argtypes = [vp, C.c_double, C.c_double, C.c_int]
    L.sr_rigid_single_layer.argtypes = [vp, vp, vp, vp]
    L.sr_rigid_velocity.argtypes = [vp, vp, i64, vp, vp, vp]
    L.sr_rigid_last_error.argtypes = []
    L.sr_rigid_last_error.restype = C.c_char_p
    L.sr_prolong_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, d, d, C.c_double, C.POINTER(C.c_int64), vp, vp,
                                    C.POINTER(C.c_int64), vp, vp]
    L.sr_prolong_apply.argtypes = [vp, vp, vp, vp]
    L.sr_prolong_destroy.argtypes = [vp]
    L.sr_mlp_num_params.argtypes = [C.c_int, i64]
    L.sr_mlp_num_params.restype = i64
    L.sr_mlp_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, i64, C.c_int]
    L.sr_mlp_destroy.argtypes = [vp]
    L.sr_mlp_set_options.argtypes = [vp, C.c_int, C.c_double, C.c_double]
    L.sr_mlp_set_params.argtypes = [vp, C.POINTER(C.c_float)]
    L.sr_mlp_get_params.argtypes = [vp, C.POINTER(C.c_float)]
    L.sr_mlp_set_output_scale.argtypes = [vp, vp, vp]
    L.sr_mlp_fit_output_scale.argtypes = [vp, i64, vp, vp]
    L.sr_mlp_get_output_scale.argtypes = [vp, vp, vp]
    L.sr_mlp_forward.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.sr_mlp_predict.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.sr_mlp_gradients.argtypes = [vp, C.c_int, vp, i64, vp, vp, vp, vp, d, vp]
    L.sr_mlp_train_step.argtypes = [vp, C.c_int, vp, i64, vp, vp, vp, C.c_float, d, vp]
    L.sr_mlp_set_profiling.argtypes = [vp, C.c_int]
    L.sr_mlp_get_profile.argtypes = [vp, d, C.POINTER(C.c_int64)]
    L.sr_mlp_gemm_test.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp]
    L.sr_mlp_last_error.argtypes = []
    L.sr_mlp_last_error.restype = C.c_char_p
    for fn in ("sr_prolong_create", "sr_prolong_apply", "sr_prolong_destroy", "sr_mlp_create", "sr_mlp_destroy",
               "sr_mlp_set_options", "sr_mlp_set_params", "sr_mlp_get_params", "sr_mlp_set_output_scale",
               "sr_mlp_fit_output_scale", "sr_mlp_get_output_scale", "sr_mlp_forward", "sr_mlp_predict",
               "sr_mlp_gradients", "sr_mlp_train_step", "sr_mlp_set_profiling", "sr_mlp_get_profile",
               "sr_mlp_gemm_test"):
        getattr(L, fn).restype = C.c_int
    L.sr_last_error.argtypes = []
    L.sr_last_error.restype = C.c_char_p
    L.sr_version.argtypes = []
    L.sr_version.restype = C.c_char_p
    for fn in ("sr_create", "sr_destroy", "sr_set_params", "sr_set_surface", "sr_set_density", "sr_eval",
               "sr_eval_far", "sr_eval_noalloc", "sr_check", "sr_near_table", "sr_set_profiling", "sr_get_profile", "sr_tree_work", "sr_rigid_create", "sr_rigid_destroy",
               "sr_rigid_set_params",
               "sr_rigid_set_spheres", "sr_rigid_rhs", "sr_rigid_matvec", "sr_rigid_solve", "sr_rigid_solve_refined",
               "sr_rigid_set_operator", "sr_rigid_single_layer", "sr_rigid_velocity"):
        getattr(L, fn).restype = C.c_int
    _lib = L
    return L


def _check(fn: str, st: int) -> None:
    if st != SR_OK:
        raise SrError(fn, st, load_library().sr_last_error().decode())


def _ptr(t, name: str, shape_last=None):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA torch.Tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous float64 tensor")
    if shape_last is not None and (t.dim() != 2 or t.shape[1] != shape_last):
        raise ValueError(f"{name}: expected shape (k, {shape_last}), got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def sr_default_params() -> SrParams:
    p = SrParams()
    load_library().sr_default_params(C.byref(p))
    return p


def sr_create(device: int = 0) -> C.c_void_p:
    h = C.c_void_p()
    _check("sr_create", load_library().sr_create(C.byref(h), int(device)))
    return h


def sr_destroy(ctx) -> None:
    _check("sr_destroy", load_library().sr_destroy(ctx))


def sr_set_params(ctx, params: SrParams) -> None:
    _check("sr_set_params", load_library().sr_set_params(ctx, C.byref(params)))


def sr_set_surface(ctx, x, nrm, w, stream=None) -> None:
    n = int(x.shape[0])
    if w.dim() != 1 or w.shape[0] != n or nrm.shape[0] != n:
        raise ValueError("sr_set_surface: x, nrm, w sizes differ")
    _check("sr_set_surface", load_library().sr_set_surface(ctx, n, _ptr(x, "x", 3), _ptr(nrm, "nrm", 3),
                                                           _ptr(w, "w"), _stream(stream)))


def sr_set_density(ctx, layer: int, dens, stream=None) -> None:
    _check("sr_set_density", load_library().sr_set_density(ctx, int(layer), _ptr(dens, "dens", 3), _stream(stream)))


def sr_eval(ctx, layers: int, y, x0, n0, b, f0=None, q0=None, u=None, v=None, u_delta=None, v_delta=None,
            stream=None) -> None:
    m = int(y.shape[0])
    for name, t, last in (("x0", x0, 3), ("n0", n0, 3), ("f0", f0, 3), ("q0", q0, 3), ("u", u, 3), ("v", v, 3)):
        if t is not None and (t.dim() != 2 or t.shape[0] != m or t.shape[1] != last):
            raise ValueError(f"sr_eval: {name} must have shape ({m}, 3)")
    if b.dim() != 1 or b.shape[0] != m:
        raise ValueError(f"sr_eval: b must have shape ({m},)")
    for name, t in (("u_delta", u_delta), ("v_delta", v_delta)):
        if t is not None and tuple(t.shape) != (m, 3, 3):
            raise ValueError(f"sr_eval: {name} must have shape ({m}, 3, 3)")
    _check("sr_eval", load_library().sr_eval(ctx, int(layers), m, _ptr(y, "y", 3), _ptr(x0, "x0", 3),
                                             _ptr(n0, "n0", 3), _ptr(b, "b"), _ptr(f0, "f0"), _ptr(q0, "q0"),
                                             _ptr(u, "u"), _ptr(v, "v"), _ptr(u_delta, "u_delta"),
                                             _ptr(v_delta, "v_delta"), _stream(stream)))


SR_NOALLOC_MAX_TARGETS = 65536


def sr_eval_noalloc(ctx, layers: int, y, x0, n0, b, f0=None, q0=None, u=None, v=None, stream=None) -> None:
    """sr_eval without device allocation (device tensors; at most SR_NOALLOC_MAX_TARGETS targets)."""
    m = int(y.shape[0])
    for name, t in (("x0", x0), ("n0", n0), ("f0", f0), ("q0", q0), ("u", u), ("v", v)):
        if t is not None and tuple(t.shape) != (m, 3):
            raise ValueError(f"sr_eval_noalloc: {name} must have shape ({m}, 3)")
    if b.dim() != 1 or b.shape[0] != m:
        raise ValueError(f"sr_eval_noalloc: b must have shape ({m},)")
    _check("sr_eval_noalloc", load_library().sr_eval_noalloc(
        ctx, int(layers), m, _ptr(y, "y", 3), _ptr(x0, "x0", 3), _ptr(n0, "n0", 3), _ptr(b, "b"), _ptr(f0, "f0"),
        _ptr(q0, "q0"), _ptr(u, "u"), _ptr(v, "v"), _stream(stream)))


def sr_eval_far(ctx, layers: int, y, u=None, v=None, stream=None) -> None:
    """Plain sums at targets with no closest point (device tensors)."""
    m = int(y.shape[0])
    for name, t in (("u", u), ("v", v)):
        if t is not None and tuple(t.shape) != (m, 3):
            raise ValueError(f"sr_eval_far: {name} must have shape ({m}, 3)")
    _check("sr_eval_far", load_library().sr_eval_far(ctx, int(layers), m, _ptr(y, "y", 3), _ptr(u, "u"),
                                                     _ptr(v, "v"), _stream(stream)))


def _hptr(a, name, shape, writable=False):
    """Host pointer of a C-contiguous float64 numpy array of the given shape (None -> NULL)."""
    import numpy as np

    if a is None:
        return None
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"{name}: expected a C-contiguous float64 numpy array")
    if a.shape != shape:
        raise ValueError(f"{name}: expected shape {shape}, got {a.shape}")
    if writable and not a.flags["WRITEABLE"]:
        raise ValueError(f"{name}: not writable")
    return C.c_void_p(a.ctypes.data)


def sr_eval_host(ctx, layers: int, y, x0, n0, b, f0=None, q0=None, u=None, v=None, stream=None) -> None:
    """sr_eval with host (numpy) arrays: SR_HOST mode, synchronous."""
    m = int(y.shape[0])
    _check("sr_eval", load_library().sr_eval(
        ctx, int(layers) | SR_HOST, m, _hptr(y, "y", (m, 3)), _hptr(x0, "x0", (m, 3)), _hptr(n0, "n0", (m, 3)),
        _hptr(b, "b", (m,)), _hptr(f0, "f0", (m, 3)), _hptr(q0, "q0", (m, 3)), _hptr(u, "u", (m, 3), True),
        _hptr(v, "v", (m, 3), True), None, None, _stream(stream)))


def sr_eval_far_host(ctx, layers: int, y, u=None, v=None, stream=None) -> None:
    """sr_eval_far with host (numpy) arrays: SR_HOST mode, synchronous."""
    m = int(y.shape[0])
    _check("sr_eval_far", load_library().sr_eval_far(ctx, int(layers) | SR_HOST, m, _hptr(y, "y", (m, 3)),
                                                     _hptr(u, "u", (m, 3), True), _hptr(v, "v", (m, 3), True),
                                                     _stream(stream)))


def sr_check(ctx, stream=None) -> None:
    """Raises SrError(SR_ENEAR) if a target treated as far from the surface had a source within the near
    radius since the last check (waits for the stream)."""
    _check("sr_check", load_library().sr_check(ctx, _stream(stream)))


def sr_max_targets() -> int:
    return int(load_library().sr_max_targets())


SR_NEAR_TABLE_INTERVALS, SR_NEAR_TABLE_DEGREE = 160, 7
SR_NEAR_TABLE_DOUBLES = SR_NEAR_TABLE_INTERVALS * 3 * (SR_NEAR_TABLE_DEGREE + 1)


def sr_near_table(rho, cutoff: float, xmax: float):
    """The surface-target smoothing table (host only): returns (coefficients as a float64 array of
    shape (3, (D + 1) / 2, NI, 2), the checked interpolation error).  Coefficient e of function f on
    interval i is out[f, e // 2, i, e % 2]."""
    import numpy as np

    r = (C.c_double * 3)(*[float(v) for v in rho])
    tab = np.zeros(SR_NEAR_TABLE_DOUBLES)
    err = C.c_double()
    _check("sr_near_table", load_library().sr_near_table(r, float(cutoff), float(xmax),
                                                         tab.ctypes.data_as(C.POINTER(C.c_double)),
                                                         SR_NEAR_TABLE_DOUBLES, C.byref(err)))
    return tab.reshape(3, (SR_NEAR_TABLE_DEGREE + 1) // 2, SR_NEAR_TABLE_INTERVALS, 2), float(err.value)


def sr_set_profiling(ctx, on: bool) -> None:
    _check("sr_set_profiling", load_library().sr_set_profiling(ctx, int(bool(on))))


def sr_get_profile(ctx):
    """Returns ([ms_far, ms_near], number_of_evaluations) accumulated since the last call."""
    ms = (C.c_double * SR_NPHASES)()
    ne = C.c_int64()
    _check("sr_get_profile", load_library().sr_get_profile(ctx, ms, C.byref(ne)))
    return list(ms), int(ne.value)


def sr_tree_work(ctx, y_host):
    """Treecode far-field work for targets y_host ((m,3) float64 numpy array, host memory):
    returns (target-proxy interactions, leaf pairs, points inside accepted clusters)."""
    import numpy as np

    y = np.ascontiguousarray(y_host, dtype=np.float64)
    if y.ndim != 2 or y.shape[1] != 3:
        raise ValueError("sr_tree_work: y must be (m, 3)")
    npx, nlf, ncl = C.c_int64(), C.c_int64(), C.c_int64()
    _check("sr_tree_work", load_library().sr_tree_work(ctx, int(y.shape[0]), y.ctypes.data_as(C.c_void_p),
                                                       C.byref(npx), C.byref(nlf), C.byref(ncl)))
    return int(npx.value), int(nlf.value), int(ncl.value)


def _rcheck(fn: str, st: int) -> None:
    if st != SR_OK:
        raise SrError(fn, st, load_library().sr_rigid_last_error().decode())


def sr_rigid_create(device: int = 0):
    h = C.c_void_p()
    _rcheck("sr_rigid_create", load_library().sr_rigid_create(C.byref(h), int(device)))
    return h


def sr_rigid_destroy(r) -> None:
    _rcheck("sr_rigid_destroy", load_library().sr_rigid_destroy(r))


def sr_rigid_set_params(r, params: SrParams) -> None:
    _rcheck("sr_rigid_set_params", load_library().sr_rigid_set_params(r, C.byref(params)))


def sr_rigid_set_spheres(r, centers, radii, counts, x, nrm, w, stream=None) -> None:
    import numpy as np

    cen = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    rad = np.ascontiguousarray(radii, dtype=np.float64).ravel()
    cnt = np.ascontiguousarray(counts, dtype=np.int64).ravel()
    ns = cen.shape[0]
    if rad.size != ns or cnt.size != ns or int(cnt.sum()) != int(x.shape[0]):
        raise ValueError("sr_rigid_set_spheres: inconsistent sizes")
    dp = C.POINTER(C.c_double)
    _rcheck("sr_rigid_set_spheres", load_library().sr_rigid_set_spheres(
        r, ns, cen.ctypes.data_as(dp), rad.ctypes.data_as(dp), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
        _ptr(x, "x", 3), _ptr(nrm, "nrm", 3), _ptr(w, "w"), _stream(stream)))


def sr_rigid_rhs(r, motion, rhs, stream=None) -> None:
    import numpy as np

    mo = np.ascontiguousarray(motion, dtype=np.float64).reshape(-1, 6)
    _rcheck("sr_rigid_rhs", load_library().sr_rigid_rhs(r, mo.ctypes.data_as(C.POINTER(C.c_double)),
                                                        _ptr(rhs, "rhs", 3), _stream(stream)))


def sr_rigid_matvec(r, q, out, stream=None) -> None:
    _rcheck("sr_rigid_matvec", load_library().sr_rigid_matvec(r, _ptr(q, "q", 3), _ptr(out, "out", 3),
                                                              _stream(stream)))


def sr_rigid_solve(r, rhs, x, x_is_guess=False, tol=1e-8, maxit=200, restart=60, stream=None):
    """Returns (iterations, relative residual)."""
    it = C.c_int()
    rr = C.c_double()
    st = load_library().sr_rigid_solve(r, _ptr(rhs, "rhs", 3), _ptr(x, "x", 3), int(bool(x_is_guess)), float(tol),
                                       int(maxit), int(restart), C.byref(it), C.byref(rr), _stream(stream))
    _rcheck("sr_rigid_solve", st)
    return int(it.value), float(rr.value)


def sr_rigid_solve_refined(r, rhs, x, x_is_guess=False, tol=1e-10, inner_tol=1e-6, maxit=400, restart=60,
                           stream=None):
    """Returns (inner iterations, outer corrections, FP64 relative residual)."""
    it = C.c_int()
    no = C.c_int()
    rr = C.c_double()
    st = load_library().sr_rigid_solve_refined(r, _ptr(rhs, "rhs", 3), _ptr(x, "x", 3), int(bool(x_is_guess)),
                                               float(tol), float(inner_tol), int(maxit), int(restart), C.byref(it),
                                               C.byref(no), C.byref(rr), _stream(stream))
    _rcheck("sr_rigid_solve_refined", st)
    return int(it.value), int(no.value), float(rr.value)


def sr_rigid_set_operator(r, a_id: float, a_dl: float, completion: bool) -> None:
    _rcheck("sr_rigid_set_operator", load_library().sr_rigid_set_operator(r, float(a_id), float(a_dl),
                                                                          int(bool(completion))))


def sr_rigid_single_layer(r, f, out, stream=None) -> None:
    _rcheck("sr_rigid_single_layer", load_library().sr_rigid_single_layer(r, _ptr(f, "f", 3), _ptr(out, "out", 3),
                                                                          _stream(stream)))


def sr_rigid_velocity(r, q, y, u, stream=None) -> None:
    _rcheck("sr_rigid_velocity", load_library().sr_rigid_velocity(r, _ptr(q, "q", 3), int(y.shape[0]),
                                                                  _ptr(y, "y", 3), _ptr(u, "u", 3),
                                                                  _stream(stream)))


def sr_prolong_create(centers, radii, hc, counts_c, xc, nc, counts_f, xf, device: int = 0, stream=None):
    import numpy as np

    ce = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    ra = np.ascontiguousarray(radii, dtype=np.float64).ravel()
    cc = np.ascontiguousarray(counts_c, dtype=np.int64).ravel()
    cf = np.ascontiguousarray(counts_f, dtype=np.int64).ravel()
    ns = ce.shape[0]
    if ra.size != ns or cc.size != ns or cf.size != ns:
        raise ValueError("sr_prolong_create: inconsistent sphere counts")
    if xc.shape[0] != int(cc.sum()) or nc.shape[0] != xc.shape[0] or xf.shape[0] != int(cf.sum()):
        raise ValueError("sr_prolong_create: inconsistent point counts")
    h = C.c_void_p()
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int64)
    _rcheck("sr_prolong_create", load_library().sr_prolong_create(
        C.byref(h), int(device), ns, ce.ctypes.data_as(dp), ra.ctypes.data_as(dp), float(hc), cc.ctypes.data_as(ip),
        _ptr(xc, "xc", 3), _ptr(nc, "nc", 3), cf.ctypes.data_as(ip), _ptr(xf, "xf", 3), _stream(stream)))
    return h


def sr_prolong_apply(p, qc, qf, stream=None) -> None:
    _rcheck("sr_prolong_apply", load_library().sr_prolong_apply(p, _ptr(qc, "qc", 3), _ptr(qf, "qf", 3),
                                                                _stream(stream)))


def sr_prolong_destroy(p) -> None:
    _rcheck("sr_prolong_destroy", load_library().sr_prolong_destroy(p))


def _mcheck(fn: str, st: int) -> None:
    if st != SR_OK:
        raise SrError(fn, st, load_library().sr_mlp_last_error().decode())


def _tptr(t, name: str, dtype_name: str, numel=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype (None -> NULL)."""
    if t is None:
        return None
    import torch

    dt = {"f32": torch.float32, "f64": torch.float64, "i64": torch.int64}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous CUDA {dt} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _rows(gap, motion, y) -> int:
    """Rows of a resident data set (gap (n,), motion (n,12), y (n,nout)), checked for agreement."""
    n = int(gap.shape[0])
    if motion.numel() != 12 * n or y.shape[0] != n:
        raise ValueError("gap, motion and y must have the same number of rows")
    return n


def sr_mlp_num_params(width: int, nout: int) -> int:
    return int(load_library().sr_mlp_num_params(int(width), int(nout)))


def sr_mlp_create(width: int, nout: int, max_batch: int, device: int = 0):
    h = C.c_void_p()
    _mcheck("sr_mlp_create", load_library().sr_mlp_create(C.byref(h), int(device), int(width), int(nout),
                                                          int(max_batch)))
    return h


def sr_mlp_destroy(net) -> None:
    _mcheck("sr_mlp_destroy", load_library().sr_mlp_destroy(net))


def sr_mlp_set_options(net, passes: int = 3, g_mid: float = -2.760730458931123, g_half: float = 1.151292546497023) -> None:
    _mcheck("sr_mlp_set_options", load_library().sr_mlp_set_options(net, int(passes), float(g_mid), float(g_half)))


def sr_mlp_set_params(net, params) -> None:
    import numpy as np

    a = np.ascontiguousarray(params, dtype=np.float32)
    _mcheck("sr_mlp_set_params", load_library().sr_mlp_set_params(net, a.ctypes.data_as(C.POINTER(C.c_float))))


def sr_mlp_get_params(net, nparam: int):
    import numpy as np

    a = np.empty(int(nparam), dtype=np.float32)
    _mcheck("sr_mlp_get_params", load_library().sr_mlp_get_params(net, a.ctypes.data_as(C.POINTER(C.c_float))))
    return a


def sr_mlp_set_output_scale(net, s, stream=None) -> None:
    _mcheck("sr_mlp_set_output_scale", load_library().sr_mlp_set_output_scale(net, _tptr(s, "s", "f64"),
                                                                              _stream(stream)))


def sr_mlp_fit_output_scale(net, y, stream=None) -> None:
    _mcheck("sr_mlp_fit_output_scale", load_library().sr_mlp_fit_output_scale(net, int(y.shape[0]),
                                                                              _tptr(y, "y", "f64"), _stream(stream)))


def sr_mlp_get_output_scale(net, s, stream=None) -> None:
    _mcheck("sr_mlp_get_output_scale", load_library().sr_mlp_get_output_scale(net, _tptr(s, "s", "f64"),
                                                                              _stream(stream)))


def sr_mlp_forward(net, gap, motion, out, stream=None) -> None:
    b = int(gap.shape[0])
    _mcheck("sr_mlp_forward", load_library().sr_mlp_forward(net, b, _tptr(gap, "gap", "f64"),
                                                            _tptr(motion, "motion", "f64", 12 * b),
                                                            _tptr(out, "out", "f32"), _stream(stream)))


def sr_mlp_predict(net, gap, motion, q, stream=None) -> None:
    b = int(gap.shape[0])
    _mcheck("sr_mlp_predict", load_library().sr_mlp_predict(net, b, _tptr(gap, "gap", "f64"),
                                                            _tptr(motion, "motion", "f64", 12 * b),
                                                            _tptr(q, "q", "f64"), _stream(stream)))


def sr_mlp_gradients(net, batch, idx, gap, motion, y, grad, stream=None) -> float:
    loss = C.c_double()
    _mcheck("sr_mlp_gradients", load_library().sr_mlp_gradients(
        net, int(batch), _tptr(idx, "idx", "i64"), _rows(gap, motion, y), _tptr(gap, "gap", "f64"),
        _tptr(motion, "motion", "f64"),
        _tptr(y, "y", "f64"), _tptr(grad, "grad", "f32"), C.byref(loss), _stream(stream)))
    return float(loss.value)


def sr_mlp_train_step(net, batch, idx, gap, motion, y, lr, want_loss=True, stream=None):
    loss = C.c_double()
    _mcheck("sr_mlp_train_step", load_library().sr_mlp_train_step(
        net, int(batch), _tptr(idx, "idx", "i64"), _rows(gap, motion, y), _tptr(gap, "gap", "f64"),
        _tptr(motion, "motion", "f64"),
        _tptr(y, "y", "f64"), float(lr), C.byref(loss) if want_loss else None, _stream(stream)))
    return float(loss.value) if want_loss else None


SR_MLP_NPHASES = 4


def sr_mlp_set_profiling(net, on: bool) -> None:
    _mcheck("sr_mlp_set_profiling", load_library().sr_mlp_set_profiling(net, int(bool(on))))


def sr_mlp_get_profile(net):
    """Returns ([ms forward, backward, adam, copies] summed over the profiled steps, steps)."""
    ms = (C.c_double * SR_MLP_NPHASES)()
    n = C.c_int64()
    _mcheck("sr_mlp_get_profile", load_library().sr_mlp_get_profile(net, ms, C.byref(n)))
    return list(ms), int(n.value)


def sr_mlp_gemm_test(a, b, c, passes: int = 3, device: int = 0, stream=None) -> None:
    m, k = a.shape
    n = b.shape[0]
    if b.shape[1] != k or tuple(c.shape) != (m, n):
        raise ValueError("sr_mlp_gemm_test: shapes")
    _mcheck("sr_mlp_gemm_test", load_library().sr_mlp_gemm_test(int(device), int(passes), int(m), int(n), int(k),
                                                                _tptr(a, "a", "f32"), _tptr(b, "b", "f32"),
                                                                _tptr(c, "c", "f32"), _stream(stream)))


def sr_version() -> str:
    return load_library().sr_version().decode()
