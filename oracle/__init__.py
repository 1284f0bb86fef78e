"""Plain FP64 CPU oracle of the extrapolated-regularization Stokes sums (paper §2).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by bench.py's CPU
baseline.  The GPU library neither imports nor links it, and it shares no code with it.

The arithmetic lives in stokes_oracle.c (literal sums over all quadrature points for each delta,
then the 3x3 extrapolation solve); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        d = C.POINTER(C.c_double)
        i64 = C.c_int64
        L.orc_smoothing.argtypes = [C.c_double, d]
        L.orc_smoothing_sharp.argtypes = [C.c_double, d]
        L.orc_sl_sharp.argtypes = [i64, d, d, d, d, i64, d, d, d, C.c_double, d]
        L.orc_dl_sharp.argtypes = [i64, d, d, d, d, i64, d, d, d, C.c_double, d]
        L.orc_I0.argtypes = [C.c_double]
        L.orc_I0.restype = C.c_double
        L.orc_I2.argtypes = [C.c_double]
        L.orc_I2.restype = C.c_double
        L.orc_extrapolate.argtypes = [C.c_double, C.c_double, d, d, d]
        L.orc_sl_delta.argtypes = [i64, d, d, d, d, i64, d, d, d, C.c_double, d]
        L.orc_dl_delta.argtypes = [i64, d, d, d, d, i64, d, d, d, d, d, C.c_double, d]
        L.orc_sl.argtypes = [i64, d, d, d, d, i64, d, d, d, d, d, C.c_double, d, d, d, d]
        L.orc_dl.argtypes = [i64, d, d, d, d, i64, d, d, d, d, d, C.c_double, d, d, d, d]
        L.orc_plain.argtypes = [i64, d, d, d, d, d, i64, d, d, d]
        L.orc_tree.argtypes = [i64, d, d, d, d, d, i64, d, d, d, d, d, d, C.c_double, d, C.c_int, C.c_double, i64,
                               C.c_double, d, d, d, d]
        L.orc_tree.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def smoothing(t: float) -> np.ndarray:
    s = np.zeros(3)
    lib().orc_smoothing(float(t), _p(s))
    return s


def smoothing_sharp(t: float) -> np.ndarray:
    s = np.zeros(3)
    lib().orc_smoothing_sharp(float(t), _p(s))
    return s


def sl_sharp(surf_x, surf_n, surf_w, f, y, n0, f0, delta):
    """On-surface single layer with s1#, s2# at one delta (targets on the surface)."""
    x, nn, w, f = _f64(surf_x), _f64(surf_n), _f64(surf_w), _f64(f)
    y, n0, f0 = _f64(y), _f64(n0), _f64(f0)
    out = np.zeros((y.shape[0], 3))
    lib().orc_sl_sharp(x.shape[0], _p(x), _p(nn), _p(w), _p(f), y.shape[0], _p(y), _p(n0), _p(f0), float(delta),
                       _p(out))
    return out


def dl_sharp(surf_x, surf_n, surf_w, q, y, n0, q0, delta):
    """On-surface double layer with s2#, s3# at one delta, plus q(y)/2 (targets on the surface)."""
    x, nn, w, q = _f64(surf_x), _f64(surf_n), _f64(surf_w), _f64(q)
    y, n0, q0 = _f64(y), _f64(n0), _f64(q0)
    out = np.zeros((y.shape[0], 3))
    lib().orc_dl_sharp(x.shape[0], _p(x), _p(nn), _p(w), _p(q), y.shape[0], _p(y), _p(n0), _p(q0), float(delta),
                       _p(out))
    return out


def I0(lam: float) -> float:
    return lib().orc_I0(float(lam))


def I2(lam: float) -> float:
    return lib().orc_I2(float(lam))


def extrapolate(b: float, h: float, rho, ud) -> np.ndarray:
    """ud: (3 deltas, 3 components) -> extrapolated (3,)."""
    r = _f64(rho, (3,))
    u = _f64(ud, (9,))
    out = np.zeros(3)
    rc = lib().orc_extrapolate(float(b), float(h), _p(r), _p(u), _p(out))
    if rc != 0:
        raise FloatingPointError("singular extrapolation system")
    return out


def extrapolation_weights(b: float, h: float, rho) -> np.ndarray:
    """w_j with u = sum_j w_j u^{delta_j} (the extrapolation is linear in the three values)."""
    w = np.zeros(3)
    for j in range(3):
        ud = np.zeros((3, 3))
        ud[j, 0] = 1.0
        w[j] = extrapolate(b, h, rho, ud)[0]
    return w


def sl_delta(surf_x, surf_n, surf_w, f, y, n0, f0, delta):
    x, nn, w, f = _f64(surf_x), _f64(surf_n), _f64(surf_w), _f64(f)
    y, n0, f0 = _f64(y), _f64(n0), _f64(f0)
    out = np.zeros((y.shape[0], 3))
    lib().orc_sl_delta(x.shape[0], _p(x), _p(nn), _p(w), _p(f), y.shape[0], _p(y), _p(n0), _p(f0),
                       float(delta), _p(out))
    return out


def dl_delta(surf_x, surf_n, surf_w, q, y, x0, n0, b, q0, delta):
    x, nn, w, q = _f64(surf_x), _f64(surf_n), _f64(surf_w), _f64(q)
    y, x0, n0, b, q0 = _f64(y), _f64(x0), _f64(n0), _f64(b), _f64(q0)
    out = np.zeros((y.shape[0], 3))
    lib().orc_dl_delta(x.shape[0], _p(x), _p(nn), _p(w), _p(q), y.shape[0], _p(y), _p(x0), _p(n0), _p(b),
                       _p(q0), float(delta), _p(out))
    return out


def _eval(fn, surf_x, surf_n, surf_w, dens, y, x0, n0, b, dens0, h, rho, want_delta):
    x, nn, w, dd = _f64(surf_x), _f64(surf_n), _f64(surf_w), _f64(dens)
    y, x0, n0, b, d0 = _f64(y), _f64(x0), _f64(n0), _f64(b), _f64(dens0)
    m = y.shape[0]
    r = _f64(rho, (3,))
    out = np.zeros((m, 3))
    od = np.zeros((m, 3, 3)) if want_delta else None
    scratch = np.zeros(9 * max(m, 1))
    rc = fn(x.shape[0], _p(x), _p(nn), _p(w), _p(dd), m, _p(y), _p(x0), _p(n0), _p(b), _p(d0), float(h),
            _p(r), _p(out), _p(od) if od is not None else None, _p(scratch))
    if rc != 0:
        raise FloatingPointError("singular extrapolation system")
    return (out, od) if want_delta else out


def sl(surf_x, surf_n, surf_w, f, y, x0, n0, b, f0, h, rho, want_delta=False):
    """Extrapolated single layer u (m,3) [and the regularized values (m, 3 deltas, 3)]."""
    return _eval(lib().orc_sl, surf_x, surf_n, surf_w, f, y, x0, n0, b, f0, h, rho, want_delta)


def dl(surf_x, surf_n, surf_w, q, y, x0, n0, b, q0, h, rho, want_delta=False):
    """Extrapolated double layer v (m,3) including chi q(x0) [and the regularized values]."""
    return _eval(lib().orc_dl, surf_x, surf_n, surf_w, q, y, x0, n0, b, q0, h, rho, want_delta)


def plain(surf_x, surf_n, surf_w, f, q, y):
    """Unregularized, unsubtracted sums (for targets far from the surface)."""
    x, nn, w, f, q, y = (_f64(a) for a in (surf_x, surf_n, surf_w, f, q, y))
    m = y.shape[0]
    us, ud = np.zeros((m, 3)), np.zeros((m, 3))
    lib().orc_plain(x.shape[0], _p(x), _p(nn), _p(w), _p(f), _p(q), m, _p(y), _p(us), _p(ud))
    return us, ud


def tree(surf_x, surf_n, surf_w, f, q, y, x0, n0, b, f0, q0, h, rho, p=8, theta=0.7, leaf=2000,
         want_delta=False, mac_rnear=None):
    """Treecode evaluation of both layers (paper section 3.4); returns (u, v[, ud, vd, nnodes]).
    mac_rnear: the radius the MAC requires a cluster's box to lie beyond (default: the near radius)."""
    x, nn, w, f, q = (_f64(a) for a in (surf_x, surf_n, surf_w, f, q))
    y, x0, n0, b, f0, q0 = (_f64(a) for a in (y, x0, n0, b, f0, q0))
    m = y.shape[0]
    r = _f64(rho, (3,))
    u, v = np.zeros((m, 3)), np.zeros((m, 3))
    ud = np.zeros((m, 3, 3)) if want_delta else None
    vd = np.zeros((m, 3, 3)) if want_delta else None
    nn_ = lib().orc_tree(x.shape[0], _p(x), _p(nn), _p(w), _p(f), _p(q), m, _p(y), _p(x0), _p(n0), _p(b), _p(f0),
                         _p(q0), float(h), _p(r), int(p), float(theta), int(leaf),
                         float(mac_rnear) if mac_rnear is not None else 0.0, _p(u), _p(v),
                         _p(ud) if ud is not None else None, _p(vd) if vd is not None else None)
    if nn_ < 0:
        raise FloatingPointError("singular extrapolation system")
    return (u, v, ud, vd, nn_) if want_delta else (u, v)


def tree_cfg(cfg, idx=None, p=8, theta=0.7, leaf=2000, want_delta=False, mac_rnear=None):
    s, t = cfg["surf"], cfg["targets"]
    sel = slice(None) if idx is None else np.asarray(idx)
    return tree(s.x, s.normal, s.w, cfg["f"], cfg["q"], t.y[sel], t.x0[sel], t.n0[sel], t.b[sel], cfg["f0"][sel],
                cfg["q0"][sel], cfg["h"], cfg["rho"], p, theta, leaf, want_delta, mac_rnear)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def sl_cfg(cfg, idx=None, want_delta=False):
    """Convenience: single layer for a workload dict from workload.build_config (optional target subset)."""
    s, t = cfg["surf"], cfg["targets"]
    sel = slice(None) if idx is None else np.asarray(idx)
    return sl(s.x, s.normal, s.w, cfg["f"], t.y[sel], t.x0[sel], t.n0[sel], t.b[sel], cfg["f0"][sel],
              cfg["h"], cfg["rho"], want_delta)


def dl_cfg(cfg, idx=None, want_delta=False):
    s, t = cfg["surf"], cfg["targets"]
    sel = slice(None) if idx is None else np.asarray(idx)
    return dl(s.x, s.normal, s.w, cfg["q"], t.y[sel], t.x0[sel], t.n0[sel], t.b[sel], cfg["q0"][sel],
              cfg["h"], cfg["rho"], want_delta)
