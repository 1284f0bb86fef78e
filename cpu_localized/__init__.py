"""Paper-style localized CPU evaluation (far pairs once, near pairs at three smoothing lengths, OpenMP
over targets): a timing baseline for the benchmark.  It is not a checker: the tests compare the GPU path
with the oracle only.  build() compiles localized.c with gcc -O2 -fopenmp (the paper's level)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "localized.c")
LIB = os.path.join(HERE, "liblocalized.so")
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built: run __graft_entry__.build()")
        L = C.CDLL(LIB)
        vp = C.c_void_p
        L.loc_eval.argtypes = [C.c_int64, vp, vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_double, vp,
                               C.c_double, vp, vp]
        L.loc_eval.restype = None
        L.loc_num_threads.restype = C.c_int
        L.loc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def evaluate(cfg, idx=None):
    """Both layers at the targets idx (default all) of a workload dict; returns (u, v)."""
    s, t = cfg["surf"], cfg["targets"]
    sel = slice(None) if idx is None else np.asarray(idx)
    arrs = [_c(a) for a in (s.x, s.normal, s.w, cfg["f"], cfg["q"], t.y[sel], t.x0[sel], t.n0[sel], t.b[sel],
                            cfg["f0"][sel], cfg["q0"][sel])]
    m = arrs[5].shape[0]
    u, v = np.empty((m, 3)), np.empty((m, 3))
    rho = _c(cfg["rho"])
    p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    lib().loc_eval(arrs[0].shape[0], p(arrs[0]), p(arrs[1]), p(arrs[2]), p(arrs[3]), p(arrs[4]), m, p(arrs[5]),
                   p(arrs[6]), p(arrs[7]), p(arrs[8]), p(arrs[9]), p(arrs[10]), float(cfg["h"]), p(rho), 6.0,
                   p(u), p(v))
    return u, v


def num_threads() -> int:
    return int(lib().loc_num_threads())


def set_num_threads(n: int) -> None:
    lib().loc_set_num_threads(int(n))
