"""The C-ABI library builds, loads and exports every entry point that include/stokesreg.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2507_00156_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokesreg.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert sorted(P.EXPORTS) == declared_symbols()


def test_library_exports_all_declared_symbols():
    lib = P.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert P.sr_version().startswith("stokesreg")


def test_default_params():
    p = P.sr_default_params()
    assert tuple(p.rho) == (2.0, 3.0, 4.0) and p.cutoff == 6.0 and p.precision == P.SR_FP64
    assert p.tree_degree == 8 and abs(p.tree_theta - 0.7) < 1e-15 and p.tree_leaf == 2000


def test_create_without_gpu_reports_enodev():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.SrError) as ei:
        P.sr_create(0)
    assert ei.value.status == -3


def test_null_arguments_rejected():
    lib = P.load_library()
    assert lib.sr_create(None, 0) == -1
    assert lib.sr_set_params(None, None) == -1
    assert lib.sr_eval(None, 1, 0, *([None] * 11)) == -1
    assert lib.sr_destroy(None) == 0


def test_target_count_cap_checked_before_anything_else():
    """The evaluation entry points reject m > 2^28 (the kernels index 3 t + component in 32 bits) before
    they look at the context, so the cap is testable without a GPU."""
    lib = P.load_library()
    cap = P.sr_max_targets()
    assert cap == 1 << 28 and 3 * cap < 2 ** 31
    nul = [None] * 11
    assert lib.sr_eval(None, P.SR_SL, cap + 1, *nul) == P.binding.SR_EINVAL
    assert "out of range" in lib.sr_last_error().decode()
    assert lib.sr_eval(None, P.SR_SL, -1, *nul) == P.binding.SR_EINVAL
    assert "out of range" in lib.sr_last_error().decode()
    assert lib.sr_eval(None, P.SR_SL, cap, *nul) == P.binding.SR_EINVAL
    assert "ctx is NULL" in lib.sr_last_error().decode()
    assert lib.sr_eval(None, P.SR_SL | P.SR_HOST, cap + 1, *nul) == P.binding.SR_EINVAL
    assert "out of range" in lib.sr_last_error().decode()
    assert lib.sr_eval_far(None, P.SR_DL, cap + 1, None, None, None, None) == P.binding.SR_EINVAL
    assert "out of range" in lib.sr_last_error().decode()
    assert lib.sr_eval_far(None, 4, 1, None, None, None, None) == P.binding.SR_EINVAL
    assert "layers" in lib.sr_last_error().decode()
    assert lib.sr_check(None, None) == P.binding.SR_EINVAL


def test_single_precision_cell_margin_bound():
    """The cell side on the mixed path is rnear (1 + 1e-5) + 4 2^-24 (2 E + rnear), E the largest
    |x_d - org_d| of the points: every pair whose single-precision squared distance (coordinates rounded
    relative to org, then the same fma chain as the kernels) is <= rnear^2 must be truly closer than that
    side, whatever the extent.  Checked on pairs placed just outside rnear at extents up to 1e4 rnear."""
    rng = np.random.default_rng(5)
    for extent in (1.0, 30.0, 1e3, 1e4):
        rnear = 1.0
        org = rng.uniform(-5 * extent, 5 * extent, 3)
        x = org + rng.uniform(-extent, extent, (200000, 3))
        d = rng.standard_normal((200000, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        y = x + d * rnear * rng.uniform(0.999, 1.001 + 8e-7 * extent, (200000, 1))
        E = np.abs(x - org).max()
        side = rnear * (1 + 1e-5) + 4 * 2.0 ** -24 * (2 * E + rnear)
        xs = (x - org).astype(np.float32)
        ys = (y - org).astype(np.float32)
        dd = ys - xs
        r2 = np.float32(dd[:, 0] * dd[:, 0])
        r2 = (dd[:, 1].astype(np.float64) * dd[:, 1] + r2).astype(np.float32)
        r2 = (dd[:, 2].astype(np.float64) * dd[:, 2] + r2).astype(np.float32)
        near = r2 <= np.float32(rnear * rnear)
        true_r = np.linalg.norm(y - x, axis=1)
        assert near.any()
        assert (true_r[near] <= side).all(), (extent, true_r[near].max(), side)


def test_noalloc_target_limit_checked_before_anything_else():
    """sr_eval_noalloc rejects m above its static scratch capacity, host arrays (SR_HOST) and bad layers
    before it looks at the context."""
    lib = P.load_library()
    cap = P.binding.SR_NOALLOC_MAX_TARGETS
    nul = [None] * 9
    assert lib.sr_eval_noalloc(None, P.SR_SL, cap + 1, *nul) == P.binding.SR_EINVAL
    assert "out of range" in lib.sr_last_error().decode()
    assert lib.sr_eval_noalloc(None, P.SR_SL | P.SR_HOST, 1, *nul) == P.binding.SR_EINVAL
    assert "layers" in lib.sr_last_error().decode()
    assert lib.sr_eval_noalloc(None, P.SR_DL, cap, *nul) == P.binding.SR_EINVAL
    assert "ctx is NULL" in lib.sr_last_error().decode()
    # the header's figures agree with the binding's
    text = open(HEADER).read()
    assert f"#define SR_NOALLOC_MAX_TARGETS {cap}" in text
