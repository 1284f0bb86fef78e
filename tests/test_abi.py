"""The C-ABI library builds, loads and exports every entry point that include/stokesreg.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

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
