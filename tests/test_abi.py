"""Host-side checks of the C-ABI library (no device computation)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tn3d.h")
LIB = os.path.join(ROOT, "paper_2310_10722_amd", "libtn3d.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tn3d_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2310_10722_amd import build
        build.build()
    return LIB


def test_library_exports_every_declared_symbol(lib_path):
    from paper_2310_10722_amd import tn3d
    names = declared()
    assert len(names) >= 15
    assert set(names) == set(tn3d.SYMBOLS)
    assert set(tn3d.exported_symbols(lib_path)) == set(names)


def test_params_defaults(lib_path):
    from paper_2310_10722_amd import tn3d
    p = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP32)
    assert (p.chi, p.chi_mps, p.precision) == (16, 16, 1)
    assert p.eps_rel == 1e-6 and p.tau_gap == 1e-2 and p.flags == 0
    p = tn3d.tn3d_params_default(4, 8, tn3d.PREC_FP64)
    assert p.eps_rel == 1e-9 and p.tau_gap == 1e-6 and p.chi_mps == 8


def test_context_rejects_missing_device(lib_path):
    import ctypes
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2310_10722_amd import tn3d
    lib = tn3d.load_library()
    h = ctypes.c_void_p()
    assert lib.tn3d_ctx_create(0, None, ctypes.byref(h)) == -1
    assert lib.tn3d_last_error(None) == b"null context"
