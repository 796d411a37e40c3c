"""The C-ABI library, and its checked build, load on a machine without a GPU
and export every entry point that include/rbf.h declares (no compute calls
here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(rbf_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("rbf_fit_plan", "rbf_assemble", "rbf_solve", "rbf_eval"):
        assert required in names


@pytest.mark.parametrize("checked", [False, True])
def test_library_exports_every_declared_symbol(checked):
    from paper_1806_07884_amd import _lib
    path = _lib.CHECKED_LIB_PATH if checked else _lib.LIB_PATH
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not built")
    handle = _lib.load(path)
    missing = [n for n in declared_functions() if not hasattr(handle, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(_lib.SIGNATURES)
    assert handle.rbf_build_checked() == int(checked)


def test_status_strings_without_gpu():
    from paper_1806_07884_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librbf.so not built")
    L = _lib.lib()
    assert L.rbf_status_string(0) == b"ok"
    assert b"invalid" in L.rbf_status_string(-1)
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    assert L.rbf_fit_plan(None, None, None, ctypes.byref(out)) == _lib.RBF_ERR_INVALID
    assert b"desc" in L.rbf_last_error()
    d = _lib.PlanDesc(4, 10, 10, 1, 1, 0.1, None, 1, 0.0)
    assert L.rbf_fit_plan(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.RBF_ERR_INVALID
    d = _lib.PlanDesc(2, 10, 10, 1, 1, -0.1, None, 1, 0.0)
    assert L.rbf_fit_plan(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.RBF_ERR_INVALID
    d = _lib.PlanDesc(2, 10, 10, 1, 1, float("inf"), None, 1, 0.0)
    assert L.rbf_fit_plan(ctypes.byref(d), None, None, ctypes.byref(out)) == _lib.RBF_ERR_NONFINITE
    assert out.value is None


def test_stream_argument_validation_without_gpu():
    # rbf_stream_begin / rbf_stream_add / rbf_stream_finish reject bad
    # arguments before any device call
    from paper_1806_07884_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librbf.so not built")
    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.rbf_stream_begin(None, None, None, ctypes.byref(out)) == _lib.RBF_ERR_INVALID
    assert b"desc" in L.rbf_last_error()
    good = dict(dim=2, n_centers=10, centers=1, rho=0.1, rho_per_center=None, min_support=1,
                lambda_rel=0.0, phi=1, precision=1, max_chunk=100, flags=0)
    bad = [dict(dim=4), dict(n_centers=0), dict(centers=None), dict(rho=-1.0),
           dict(min_support=0), dict(lambda_rel=-1.0), dict(phi=7), dict(precision=3),
           dict(max_chunk=0), dict(max_chunk=1 << 31), dict(flags=8)]
    for change in bad:
        d = _lib.StreamDesc(**{**good, **change})
        assert L.rbf_stream_begin(ctypes.byref(d), None, None, ctypes.byref(out)) \
            == _lib.RBF_ERR_INVALID, change
        assert out.value is None
    d = _lib.StreamDesc(**{**good, "rho": float("nan")})
    assert L.rbf_stream_begin(ctypes.byref(d), None, None, ctypes.byref(out)) \
        in (_lib.RBF_ERR_INVALID, _lib.RBF_ERR_NONFINITE)
    assert L.rbf_stream_add(None, 1, None, None, 0) == _lib.RBF_ERR_INVALID
    assert L.rbf_stream_finish(None) == _lib.RBF_ERR_INVALID
