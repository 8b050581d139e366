"""C-ABI contract checks that run without a GPU: the library loads, exports
every symbol the header declares, and reports the documented errors."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tn.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tn_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for f in ("tn_create", "tn_destroy", "tn_boundary_contract", "tn_environments", "tn_sample",
              "tn_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_2507_11424_amd as tnb
    if not os.path.exists(tnb.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(tnb.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(tnb.EXPORTS) == _declared()


def test_create_without_gpu_reports_hip_error():
    import paper_2507_11424_amd as tnb
    import torch
    if not os.path.exists(tnb.LIB_PATH):
        pytest.skip("library not built")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = tnb.lib()
    h = ctypes.c_void_p()
    assert L.tn_create(ctypes.byref(h), 0, None) == 4  # TN_ERR_HIP
    assert L.tn_destroy(None) == 1  # TN_ERR_INVALID
    assert L.tn_last_error(None) == b"null handle"


def test_default_opts():
    import paper_2507_11424_amd as tnb
    if not os.path.exists(tnb.LIB_PATH):
        pytest.skip("library not built")
    o = tnb.make_opts(chi=64, chi_x=32, prec="bf16x3")
    assert (o.chi, o.chi_x, o.sweeps, o.direction, o.init, o.prec) == (64, 32, 2, 0, 0, 2)


def test_binding_fails_loudly_without_gpu():
    import paper_2507_11424_amd as tnb
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        tnb.Handle(0)


def _declared_arity():
    """Parameter count of every function the header declares (top-level commas
    of its parameter list; comments stripped)."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(tn_[a-z_]+)\s*\(([^;{]*?)\)\s*;", txt):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argtypes_match_the_header():
    """The ctypes binding declares every call with the header's parameter
    count, so a changed signature cannot go unnoticed."""
    import paper_2507_11424_amd as tnb
    if not os.path.exists(tnb.LIB_PATH):
        pytest.skip("library not built")
    L = tnb.lib()
    arity = _declared_arity()
    assert set(arity) == set(_declared())
    for name, n in arity.items():
        at = getattr(L, name).argtypes
        assert at is not None and len(at) == n, (name, n, at)
