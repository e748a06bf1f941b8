"""Host-side checks of the C ABI that need no GPU: the library builds, loads,
exports every entry point declared in include/esi.h, and rejects bad arguments
with a status code and a message before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esi.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2211_06300_amd import esi
    if not os.path.exists(esi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return esi.load_library()


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:esi_status_t|const char\*|int64_t)\s+(esi_\w+)\(", text, re.M)))


def test_header_declares_the_calls():
    names = declared()
    for n in ["esi_forward", "esi_adjoint", "esi_normal_apply", "esi_cg_solve", "esi_gradient",
              "esi_plan_create", "esi_plan_destroy", "esi_last_error"]:
        assert n in names


def test_exports_every_declared_symbol(lib):
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_2211_06300_amd import esi
    assert sorted(esi.EXPORTS) == declared()


def test_null_arguments_rejected(lib):
    vp = ctypes.c_void_p
    assert lib.esi_plan_create(None, None, None, None, None) == 1
    assert b"null" in lib.esi_last_error()
    assert lib.esi_forward(None, 0, 1, 0, None, None) == 1
    assert lib.esi_adjoint(None, 0, 1, None, None) == 1
    assert lib.esi_normal_apply(None, 0, 1, None, None, None) == 1
    assert lib.esi_cg_solve(None, 0, 1, None, None, None, 5, 0.0, None) == 1
    assert lib.esi_gradient(None, 0, 1, 0, 1, None, None, None, None, 0) == 1
    for setter, value in (("esi_plan_set_cg_rfuse", 1), ("esi_plan_set_dtft_block", 64),
                          ("esi_plan_set_ds_ckpt", 50)):
        assert getattr(lib, setter)(None, value) == 1, setter
        assert b"null plan" in lib.esi_last_error(), setter
    assert lib.esi_plan_destroy(None) == 0


def test_grid_validation_before_device(lib):
    from paper_2211_06300_amd.esi import _Grid, _Geom
    import numpy as np
    src = np.zeros((1, 2), dtype=np.int32)
    ptr = np.zeros(2, dtype=np.int64)
    geo = _Geom(1, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)      # never dereferenced: validation fails first
    cases = [
        (_Grid(4, 10, 10, 1, 8, 10, 10.0, 1e-3, -1.0, 0.0, 1.0), 1, b"ndim"),
        (_Grid(2, 10, 10, 2, 8, 10, 10.0, 1e-3, -1.0, 0.0, 1.0), 2, b"ny"),
        (_Grid(2, 10, 10, 1, 2, 10, 10.0, 1e-3, -1.0, 0.0, 1.0), 2, b"nb"),
        (_Grid(2, 10, 10, 1, 8, 0, 10.0, 1e-3, -1.0, 0.0, 1.0), 2, b"nt"),
        (_Grid(2, 10, 10, 1, 8, 10, -1.0, 1e-3, -1.0, 0.0, 1.0), 1, b"dx"),
        (_Grid(2, 10, 10, 1, 8, 10, 10.0, 1e-3, -1.0, 0.1, 0.0), 1, b"b_eps"),
    ]
    for g, code, msg in cases:
        assert lib.esi_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(geo), fake, None) == code
        assert msg in lib.esi_last_error()
    src_bad = np.array([[10, 0]], dtype=np.int32)
    geo_bad = _Geom(1, src_bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None)
    g = _Grid(2, 10, 10, 1, 8, 10, 10.0, 1e-3, -1.0, 0.0, 1.0)
    assert lib.esi_plan_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(geo_bad), fake, None) == 2
    assert b"outside" in lib.esi_last_error()


def test_product_path_does_not_import_oracle():
    """The GPU package never reaches into the oracle (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2211_06300_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from\s+oracle|import\s+oracle)|liboracle", text, re.M), f
