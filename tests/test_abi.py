"""The C-ABI library loads on any host and exports every function that
include/pccp.h declares (no device call is made here)."""
import ctypes
import os
import re

from paper_2207_12116_amd import pccp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "pccp.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pccp_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(pccp.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pccp.EXPORTS) == names


def test_version_and_error_text():
    assert "pccp" in pccp.version()
    L = pccp.lib()
    assert L.pccp_model_create(None) == pccp.E_INVALID_ARG
    assert b"NULL" in L.pccp_last_error()


def test_model_building_errors_without_device():
    L = pccp.lib()
    h = ctypes.c_void_p()
    assert L.pccp_model_create(ctypes.byref(h)) == 0
    lb = (ctypes.c_int32 * 2)(0, 0)
    ub = (ctypes.c_int32 * 2)(5, 5)
    assert L.pccp_model_add_vars(h, 2, lb, ub, None) == 0
    coef = (ctypes.c_int32 * 1)(1)
    var = (ctypes.c_int32 * 1)(0)
    assert L.pccp_model_add_linear_le(h, 0, coef, var, 3) == pccp.E_INVALID_ARG
    assert L.pccp_model_add_linear_le(h, 1, coef, var, 3) == 0
    n = ctypes.c_int32(0)
    assert L.pccp_model_info(h, ctypes.byref(n), None, None, None, None) == 0 and n.value == 2
    assert L.pccp_model_destroy(h) == 0


def test_config_validation_without_device():
    """Invalid launch configurations are refused before any device call:
    item lists together with dependency-driven propagation, out-of-range
    mode fields, a negative trail capacity, the high-occupancy build with
    more than 256 threads."""
    from paper_2207_12116_amd import instances as I
    L = pccp.lib()
    mh = pccp.ModelHandle(I.tiny_rcpsp(4, 0))
    bad = [dict(live=1, dep=1), dict(dep=3), dict(live=-1), dict(trail_cap=-1),
           dict(occupancy=1, wg_size=512), dict(wg_size=96)]
    for kw in bad:
        cfg = pccp.Config(**kw)
        h = ctypes.c_void_p()
        rc = L.pccp_solver_create(mh.h, ctypes.byref(cfg), None, ctypes.byref(h))
        assert rc == pccp.E_INVALID_ARG, (kw, rc)
        assert not h.value
