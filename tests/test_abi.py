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


def _handle_arrays(path):
    """Arrays of a model file as written by the library (read back with the
    data-only reader)."""
    from paper_2207_12116_amd import instances as I
    m = I.load_model(path)
    return [m.lb, m.ub, m.lin_ptr, m.lin_coef, m.lin_var, m.lin_rhs, m.reif.reshape(-1),
            m.decision, m.objective]


def test_model_file_round_trip_without_device(tmp_path):
    """pccp_model_save_file writes what was built; the data-only reader of
    the generator module reads it back array by array; a file written by the
    generator module loads into the library with the same sizes and saves
    back to the same bytes."""
    import numpy as np
    from paper_2207_12116_amd import instances as I
    for model in (I.rcpsp(30, 2), I.tiny_csp(3), I.jobshop(3, 3, 1),
                  I.jobshop(3, 3, 1, guarded=True)):
        mh = pccp.ModelHandle(model)
        p1 = str(tmp_path / "lib.pccp")
        mh.save(p1)
        got = _handle_arrays(p1)
        want = [model.lb, model.ub, model.lin_ptr, model.lin_coef, model.lin_var,
                model.lin_rhs, np.asarray(model.reif).reshape(-1), model.decision,
                model.objective]
        for a, b in zip(got, want):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        back = I.load_model(p1)
        assert back.ncmd == model.ncmd
        for f in ("cmd", "cmd_gptr", "cmd_guard", "cmd_tptr", "cmd_term"):
            assert np.array_equal(np.asarray(getattr(back, f)).reshape(-1),
                                  np.asarray(getattr(model, f)).reshape(-1)), f
        p2 = str(tmp_path / "gen.pccp")
        I.save_model(model, p2)
        h2 = pccp.ModelHandle.from_file(p2)
        assert h2.info() == dict(nvars=model.nvars, nlinear=model.nrows, nterms=model.nterms,
                                 nreified=model.nreif, ndecision=int(model.decision.shape[0]))
        p3 = str(tmp_path / "again.pccp")
        h2.save(p3)
        with open(p1, "rb") as a, open(p3, "rb") as b:
            assert a.read() == b.read()
        assert I.load_model(p2).content_hash() == model.content_hash()


def test_model_file_errors_without_device(tmp_path):
    import numpy as np
    from paper_2207_12116_amd import instances as I
    L = pccp.lib()
    h = ctypes.c_void_p()
    assert L.pccp_model_load_file(str(tmp_path / "none").encode(), ctypes.byref(h)) == \
        pccp.E_INVALID_ARG
    good = str(tmp_path / "m.pccp")
    I.save_model(I.tiny_rcpsp(5, 1), good)
    data = open(good, "rb").read()
    cases = {"truncated": data[:-4], "extra": data + b"\0\0\0\0",
             "magic": b"PCCP-MODEL 2" + data[12:],
             "header": data.replace(b'"nvars"', b'"nvarz"', 1)}
    for name, blob in cases.items():
        p = str(tmp_path / f"{name}.pccp")
        with open(p, "wb") as f:
            f.write(blob)
        h = ctypes.c_void_p()
        assert L.pccp_model_load_file(p.encode(), ctypes.byref(h)) == pccp.E_MODEL, name
        assert not h.value
    # guarded-command pointers that stop short of their count, or decrease
    for name in ("short", "decreasing"):
        gm = I.jobshop(3, 3, 1, guarded=True)
        gm.cmd_tptr = gm.cmd_tptr.copy()
        if name == "short":
            gm.cmd_tptr[-1] -= 1
        else:
            i = int(np.argmax(np.diff(gm.cmd_tptr) > 0))
            gm.cmd_tptr[i], gm.cmd_tptr[i + 1] = gm.cmd_tptr[i + 1], gm.cmd_tptr[i]
        bad = str(tmp_path / f"cmdptr_{name}.pccp")
        I.save_model(gm, bad)
        h = ctypes.c_void_p()
        assert L.pccp_model_load_file(bad.encode(), ctypes.byref(h)) == pccp.E_MODEL, name
    # a row pointer that decreases
    m = I.tiny_rcpsp(5, 1)
    m.lin_ptr = m.lin_ptr.copy()
    m.lin_ptr[1], m.lin_ptr[2] = m.lin_ptr[2], m.lin_ptr[1]
    bad = str(tmp_path / "ptr.pccp")
    I.save_model(m, bad)
    assert L.pccp_model_load_file(bad.encode(), ctypes.byref(h)) == pccp.E_MODEL


def test_query_and_tuning_errors_without_device():
    """The result queries refuse a missing solver or output pointer before
    touching a device; the tuner refuses bad options the same way."""
    L = pccp.lib()
    assert L.pccp_get_solution_hash(None, None) == pccp.E_INVALID_ARG
    best = pccp.Config()
    assert L.pccp_autotune(None, 1, pccp.MINIMIZE, None, ctypes.byref(best), None, 0, None) == \
        pccp.E_INVALID_ARG
    assert L.pccp_measure_lds_peaks(None) == pccp.E_INVALID_ARG
