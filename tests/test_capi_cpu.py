"""CPU checks of the C ABI: the library loads, exports every entry point that
include/xy.h declares, and rejects invalid configurations without touching
a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1211_0780_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "xy.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(xy_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_four_verbs():
    names = declared_functions()
    for v in ("xy_init", "xy_sweep", "xy_measure", "xy_exchange"):
        assert v in names


def test_library_exports_every_declared_symbol(xylib):
    for name in declared_functions():
        assert hasattr(xylib, name), name
    # and the binding's list is a subset of the header's
    assert set(C.EXPORTS) <= set(declared_functions())


def test_library_exports_no_undeclared_c_symbol(xylib):
    """Every C-linkage function the library exports is declared in the header
    (internal helpers have internal linkage; C++ symbols are mangled)."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", xylib._name], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[1] in "TtWw"}
    c_funcs = {n for n in exported if not n.startswith("_Z")}
    assert c_funcs <= set(declared_functions()), sorted(c_funcs - set(declared_functions()))


def _cfg(L, R, beta, prec=C.XY_FP32, start=C.XY_START_RANDOM):
    cfg = C.XYConfig()
    Ls = (ctypes.c_int32 * len(L))(*L)
    Rs = (ctypes.c_int32 * len(R))(*R)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    cfg.n_lattices = len(L)
    cfg.L = Ls
    cfg.n_replicas = Rs
    cfg.beta = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.prec = prec
    cfg.start = start
    cfg._keep = (Ls, Rs, b)
    return cfg


def _init_status(cfg):
    ctx = ctypes.c_void_p(123)
    st = C.lib().xy_init(ctypes.byref(cfg), ctypes.byref(ctx))
    return st, ctx.value, C.lib().xy_last_error(None).decode()


@pytest.mark.parametrize("L", [7, 2, 0, -4, 1026])
def test_rejects_bad_L(xylib, L):
    st, ctx, msg = _init_status(_cfg([L], [1], [0.4]))
    assert st == C.XY_ERR_ODD_L and ctx is None and "L" in msg


def test_rejects_bad_ladders(xylib):
    assert _init_status(_cfg([8], [3], [0.4, 0.4, 0.5]))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8], [2], [0.5, 0.4]))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8], [2], [0.4, np.nan]))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8], [2], [-0.1, 0.4]))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8], [0], [0.4]))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8, 6], [2, 2], [0.1, 0.2, 0.3, 0.3]))[0] == C.XY_ERR_ARG


def test_rejects_bad_enums_and_nulls(xylib):
    assert _init_status(_cfg([8], [1], [0.4], prec=7))[0] == C.XY_ERR_ARG
    assert _init_status(_cfg([8], [1], [0.4], start=5))[0] == C.XY_ERR_ARG
    cfg = _cfg([8], [1], [0.4])
    cfg.beta = None
    assert _init_status(cfg)[0] == C.XY_ERR_ARG
    assert xylib.xy_init(None, ctypes.byref(ctypes.c_void_p())) == C.XY_ERR_ARG
    assert xylib.xy_init(ctypes.byref(_cfg([8], [1], [0.4])), None) == C.XY_ERR_ARG


def test_null_context_calls_fail_cleanly(xylib):
    assert xylib.xy_sweep(None, 1, 1) == C.XY_ERR_ARG
    assert xylib.xy_measure(None, None, 0) == C.XY_ERR_ARG
    assert xylib.xy_exchange(None, None) == C.XY_ERR_ARG
    assert xylib.xy_run(None, 1, 1, 1, 1, None) == C.XY_ERR_ARG
    xylib.xy_destroy(None)


def test_every_context_entry_point_rejects_a_null_context(xylib):
    """Every entry point whose first argument is the context returns
    XY_ERR_ARG for NULL, whatever the other arguments are."""
    skip = {"xy_angles_bytes", "xy_init", "xy_last_error", "xy_destroy"}
    checked = 0
    for name in C.EXPORTS:
        if name in skip:
            continue
        fn = getattr(xylib, name)
        nargs = len(fn.argtypes)
        args = [None] + [None if t in (ctypes.c_void_p,) or hasattr(t, "contents") or t is ctypes.c_char_p
                         else 0 for t in fn.argtypes[1:]]
        assert len(args) == nargs
        assert fn(*args) == C.XY_ERR_ARG, name
        checked += 1
    assert checked == len(C.EXPORTS) - len(skip)


def test_angle_bytes(xylib):
    assert xylib.xy_angles_bytes(ctypes.byref(_cfg([8], [3], [0.1, 0.2, 0.3]))) == 3 * 512 * 4
    assert xylib.xy_angles_bytes(ctypes.byref(_cfg([8, 4], [1, 2], [0.1, 0.2, 0.3],
                                                   prec=C.XY_FP64))) == (512 + 2 * 64) * 8
    assert xylib.xy_angles_bytes(ctypes.byref(_cfg([9], [1], [0.1]))) == 0


def test_valid_config_without_gpu_reports_hip_error(xylib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, ctx, msg = _init_status(_cfg([8], [2], [0.1, 0.2]))
    assert st == C.XY_ERR_HIP and ctx is None and msg
