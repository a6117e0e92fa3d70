"""The C ABI without a GPU: the library loads, exports every function that
include/mxlu.h declares (and the binding binds exactly those), argument
checks return -k before anything touches a device, status strings exist.
No call here computes; calls with valid arguments happen only where no
device is visible (they must return MXLU_E_NODEV)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mxlu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2604_09517_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2604_09517_amd import build
        build.build()
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lu_factor", "lu_solve", "mxp_solve"):
        assert required in names
    assert len(names) >= 15


def test_library_exports_every_declared_symbol(L):
    from paper_2604_09517_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(L, name)
    # the Python binding binds exactly the declared functions
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_argument_errors_return_minus_k(L):
    p = ctypes.c_void_p(16)   # never dereferenced: every call below fails its checks
    assert L.lu_factor(-1, 64, p, 1, p, None) == -1
    assert L.lu_factor(10, 0, p, 10, p, None) == -2
    assert L.lu_factor(10, 2048, p, 10, p, None) == -2
    assert L.lu_factor(10, 64, None, 10, p, None) == -3
    assert L.lu_factor(10, 64, p, 9, p, None) == -4
    assert L.lu_factor(10, 64, p, 10, None, None) == -5
    assert L.lu_solve(10, -1, p, 10, p, p, 10, 0, None) == -2
    assert L.lu_solve(10, 1, p, 10, p, p, 9, 0, None) == -7
    assert L.lu_solve(10, 1, p, 10, p, p, 10, 3, None) == -8
    assert L.mxlu_schur_update_f64(4, 4, 4, p, 3, p, 4, p, 4, None) == -5
    assert L.mxlu_outer_update_f64(4, 4, 4, p, 4, p, 4, p, 4, 2, None) == -10
    assert L.mxlu_fill_uniform(4, 4, p, 3, 1, 0, None) == -4
    assert L.mxp_convert(7, 4, 4, p, 4, p, 4, None) == -1
    # zero-size problems succeed without touching anything
    assert L.lu_factor(0, 64, None, 1, None, None) == 0
    assert L.lu_solve(5, 0, p, 5, p, None, 5, 0, None) == 0


def test_mxp_options_and_workspace(L):
    from paper_2604_09517_amd import _lib
    o = _lib.MxpOpts()
    L.mxp_default_opts(ctypes.byref(o))
    assert (o.prec, o.pivot, o.nb, o.refine, o.restart) == (0, 0, 512, 1, 30)
    assert o.resid_threshold == 16.0 and o.scale_tile == 128
    ldf = L.mxp_factor_ld(1000)
    assert ldf >= 1000 and ldf % 64 == 0
    assert L.mxp_workspace_bytes(1000, ctypes.byref(o)) >= 2 * ldf * 1000
    assert L.mxp_workspace_bytes(-1, ctypes.byref(o)) == 0
    p = ctypes.c_void_p(16)
    rep = _lib.MxpReport()
    bad = _lib.MxpOpts()
    L.mxp_default_opts(ctypes.byref(bad))
    bad.nb = 48                                    # not a multiple of 32
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -12
    bad.nb = 64
    bad.prec = 2                                   # FP8 needs nb % 128 == 0
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -12
    bad.prec = 0
    bad.pivot = 1                                  # pivoting needs ipiv
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -11
    bad.pivot = 0                                  # workspace too small
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 16, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -1006


def test_status_strings(L):
    for code in (0, -1001, -1002, -1003, -1004, -1005, -1006, -3, 7):
        assert len(L.mxlu_status_string(code)) > 0
    assert L.mxlu_status_string(-1004) == b"iterative refinement did not converge"


def test_no_device_is_reported(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is visible: the no-device path is not reachable")
    p = ctypes.c_void_p(16)   # not dereferenced: the device check comes first
    assert L.lu_factor(8, 4, p, 8, p, None) == -1001
    assert L.lu_solve(8, 1, p, 8, p, p, 8, 0, None) == -1001
    assert b"no HIP device" in L.mxlu_last_error()


def test_python_layer_rejects_bad_tensors():
    import torch
    from paper_2604_09517_amd import api
    with pytest.raises(ValueError):
        api._mat(torch.zeros(4, 4, dtype=torch.float32), "A")
    with pytest.raises(ValueError):
        api._mat(torch.zeros(4, 4, dtype=torch.float64), "A")   # on the CPU
