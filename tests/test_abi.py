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
    assert o.factor_steps == 0
    assert L.mxp_workspace_bytes(1000, 1000, ctypes.byref(o)) >= 2 * ldf * 1000
    assert L.mxp_workspace_bytes(1000, 1004, ctypes.byref(o)) >= 2 * ldf * 1000
    assert L.mxp_workspace_bytes(-1, 1, ctypes.byref(o)) == 0
    assert L.mxp_workspace_bytes(1000, 999, ctypes.byref(o)) == 0     # lda < n
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
    bad.pivot = 0
    bad.factor_steps = -1                          # negative step count
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -12
    bad.factor_steps = 0                           # workspace too small
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 16, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -1006
    bad.prec = 5                                   # no such precision
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -12
    bad.prec = 4                                   # FP32 storage: forward solves only
    bad.trans = 1
    assert L.mxp_solve(64, 1, p, 64, p, 64, p, 64, p, 1 << 20, None, ctypes.byref(bad),
                       ctypes.byref(rep), None) == -12
    bad.trans = 0
    # FP32 storage holds 4 bytes per factor value
    assert L.mxp_workspace_bytes(1000, 1000, ctypes.byref(bad)) >= 4 * ldf * 1000
    assert L.mxp_convert(4, 8, 8, p, 8, p, 8, None) == -1   # not a 16-bit format


def test_seeded_solve_argument_checks(L):
    from paper_2604_09517_amd import _lib
    o = _lib.MxpOpts()
    L.mxp_default_opts(ctypes.byref(o))
    rep = _lib.MxpReport()
    p = ctypes.c_void_p(16)   # never dereferenced: every call below fails its checks
    args = lambda n, dom, ldb, opts: (n, 1, 0, dom, 1, p, ldb, p, n, p, 1 << 30, None, opts,
                                      ctypes.byref(rep), None)
    assert L.mxp_solve_seeded(*args(-1, 1, 10, ctypes.byref(o))) == -1
    assert L.mxp_solve_seeded(*args(10, 2, 10, ctypes.byref(o))) == -4
    assert L.mxp_solve_seeded(*args(10, 1, 9, ctypes.byref(o))) == -7
    assert L.mxp_solve_seeded(*args(10, 1, 10, None)) == -13
    bad = _lib.MxpOpts()
    L.mxp_default_opts(ctypes.byref(bad))
    bad.pivot = 1                                  # pivoting needs ipiv
    assert L.mxp_solve_seeded(*args(10, 0, 10, ctypes.byref(bad))) == -12


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


# ------------------------------------------------------- planning (host only)
LDS_BUDGET = 160 * 1024 - 4096     # dynamic LDS of the LDS-form leaf, about


def plan_leaf(L, m, cap, cus=256, occ1=2, occ2=2, budget=LDS_BUDGET, elem=8):
    R, G = ctypes.c_int64(0), ctypes.c_int64(0)
    form = L.mxlu_plan_panel_leaf(m, cap, cus, occ1, occ2, budget, elem, ctypes.byref(R),
                                  ctypes.byref(G))
    return form, R.value, G.value


def test_panel_cus_even_split_only(L):
    """The look-ahead's panel stream gets a quarter of the CUs only when that
    is an equal number per shader engine (a multiple of 32 on an 8-XCD,
    4-engine-per-XCD part): 256 CUs -> 64; the uneven 48-of-192 and 76-of-304
    splits are refused (no look-ahead)."""
    assert L.mxlu_plan_panel_cus(256) == 64
    assert L.mxlu_plan_panel_cus(128) == 32
    for cus in (192, 304, 240, 100, 0, -1, 2048):
        assert L.mxlu_plan_panel_cus(cus) == 0, cus


def test_leaf_planner_forms_and_residency(L):
    # register form, one row per thread, while groups fit two per CU
    assert plan_leaf(L, 32768, 0) == (1, 256, 128)
    assert plan_leaf(L, 65536, 0) == (1, 256, 256)
    # beyond kMaxGroups (256) groups: two rows per thread
    assert plan_leaf(L, 65537, 0)[:2] == (2, 512)
    # a cap of 56 CUs (7/8 of the 64 panel CUs) holds 112 groups
    assert plan_leaf(L, 28672, 56) == (1, 256, 112)
    assert plan_leaf(L, 28673, 56)[:2] == (2, 512)
    assert plan_leaf(L, 57344, 56) == (2, 512, 112)
    # one row more: neither register form fits in 56 CUs, and the LDS form
    # (one group per CU, rows in LDS) needs more LDS than a CU has
    assert plan_leaf(L, 57345, 56)[0] == 0
    # FP32 panels take the LDS form
    form, R, G = plan_leaf(L, 40000, 0, elem=4)
    assert form == 3 and G <= 256 and R * G >= 40000 and 4 * 32 * R <= LDS_BUDGET
    # every form keeps all groups resident: G <= CUs x groups per CU
    for m in (1, 255, 257, 5000, 30000, 60000, 100000, 131072):
        for cap in (0, 56):
            form, R, G = plan_leaf(L, m, cap)
            if form:
                cus = cap or 256
                assert R * G >= m and G <= (2 if form < 3 else 1) * cus


def test_lookahead_plan_boundary(L):
    """The first panel (n rows) runs on the caller's stream with every CU, so
    only the later panels (at most n - nb rows) are bound by the panel
    stream's cap: n = 57472 with nb = 128 (first panel 57472 rows, next
    57344) takes look-ahead; n = 57600 does not (next panel 57472 rows)."""
    args = (256, 2, 2, LDS_BUDGET)
    assert L.mxlu_plan_lookahead(32768, 256, *args) == 64
    assert L.mxlu_plan_lookahead(57472, 128, *args) == 64
    assert L.mxlu_plan_lookahead(57600, 128, *args) == 0
    assert L.mxlu_plan_lookahead(57600, 256, *args) == 64
    assert L.mxlu_plan_lookahead(32768, 64, *args) == 0        # nb % 128
    assert L.mxlu_plan_lookahead(32704, 256, *args) == 0       # n % 128
    assert L.mxlu_plan_lookahead(256, 256, *args) == 0         # a single panel
    assert L.mxlu_plan_lookahead(32768, 256, 304, 2, 2, LDS_BUDGET) == 0   # uneven split


def test_debug_and_release_hooks_validate(L):
    assert L.mxlu_debug_expire_waits(2) == -1
    assert L.mxlu_debug_expire_waits(0) == 0
    p = ctypes.c_void_p(16)
    assert L.mxlu_panel_factor_f64(10, 11, p, 10, p, None) == -2     # nb > m
    assert L.mxlu_panel_factor_f64(10, 4, p, 9, p, None) == -4
    assert L.mxlu_panel_factor_f64(10, 4, p, 10, None, None) == -5
