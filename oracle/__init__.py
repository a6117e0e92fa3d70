"""CPU oracle for the dense LU solver -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the smoke check and the bench's CPU-baseline leg may import
this package.  It shares no code with the HIP library (`paper_2604_09517_amd`)
and never imports it; the only module both sides use is the seeded input
generator `paper_2604_09517_amd.inputs`, which holds none of the solver's
arithmetic.

Layout:
  mxlu_oracle.c   plain C: blocked GEPP, getrs (N/T), low-precision rounding,
                  low-precision LU, FP32 preconditioner        (this wrapper)
  checks.py       HPL scaled residual, factorization ratio, pivot comparison
  refine.py       classical and GMRES iterative refinement in FP64 (numpy)
  grad.py         gradient of a loss through the solve
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_PATH = os.path.join(_HERE, "mxlu_oracle.c")
LIB_PATH = os.path.join(_HERE, "libmxlu_oracle.so")

# -O2 plain C, OpenMP for the independent column loops, no contraction of
# a*b+c beyond the explicit fma() calls, hardware fma for those calls.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-mfma", "-fPIC", "-shared",
          "-std=c11"]

BF16, FP16, E4M3, FP32 = 0, 1, 2, 3

_lib = None


def build() -> str:
    """Compile the C oracle into oracle/libmxlu_oracle.so (always rebuilds)."""
    tmp = f"{LIB_PATH}.{os.getpid()}.tmp"   # per process: concurrent builds do not collide
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC_PATH, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def build_variant(src_path: str, out_path: str) -> str:
    """Compile another copy of the oracle source (used by the mutation tests,
    which plant mistakes in a copy to show that the pins catch them)."""
    subprocess.check_call(["gcc", *CFLAGS, "-o", out_path, src_path, "-lm"])
    return out_path


def load(path: str):
    """Make the functions of this module use the library at `path`; returns
    the previously loaded handle so a caller can restore it."""
    global _lib
    old = _lib
    _lib = _bind(ctypes.CDLL(path))
    return old


def restore(handle):
    global _lib
    _lib = handle


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or (
                os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH)):
            build()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def _bind(L):
    i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    L.oracle_getrf_steps.argtypes = [i64, i64, dp, i64, dp, i64]
    L.oracle_getrf_steps.restype = i32
    L.oracle_getrf_gaps.argtypes = [i64, i64, dp, i64, dp, dp]
    L.oracle_getrf_gaps.restype = i32
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = i32
    L.oracle_panel_getf2.argtypes = [i64, i64, dp, i64, dp]
    L.oracle_panel_getf2.restype = i32
    L.oracle_getrs.argtypes = [i64, i64, dp, i64, dp, dp, i64, i32]
    L.oracle_getrs.restype = i32
    L.oracle_round.argtypes = [ctypes.c_double, i32]
    L.oracle_round.restype = ctypes.c_double
    L.oracle_round_array.argtypes = [i64, dp, dp, i32]
    L.oracle_round_array.restype = None
    L.oracle_fp8_scale.argtypes = [ctypes.c_double]
    L.oracle_fp8_scale.restype = ctypes.c_double
    L.oracle_mx_scale.argtypes = [ctypes.c_double]
    L.oracle_mx_scale.restype = ctypes.c_double
    L.oracle_lp_getrf.argtypes = [i64, i64, i32, i32, i64, dp, i64, dp]
    L.oracle_lp_getrf.restype = i32
    L.oracle_lp_getrf_steps.argtypes = [i64, i64, i32, i32, i64, dp, i64, dp, i64]
    L.oracle_lp_getrf_steps.restype = i32
    L.oracle_lp_precond.argtypes = [i64, dp, i64, dp, dp, dp, i32]
    L.oracle_lp_precond.restype = i32
    return L


def threads():
    """Number of OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def getrf_inplace(A, nb, max_steps=-1):
    """getrf on a Fortran-ordered FP64 array in place (no copy; for timing
    large samples).  Returns (ipiv, info)."""
    assert A.dtype == np.float64 and A.flags["F_CONTIGUOUS"]
    n = A.shape[0]
    ipiv = np.arange(n, dtype=np.int32)
    info = lib().oracle_getrf_steps(n, int(nb), _ptr(A), max(n, 1), _ptr(ipiv),
                                    int(max_steps))
    if info < 0:
        raise ValueError(f"oracle_getrf: bad argument ({info})")
    return ipiv, info


def _fortran(a, dtype=np.float64):
    return np.array(a, dtype=dtype, order="F", copy=True)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def getrf(A, nb, max_steps=-1):
    """Blocked GEPP (Sec. III-A.1).  Returns (LU, ipiv 0-based int32, info)."""
    LU = _fortran(A)
    n = LU.shape[0]
    assert LU.shape == (n, n)
    ipiv = np.arange(n, dtype=np.int32)
    info = lib().oracle_getrf_steps(n, int(nb), _ptr(LU), max(n, 1), _ptr(ipiv),
                                    int(max_steps))
    if info < 0:
        raise ValueError(f"oracle_getrf: bad argument ({info})")
    return LU, ipiv, info


def getrf_gaps_inplace(A, nb):
    """getrf in place on a Fortran-ordered FP64 array, also returning the
    relative gap between the two largest candidates of every pivot search.
    Returns (ipiv, gaps, info)."""
    assert A.dtype == np.float64 and A.flags["F_CONTIGUOUS"]
    n = A.shape[0]
    ipiv = np.arange(n, dtype=np.int32)
    gaps = np.zeros(n, dtype=np.float64)
    info = lib().oracle_getrf_gaps(n, int(nb), _ptr(A), max(n, 1), _ptr(ipiv), _ptr(gaps))
    if info < 0:
        raise ValueError(f"oracle_getrf_gaps: bad argument ({info})")
    return ipiv, gaps, info


def panel_getrf(P):
    """GEPP of an m x kb panel (the first PFACT step).  Returns (LU, ipiv, info)."""
    LU = _fortran(P)
    m, kb = LU.shape
    ipiv = np.arange(kb, dtype=np.int32)
    info = lib().oracle_panel_getf2(m, kb, _ptr(LU), max(m, 1), _ptr(ipiv))
    if info < 0:
        raise ValueError("oracle_panel_getf2: bad argument")
    return LU, ipiv, info


def getrs(LU, ipiv, B, trans=False):
    """Solve A X = B (trans=False) or A^T X = B with the factors of getrf."""
    n = LU.shape[0]
    X = _fortran(B)
    vec = X.ndim == 1
    if vec:
        X = X.reshape(n, 1, order="F")
    LUf = np.asfortranarray(LU, dtype=np.float64)
    piv = np.ascontiguousarray(ipiv, dtype=np.int32)
    rc = lib().oracle_getrs(n, X.shape[1], _ptr(LUf), max(n, 1), _ptr(piv),
                            _ptr(X), max(n, 1), 1 if trans else 0)
    if rc != 0:
        raise ValueError(f"oracle_getrs: bad argument ({rc})")
    return X.reshape(n) if vec else X


def round_lp(x, fmt):
    """Round FP64 values to bf16 (0), fp16 (1), e4m3fn (2) or fp32 (3), returned as FP64."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(a)
    lib().oracle_round_array(a.size, _ptr(a), _ptr(out), int(fmt))
    return out


def fp8_scale(amax):
    return lib().oracle_fp8_scale(float(amax))


def mx_scale(amax):
    """E8M0 block scale of the MX FP8 form (power of two, exponent in [-127, 127])."""
    return lib().oracle_mx_scale(float(amax))


def lp_getrf(A, nb, prec, pivot=False, tile=128, max_steps=-1):
    """Low-precision blocked LU (Sec. III-A.2).  prec: 0 bf16, 1 fp16, 2 fp8
    updates with fp16 storage and per-tile scales, 3 fp8 updates with fp16
    storage and MX (E8M0 per 32 k) block scales, 4 fp32 storage.  Returns (F, ipiv or None, info) where F holds
    the stored factor values as FP64 numbers.  max_steps >= 0 stops after that
    many panel steps (the trailing block then holds the updated, unfactored
    Schur complement in storage precision)."""
    F = _fortran(A)
    n = F.shape[0]
    ipiv = np.arange(n, dtype=np.int32)
    info = lib().oracle_lp_getrf_steps(n, int(nb), int(prec), 1 if pivot else 0,
                                       int(tile), _ptr(F), max(n, 1), _ptr(ipiv),
                                       int(max_steps))
    if info < 0:
        raise ValueError(f"oracle_lp_getrf failed ({info})")
    return F, (ipiv if pivot else None), info


def lp_precond(F, ipiv, r, trans=False):
    """d = M r (or M^T r), M = U^-1 L^-1 P applied in FP32 with vector scaling."""
    n = F.shape[0]
    Ff = np.asfortranarray(F, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    d = np.empty(n, dtype=np.float64)
    piv = None if ipiv is None else np.ascontiguousarray(ipiv, dtype=np.int32)
    rc = lib().oracle_lp_precond(n, _ptr(Ff), max(n, 1), _ptr(piv), _ptr(rr),
                                 _ptr(d), 1 if trans else 0)
    if rc != 0:
        raise ValueError(f"oracle_lp_precond failed ({rc})")
    return d
