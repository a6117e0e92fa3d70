"""Python entry points over the C ABI (include/mxlu.h).

Matrices are torch tensors on the GPU, FP64, column-major: a rows x cols
tensor whose stride(0) == 1 and stride(1) = leading dimension >= rows (the
transpose view of a row-major tensor, see `fortran_empty`).  Vectors are 1-D
contiguous tensors.  Every call enqueues on torch's current stream.  Nothing
here computes: all work runs in the HIP library.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import MxpOpts, MxpReport, check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def fortran_empty(rows, cols, dtype=torch.float64, device="cuda", ld=None):
    """Uninitialised column-major rows x cols tensor with leading dimension ld."""
    ld = max(1, rows) if ld is None else ld
    base = torch.empty((cols, ld), dtype=dtype, device=device)
    return base.t()[:rows, :]


def _mat(t, name, dtype=torch.float64):
    """(ptr, rows, cols, ld) of a column-major matrix or a 1-D vector."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dim() == 1:
        if t.numel() > 0 and t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr(), t.shape[0], 1, max(1, t.shape[0])
    if t.dim() != 2:
        raise ValueError(f"{name} must be 1-D or 2-D")
    rows, cols = t.shape
    if rows > 0 and cols > 0:
        if t.stride(0) != 1 and rows > 1:
            raise ValueError(f"{name} must be column-major (stride(0) == 1)")
        ld = t.stride(1) if cols > 1 else max(rows, t.stride(1))
        if ld < max(1, rows):
            raise ValueError(f"{name}: leading dimension {ld} < rows {rows}")
    else:
        ld = max(1, rows)
    return t.data_ptr(), rows, cols, ld


def set_lookahead(depth):
    """Look-ahead depth of lu_factor (0 or 1, process-wide; default 1)."""
    check("mxlu_set_lookahead", lib().mxlu_set_lookahead(int(depth)))


def lu_factor(A, nb=256, ipiv=None):
    """In-place blocked LU with partial pivoting.  Returns (A, ipiv, info)."""
    pa, n, n2, lda = _mat(A, "A")
    if n != n2:
        raise ValueError("A must be square")
    if ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int32, device=A.device)
    pp, _, _, _ = _mat(ipiv, "ipiv", torch.int32)
    rc = lib().lu_factor(n, nb, pa, lda, pp, _stream())
    info = check("lu_factor", rc, positive_ok=True)
    return A, ipiv, info


def lu_solve_noalloc(LU, ipiv, B, trans=False):
    """lu_solve without device allocation (library-owned scratch, n <= 65536)."""
    pl, n, _, lda = _mat(LU, "LU")
    pp, _, _, _ = _mat(ipiv, "ipiv", torch.int32)
    pb, nb_rows, nrhs, ldb = _mat(B, "B")
    if nb_rows != n:
        raise ValueError("B must have n rows")
    rc = lib().lu_solve_noalloc(n, nrhs, pl, lda, pp, pb, ldb, 1 if trans else 0, _stream())
    check("lu_solve_noalloc", rc)
    return B


def panel_factor(P, ipiv=None):
    """In-place GEPP of an m x nb FP64 panel (the PFACT phase alone).
    Returns (P, ipiv with 0-based panel rows, info)."""
    pp, m, nb, ldp = _mat(P, "P")
    if ipiv is None:
        ipiv = torch.empty(nb, dtype=torch.int32, device=P.device)
    pi, _, _, _ = _mat(ipiv, "ipiv", torch.int32)
    rc = lib().mxlu_panel_factor_f64(m, nb, pp, ldp, pi, _stream())
    info = check("mxlu_panel_factor_f64", rc, positive_ok=True)
    return P, ipiv, info


def release():
    """Destroy the library's cached streams and events (no work in flight)."""
    check("mxlu_release", lib().mxlu_release())


def debug_expire_waits(on):
    """Test hook: panel factorizations start with their waits expired."""
    check("mxlu_debug_expire_waits", lib().mxlu_debug_expire_waits(1 if on else 0))


def debug_poison_scratch(byte):
    """Test hook: every scratch buffer starts filled with `byte` (None: off)."""
    check("mxlu_debug_poison_scratch",
          lib().mxlu_debug_poison_scratch(-1 if byte is None else int(byte)))


def lu_solve(LU, ipiv, B, trans=False):
    """In-place solve A X = B (or A^T X = B) with the factors of lu_factor."""
    pl, n, _, lda = _mat(LU, "LU")
    pp, _, _, _ = _mat(ipiv, "ipiv", torch.int32)
    pb, nb_rows, nrhs, ldb = _mat(B, "B")
    if nb_rows != n:
        raise ValueError("B must have n rows")
    rc = lib().lu_solve(n, nrhs, pl, lda, pp, pb, ldb, 1 if trans else 0, _stream())
    check("lu_solve", rc)
    return B


def schur_update(C, A, B):
    """C <- C - A B (FP64 matrix cores)."""
    pc, m, n, ldc = _mat(C, "C")
    pa, m2, k, lda = _mat(A, "A")
    pb, k2, n2, ldb = _mat(B, "B")
    if m2 != m or n2 != n or k2 != k:
        raise ValueError("shape mismatch")
    rc = lib().mxlu_schur_update_f64(m, n, k, pa, lda, pb, ldb, pc, ldc, _stream())
    check("mxlu_schur_update_f64", rc)
    return C


def outer_update(C, A, B, accumulate=False):
    """C <- (accumulate ? C : 0) - A B^T (FP64 matrix cores); B is N x K."""
    pc, m, n, ldc = _mat(C, "C")
    pa, m2, k, lda = _mat(A, "A")
    pb, n2, k2, ldb = _mat(B, "B")
    if m2 != m or n2 != n or k2 != k:
        raise ValueError("shape mismatch")
    rc = lib().mxlu_outer_update_f64(m, n, k, pa, lda, pb, ldb, pc, ldc, 1 if accumulate else 0,
                                     _stream())
    check("mxlu_outer_update_f64", rc)
    return C


def fill_uniform(A, seed, stream_id):
    """Seeded i.i.d. values in [-0.5, 0.5) (the shared counter-based generator)."""
    pa, r, c, lda = _mat(A, "A")
    rc = lib().mxlu_fill_uniform(r, c, pa, lda, int(seed), int(stream_id), _stream())
    check("mxlu_fill_uniform", rc)
    return A


def make_diag_dominant(A):
    pa, n, _, lda = _mat(A, "A")
    rc = lib().mxlu_make_diag_dominant(n, pa, lda, _stream())
    check("mxlu_make_diag_dominant", rc)
    return A


def scaled_residual(A, X, B, trans=False):
    """HPL scaled residuals (one per column), computed in FP64 on the GPU."""
    pa, n, _, lda = _mat(A, "A")
    px, _, nrhs, ldx = _mat(X, "X")
    pb, _, _, ldb = _mat(B, "B")
    out = (ctypes.c_double * max(1, nrhs))()
    rc = lib().mxlu_scaled_residual(n, nrhs, pa, lda, px, ldx, pb, ldb, 1 if trans else 0,
                                    out, _stream())
    check("mxlu_scaled_residual", rc)
    return [out[i] for i in range(nrhs)]


PREC = {"bf16": 0, "fp16": 1, "fp8": 2, "fp8_mx": 3, "fp32": 4}
REFINE = {"classical": 0, "gmres": 1}


def mxp_options(prec="bf16", pivot=False, nb=512, refine="gmres", restart=30, max_outer=20,
                max_inner_total=300, inner_tol=1e-6, resid_threshold=16.0, scale_tile=128,
                reuse_factors=False, trans=False, x_init=False, factor_steps=0):
    o = MxpOpts()
    lib().mxp_default_opts(ctypes.byref(o))
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.pivot = 1 if pivot else 0
    o.nb = int(nb)
    o.refine = REFINE[refine] if isinstance(refine, str) else int(refine)
    o.restart = int(restart)
    o.max_outer = int(max_outer)
    o.max_inner_total = int(max_inner_total)
    o.inner_tol = float(inner_tol)
    o.resid_threshold = float(resid_threshold)
    o.scale_tile = int(scale_tile)
    o.reuse_factors = 1 if reuse_factors else 0
    o.trans = 1 if trans else 0
    o.x_init = 1 if x_init else 0
    o.factor_steps = int(factor_steps)
    return o


def mxp_workspace_bytes(n, opts, lda=None):
    lda = max(1, int(n)) if lda is None else int(lda)
    return int(lib().mxp_workspace_bytes(int(n), lda, ctypes.byref(opts)))


def mxp_factor_ld(n):
    return int(lib().mxp_factor_ld(int(n)))


def mxp_factors(work, n, prec="bf16"):
    """View of the low-precision factors held at the start of `work`
    (n x n, column-major, as torch.bfloat16, torch.float16 or, for FP32
    storage, torch.float32)."""
    ldf = mxp_factor_ld(n)
    if prec in ("fp32", 4):
        dt, esz = torch.float32, 4
    else:
        dt, esz = (torch.bfloat16 if prec in ("bf16", 0) else torch.float16), 2
    words = work[: esz * ldf * n].view(dt)
    return words.view(n, ldf).t()[:n, :]


def mxp_convert(A, prec="bf16", out=None):
    """A (FP64) rounded to bf16 / fp16 on the GPU (column-major result)."""
    pa, r, c, lda = _mat(A, "A")
    dt = torch.bfloat16 if prec in ("bf16", 0) else torch.float16
    if out is None:
        out = fortran_empty(r, c, dtype=dt, device=A.device)
    po, _, _, ldo = _mat(out, "out", dt)
    code = PREC[prec] if isinstance(prec, str) else int(prec)
    rc = lib().mxp_convert(code, r, c, pa, lda, po, ldo, _stream())
    check("mxp_convert", rc)
    return out


def mxp_solve(A, B, X=None, work=None, ipiv=None, opts=None, allow_notconv=False, **kw):
    """Mixed-precision solve.  Returns (X, report dict, work, ipiv)."""
    opts = opts if opts is not None else mxp_options(**kw)
    pa, n, _, lda = _mat(A, "A")
    pb, _, nrhs, ldb = _mat(B, "B")
    if X is None:
        X = fortran_empty(n, nrhs, device=A.device) if B.dim() == 2 else torch.empty(
            n, dtype=torch.float64, device=A.device)
    px, _, _, ldx = _mat(X, "X")
    need = mxp_workspace_bytes(n, opts, lda)
    if work is None:
        work = torch.empty(max(1, need), dtype=torch.uint8, device=A.device)
    if opts.pivot and ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int32, device=A.device)
    pp = ipiv.data_ptr() if (opts.pivot and ipiv is not None) else None
    rep = MxpReport()
    rc = lib().mxp_solve(n, nrhs, pa, lda, pb, ldb, px, ldx, work.data_ptr(), work.numel(), pp,
                         ctypes.byref(opts), ctypes.byref(rep), _stream())
    report = {f: getattr(rep, f) for f, _ in MxpReport._fields_}
    if not (allow_notconv and rc == -1004):
        check("mxp_solve", rc)
    report["status"] = rc
    return X, report, work, ipiv


def mxp_solve_seeded(n, seed, stream_id, B, dominant=True, X=None, work=None, ipiv=None,
                     opts=None, allow_notconv=False, **kw):
    """Mixed-precision solve of the seeded matrix regenerated on the fly (no
    FP64 copy of A).  Returns (X, report dict, work, ipiv)."""
    opts = opts if opts is not None else mxp_options(**kw)
    pb, nb_rows, nrhs, ldb = _mat(B, "B")
    if nb_rows != n:
        raise ValueError("B must have n rows")
    if X is None:
        X = fortran_empty(n, nrhs, device=B.device) if B.dim() == 2 else torch.empty(
            n, dtype=torch.float64, device=B.device)
    px, _, _, ldx = _mat(X, "X")
    need = mxp_workspace_bytes(n, opts, n)
    if work is None:
        work = torch.empty(max(1, need), dtype=torch.uint8, device=B.device)
    if opts.pivot and ipiv is None:
        ipiv = torch.empty(n, dtype=torch.int32, device=B.device)
    pp = ipiv.data_ptr() if (opts.pivot and ipiv is not None) else None
    rep = MxpReport()
    rc = lib().mxp_solve_seeded(int(n), int(seed), int(stream_id), 1 if dominant else 0, nrhs, pb,
                                ldb, px, ldx, work.data_ptr(), work.numel(), pp,
                                ctypes.byref(opts), ctypes.byref(rep), _stream())
    report = {f: getattr(rep, f) for f, _ in MxpReport._fields_}
    if not (allow_notconv and rc == -1004):
        check("mxp_solve_seeded", rc)
    report["status"] = rc
    return X, report, work, ipiv


def exported_symbols():
    """Names the binding expects the library to export."""
    return list(_lib.SIGNATURES)


PHASES = ["pfact", "swap", "trsm", "gemm", "solve", "convert", "lp_factor", "refine",
          "lp_schur"]


def profile_enable(on=True):
    check("mxlu_profile_enable", lib().mxlu_profile_enable(1 if on else 0))


def profile_reset():
    check("mxlu_profile_reset", lib().mxlu_profile_reset())


def profile_read():
    """{phase: (ms, work, count)} accumulated since the last reset."""
    n = len(PHASES)
    ms = (ctypes.c_double * n)()
    work = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    check("mxlu_profile_read", lib().mxlu_profile_read(ms, work, cnt, n))
    return {p: (ms[i], work[i], cnt[i]) for i, p in enumerate(PHASES)}


def profile_intervals(phase):
    """[(step, ms, work), ...] of one phase (a name of PHASES) since the last reset."""
    k = PHASES.index(phase)
    n = int(lib().mxlu_profile_intervals(k, None, None, None, 0))
    if n < 0:
        raise RuntimeError(f"mxlu_profile_intervals failed ({n})")
    step = (ctypes.c_int64 * max(1, n))()
    ms = (ctypes.c_double * max(1, n))()
    work = (ctypes.c_double * max(1, n))()
    lib().mxlu_profile_intervals(k, step, ms, work, n)
    return [(step[i], ms[i], work[i]) for i in range(n)]
