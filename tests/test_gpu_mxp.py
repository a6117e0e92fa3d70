"""GPU parity of the mixed-precision path (Sec. III-A.2: low-precision LU
without pivoting and FP64 refinement; Sec. II-B: GMRES-based refinement)
against the CPU oracle, through the C ABI.

What is compared, and how:
  * conversion FP64 -> bf16/fp16: bit for bit;
  * factors: the first panel step (panel and U12 block row, FP32 arithmetic in
    the same operation order) bit for bit; the rest within a bound, since
    the MFMA trailing update sums products in its own order; the backward
    error ||LU - A|| / ||A|| of the GPU factors within 4 u (u = 2^-8 bf16,
    2^-11 fp16, 2^-4 for the FP8 update);
  * preconditioner M b on identical (oracle) factors: bit for bit;
  * solves: the HPL scaled residual < 16 (the acceptance threshold), the
    forward error against the FP64 oracle solution within the bound that
    rho < 16 implies, iteration counts close to the oracle refinement's.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import checks, refine
from paper_2604_09517_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53
U_LP = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp8": 2.0 ** -4}
PREC_ID = {"bf16": 0, "fp16": 1, "fp8": 2}


@pytest.fixture(scope="module")
def api():
    from paper_2604_09517_amd import api as _api
    _api.lib()
    torch.cuda.set_device(0)
    return _api


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, ld=None):
    from paper_2604_09517_amd import api as _api
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    t = _api.fortran_empty(a.shape[0], a.shape[1], ld=ld)
    t.copy_(torch.from_numpy(a))
    return t


def factors_to_host(api, work, n, prec):
    return api.mxp_factors(work, n, prec).to(torch.float64).cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_convert_bitwise(api, prec):
    rng = np.random.default_rng(1)
    rows, cols = 300, 7
    A = rng.standard_normal((rows, cols)) * 2.0 ** rng.integers(-30, 20, (rows, cols))
    A[0, 0] = 1.0 + 2.0 ** -8 + 2.0 ** -40      # above a bf16 halfway point
    A[1, 0] = 1.0 + 2.0 ** -8                    # exact halfway: ties to even
    A[2, 0] = 65520.0                            # fp16 overflow to inf
    A[3, 0] = 2.0 ** -25 * 3                     # fp16 subnormal rounding
    out = api.mxp_convert(to_dev(A, ld=rows + 3), prec)
    torch.cuda.synchronize()
    got = out.to(torch.float64).cpu().numpy()
    ref = oracle.round_lp(A, oracle.BF16 if prec == "bf16" else oracle.FP16)
    assert np.array_equal(got, ref)


def run_mxp(api, A_h, b_h, **kw):
    dA = to_dev(A_h)
    db = to_dev(b_h)
    X, rep, work, ipiv = api.mxp_solve(dA, db, allow_notconv=True, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), rep, work, dA


@pytest.mark.parametrize("prec,n,nb", [("bf16", 256, 64), ("fp16", 300, 64), ("bf16", 640, 128),
                                       ("fp8", 512, 128), ("fp8", 700, 128)])
def test_lp_factors_against_oracle(api, prec, n, nb):
    note(f"lp factors prec={prec} n={n} nb={nb}")
    A = inputs.diag_dominant_matrix(31 + n, 0, n)
    b = inputs.uniform_matrix(31 + n, 1, n, 1)[:, 0]
    _, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, max_outer=0, scale_tile=64)
    F = factors_to_host(api, work, n, prec)
    F_ref, _, info = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=64)
    assert rep["info"] == info == 0
    # first panel and first block row: FP32 arithmetic in the same order
    assert np.array_equal(F[:, :nb], F_ref[:, :nb])
    assert np.array_equal(F[:nb, :], F_ref[:nb, :])
    u = U_LP[prec]
    assert np.abs(F - F_ref).max() <= 4 * u * np.abs(F_ref).max()
    L, U = checks.unpack_lu(F)
    err = np.abs(L @ U - A).sum(1).max() / np.abs(A).sum(1).max()
    assert err <= 4 * u


@pytest.mark.parametrize("prec,trans", [("bf16", 0), ("fp16", 0), ("bf16", 1)])
def test_preconditioner_bitwise_on_oracle_factors(api, prec, trans):
    n, nb = 600, 64
    A = inputs.diag_dominant_matrix(77, 0, n)
    b = inputs.uniform_matrix(77, 1, n, 1)[:, 0]
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False)
    dA, db = to_dev(A), to_dev(b)
    opts = api.mxp_options(prec=prec, nb=nb, max_outer=0, reuse_factors=True, trans=bool(trans))
    work = torch.zeros(api.mxp_workspace_bytes(n, opts), dtype=torch.uint8, device="cuda")
    api.mxp_factors(work, n, prec).copy_(torch.from_numpy(F_ref).to(
        torch.bfloat16 if prec == "bf16" else torch.float16))
    X, rep, _, _ = api.mxp_solve(dA, db, work=work, opts=opts, allow_notconv=True)
    torch.cuda.synchronize()
    x0 = X.cpu().numpy()
    ref = oracle.lp_precond(F_ref, None, b, trans=bool(trans))
    if trans == 0:
        assert np.array_equal(x0, ref)
    else:
        assert np.abs(x0 - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("prec,method,n,nb", [
    ("bf16", "gmres", 512, 128), ("bf16", "classical", 512, 128), ("fp16", "gmres", 777, 64),
    ("fp8", "gmres", 1024, 128), ("bf16", "gmres", 2048, 256), ("fp8", "classical", 640, 128)])
def test_mxp_solve_matches_oracle(api, prec, method, n, nb):
    note(f"mxp_solve prec={prec} refine={method} n={n} nb={nb}")
    seed = inputs.config_seed(2) + n
    A = inputs.diag_dominant_matrix(seed, 0, n)
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    x, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, refine=method, scale_tile=128)
    assert rep["status"] == 0 and rep["converged"] == 1
    rho = checks.scaled_residual(A, x, b)
    assert rho < 16 and rep["scaled_residual"] < 16
    # oracle: the same algorithm on the oracle's factors
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=128)
    out = refine.refine(A, b, F_ref, None, method=method)
    assert out["converged"]
    assert abs(rep["outer_iters"] - out["outer_iters"]) <= 1
    LU, ipiv, _ = oracle.getrf(A, nb)
    x64 = oracle.getrs(LU, ipiv, b)
    kappa = np.linalg.cond(A, np.inf)
    fe = checks.forward_error(x, x64)
    note(f"  outer {rep['outer_iters']} (oracle {out['outer_iters']}), inner "
         f"{rep['inner_iters']} (oracle {out['inner_iters']}), rho {rho:.2f}, fwd err {fe:.2e}")
    assert fe < 4 * 16 * n * EPS * kappa


def test_mxp_transposed_and_multiple_rhs(api):
    n, nb = 500, 64
    A = inputs.diag_dominant_matrix(5, 0, n)
    B = inputs.uniform_matrix(5, 1, n, 3)
    dA, dB = to_dev(A), to_dev(B)
    X, rep, work, _ = api.mxp_solve(dA, dB, prec="bf16", nb=nb)
    torch.cuda.synchronize()
    assert rep["converged"] == 1
    assert checks.scaled_residual(A, X.cpu().numpy(), B) < 16
    # A^T X = B with the same factors
    Xt, rep2, _, _ = api.mxp_solve(dA, dB, work=work, prec="bf16", nb=nb, trans=True,
                                   reuse_factors=True)
    torch.cuda.synchronize()
    assert rep2["converged"] == 1
    assert checks.scaled_residual(A.T, Xt.cpu().numpy(), B) < 16


def test_mxp_nonconvergence_reported(api):
    n = 256
    A = inputs.diag_dominant_matrix(9, 0, n)
    b = inputs.uniform_matrix(9, 1, n, 1)[:, 0]
    _, rep, _, _ = run_mxp(api, A, b, prec="bf16", nb=64, refine="classical", max_outer=0)
    assert rep["status"] == -1004 and rep["converged"] == 0
    assert rep["outer_iters"] == 0 and rep["scaled_residual"] >= 16


def test_mxp_argument_errors(api):
    dA = api.fortran_empty(64, 64)
    db = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        api.mxp_solve(dA, db, nb=48)          # not a multiple of 32
    with pytest.raises(ValueError):
        api.mxp_solve(dA, db, prec="fp8", nb=64)   # FP8 needs nb % 128 == 0
    opts = api.mxp_options(nb=64)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        api.mxp_solve(dA, db, work=small, opts=opts)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_bf16_configuration(api):
    """N = 65536 diagonally dominant, BF16 storage, NB = 512, GMRES-IR."""
    cfg = inputs.WORKLOADS["bf16_ir"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size bf16 n={n} nb={nb}")
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    api.make_diag_dominant(dA)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    X, rep, work, _ = api.mxp_solve(dA, db, prec="bf16", nb=nb, refine="gmres")
    torch.cuda.synchronize()
    note(f"report {rep}")
    assert rep["converged"] == 1 and rep["info"] == 0
    rho = api.scaled_residual(dA, X, db)[0]
    note(f"independent scaled residual {rho:.3e}")
    assert rho < 16
    # sampled rows: x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii on the host
    x = X.cpu().numpy()
    b = db.cpu().numpy()
    for i in (0, 1, 4097, n - 1):
        arow = inputs.uniform_at(seed, inputs.STREAM_A,
                                 np.arange(n, dtype=np.uint64) * np.uint64(n) + np.uint64(i))
        arow[i] = np.abs(arow).sum() - np.abs(arow[i])
        r_i = b[i] - arow @ x
        assert abs(r_i) <= 16 * EPS * n * (np.abs(arow).sum() * np.abs(x).max() + np.abs(b).max())


def test_lp_pivoted_first_panel_matches_oracle(api):
    """Partial pivoting on FP32 panel values: the first panel (same FP32
    operation order) gives the oracle's pivots and values bit for bit."""
    n, nb = 320, 64
    A = inputs.uniform_matrix(91, 0, n, n)
    b = inputs.uniform_matrix(91, 1, n, 1)[:, 0]
    dA, db = to_dev(A), to_dev(b)
    X, rep, work, ipiv = api.mxp_solve(dA, db, prec="bf16", pivot=True, nb=nb, max_outer=0,
                                       allow_notconv=True)
    torch.cuda.synchronize()
    F = factors_to_host(api, work, n, "bf16")
    F_ref, piv_ref, info = oracle.lp_getrf(A, nb, 0, pivot=True)
    piv = ipiv.cpu().numpy()
    assert rep["info"] == info == 0
    assert np.array_equal(piv[:nb], piv_ref[:nb])
    # later panels may legitimately pick other pivots (their inputs passed
    # through the MFMA update) and move the first panel's rows differently:
    # compare the first panel row by row of the original matrix
    by_orig = np.empty_like(F[:, :nb])
    by_orig[checks.perm_from_ipiv(piv, n)] = F[:, :nb]
    by_orig_ref = np.empty_like(F_ref[:, :nb])
    by_orig_ref[checks.perm_from_ipiv(piv_ref, n)] = F_ref[:, :nb]
    assert np.array_equal(by_orig, by_orig_ref)
    # whole factorization: a valid interchange sequence and a small backward error
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    p = checks.perm_from_ipiv(piv, n)
    L, U = checks.unpack_lu(F)
    err = np.abs(L @ U - A[p, :]).sum(1).max() / np.abs(A).sum(1).max()
    assert err <= 64 * U_LP["bf16"]


@pytest.mark.parametrize("n,nb", [(512, 128), (1000, 64)])
def test_mxp_pivoted_solve_uniform_matrix(api, n, nb):
    A = inputs.uniform_matrix(93 + n, 0, n, n)
    b = inputs.uniform_matrix(93 + n, 1, n, 1)[:, 0]
    x, rep, work, _ = run_mxp(api, A, b, prec="bf16", pivot=True, nb=nb, refine="gmres",
                              restart=100, max_outer=30, max_inner_total=1000)
    note(f"pivoted bf16 n={n}: {rep}")
    assert rep["converged"] == 1
    assert checks.scaled_residual(A, x, b) < 16
