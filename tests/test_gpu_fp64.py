"""GPU parity of the FP64 path (Sec. III-A.1) against the CPU oracle, through
the C ABI.

Acceptance per factorization: pivots identical to the oracle's (a mismatch is
tolerated only at a certified near-tie, after which the rest is compared by
the unique measures), HPL scaled residual < 16 and
||PA - LU||_1 / (||A||_1 n eps) < 10 with eps = 2^-53.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import checks
from paper_2604_09517_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


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


def assert_pivots_match(A, ipiv_gpu, ipiv_ref):
    bad = checks.pivot_mismatches(ipiv_gpu, ipiv_ref)
    if len(bad):
        j = int(bad[0])
        assert checks.near_tie_at(A, ipiv_ref, j, rel=1e-12), \
            f"pivot mismatch at column {j} without a near-tie"
        note(f"near-tie pivot flip at column {j}: compared by residuals only")
        return False
    return True


# ---------------------------------------------------------------- generator
@pytest.mark.parametrize("rows,cols,ld", [(1, 1, 1), (300, 7, 305), (1024, 3, 1024)])
def test_device_generator_bitwise(api, rows, cols, ld):
    note(f"generator rows={rows} cols={cols} ld={ld}")
    t = api.fortran_empty(rows, cols, ld=ld)
    api.fill_uniform(t, 1234, 5)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), inputs.uniform_matrix(1234, 5, rows, cols))


def test_device_diag_dominant_bitwise(api):
    n = 257
    t = api.fortran_empty(n, n)
    api.fill_uniform(t, 7, 0)
    api.make_diag_dominant(t)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), inputs.diag_dominant_matrix(7, 0, n))


# ---------------------------------------------------------------- Schur GEMM
@pytest.mark.parametrize("M,N,K", [(128, 128, 16), (256, 384, 256), (130, 257, 33), (1, 1, 1),
                                   (17, 5, 3), (1000, 16, 256), (200, 17, 64), (513, 129, 7)])
def test_schur_update_against_definition(api, M, N, K):
    note(f"schur M={M} N={N} K={K}")
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.uniform(-1, 1, (M, K))
    B = rng.uniform(-1, 1, (K, N))
    C = rng.uniform(-1, 1, (M, N))
    dA, dB, dC = to_dev(A, ld=M + 3), to_dev(B), to_dev(C, ld=M + 1)
    api.schur_update(dC, dA, dB)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    ref = C - A @ B
    # both deviate from the exact C - AB by at most gamma_{K+1}(|C| + |A||B|)
    g = (K + 1) * EPS / (1 - (K + 1) * EPS)
    bound = 2 * g * (np.abs(C) + np.abs(A) @ np.abs(B)) + 1e-300
    assert np.all(np.abs(got - ref) <= bound)


def test_schur_update_uses_each_product_once(api):
    """Integer data: every product and partial sum is exact, so the result is
    exactly C - AB (catches a dropped or doubled k step or a wrong layout)."""
    rng = np.random.default_rng(3)
    M, N, K = 160, 144, 48
    A = rng.integers(-4, 5, (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, (K, N)).astype(np.float64)
    C = rng.integers(-100, 100, (M, N)).astype(np.float64)
    dC = to_dev(C)
    api.schur_update(dC, to_dev(A), to_dev(B))
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), C - A @ B)


# ---------------------------------------------------------------- lu_factor
CASES = [(1, 1), (2, 1), (5, 2), (31, 8), (64, 64), (100, 32), (257, 64), (300, 96),
         (600, 256), (130, 1024), (1024, 64), (1500, 256)]


@pytest.mark.parametrize("n,nb", CASES)
def test_lu_factor_matches_oracle(api, n, nb):
    note(f"lu_factor n={n} nb={nb}")
    seed = inputs.config_seed(0) + n
    A_h = inputs.uniform_matrix(seed, 0, n, n)
    ld = n + (5 if n % 2 else 0)
    dA = to_dev(A_h, ld=ld)
    _, ipiv, info = api.lu_factor(dA, nb)
    torch.cuda.synchronize()
    LU = dA.cpu().numpy()
    piv = ipiv.cpu().numpy()
    LU_ref, piv_ref, info_ref = oracle.getrf(A_h, nb)
    assert info == info_ref
    same = assert_pivots_match(A_h, piv, piv_ref)
    assert checks.factorization_ratio(A_h, LU, piv) < 10
    assert np.abs(np.tril(LU, -1)).max(initial=0.0) <= 1.0
    if same:
        # different summation order only: elementwise agreement far inside
        # the factorization-ratio bound
        scale = max(1.0, np.abs(LU_ref).max())
        assert np.abs(LU - LU_ref).max() <= 1e-9 * scale


# Sizes where depth-1 look-ahead applies (n, nb multiples of 128): the next
# panel is factored on its own CU-masked stream while the rest of the update
# runs on another.  Each element takes the same operations in the same order
# as at depth 0, so the factors must agree bit for bit.
LOOKAHEAD_CASES = [(1024, 128), (1152, 256), (2048, 256), (2560, 512)]


@pytest.mark.parametrize("n,nb", LOOKAHEAD_CASES)
def test_lookahead_matches_depth0_and_oracle(api, n, nb):
    note(f"lookahead n={n} nb={nb}")
    seed = inputs.config_seed(0) + 7 * n + nb
    A_h = inputs.uniform_matrix(seed, 0, n, n)
    out = {}
    try:
        for depth in (0, 1):
            api.set_lookahead(depth)
            dA = to_dev(A_h)
            _, ipiv, info = api.lu_factor(dA, nb)
            torch.cuda.synchronize()
            out[depth] = (dA.cpu().numpy(), ipiv.cpu().numpy(), info)
    finally:
        api.set_lookahead(1)
    (LU0, piv0, info0), (LU1, piv1, info1) = out[0], out[1]
    assert info0 == info1 == 0
    assert np.array_equal(piv0, piv1)
    assert np.array_equal(LU0, LU1)
    LU_ref, piv_ref, _ = oracle.getrf(A_h, nb)
    same = assert_pivots_match(A_h, piv1, piv_ref)
    assert checks.factorization_ratio(A_h, LU1, piv1) < 10
    if same:
        assert np.abs(LU1 - LU_ref).max() <= 1e-9 * max(1.0, np.abs(LU_ref).max())


def test_lookahead_depth_argument(api):
    assert api.lib().mxlu_set_lookahead(2) == -1
    assert api.lib().mxlu_set_lookahead(-1) == -1
    assert api.lib().mxlu_set_lookahead(1) == 0


def test_lu_factor_c1_configuration(api):
    """The small configuration (n = 1024, NB = 64, device-generated input)."""
    n, nb = 1024, 64
    seed = inputs.config_seed(0)
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    b_h = inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]
    db = torch.from_numpy(b_h).cuda()
    A0 = dA.clone()
    _, ipiv, info = api.lu_factor(dA, nb)
    x = api.lu_solve(dA, ipiv, db.clone())
    rho_dev = api.scaled_residual(A0, x, db)[0]
    torch.cuda.synchronize()
    A_h = inputs.uniform_matrix(seed, inputs.STREAM_A, n, n)
    LU_ref, piv_ref, _ = oracle.getrf(A_h, nb)
    assert info == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    rho = checks.scaled_residual(A_h, x.cpu().numpy(), b_h)
    assert rho < 16 and rho_dev < 16
    assert abs(rho - rho_dev) <= 1e-6 * max(rho, 1e-3) + 1e-3
    assert checks.factorization_ratio(A_h, dA.cpu().numpy(), piv_ref) < 10


def test_zero_pivot_column(api):
    n, nb = 70, 16
    A_h = inputs.uniform_matrix(99, 0, n, n)
    A_h[:, 20] = 0.0
    dA = to_dev(A_h)
    _, ipiv, info = api.lu_factor(dA, nb)
    torch.cuda.synchronize()
    LU_ref, piv_ref, info_ref = oracle.getrf(A_h, nb)
    assert info == info_ref == 21
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    assert np.abs(dA.cpu().numpy() - LU_ref).max() < 1e-9


def test_permutation_matrix_exact(api):
    n = 200
    perm = np.random.default_rng(4).permutation(n)
    A_h = np.zeros((n, n))
    A_h[perm, np.arange(n)] = 1.0
    dA = to_dev(A_h)
    _, ipiv, info = api.lu_factor(dA, 64)
    torch.cuda.synchronize()
    assert info == 0
    assert np.array_equal(dA.cpu().numpy(), np.eye(n))
    p = checks.perm_from_ipiv(ipiv.cpu().numpy(), n)
    assert np.array_equal(A_h[p, :], np.eye(n))


def test_upper_triangular_exact(api):
    n = 160
    rng = np.random.default_rng(8)
    U = np.triu(rng.uniform(-1, 1, (n, n))) + 3 * np.eye(n)
    dA = to_dev(U)
    _, ipiv, _ = api.lu_factor(dA, 64)
    torch.cuda.synchronize()
    assert np.array_equal(ipiv.cpu().numpy(), np.arange(n))
    assert np.array_equal(dA.cpu().numpy(), U)


# ---------------------------------------------------------------- lu_solve
@pytest.mark.parametrize("n,nrhs,trans", [(1, 1, 0), (100, 1, 0), (100, 3, 1), (1024, 1, 0),
                                          (1024, 1, 1), (700, 16, 0), (700, 17, 1),
                                          (513, 5, 0)])
def test_lu_solve_matches_oracle(api, n, nrhs, trans):
    note(f"lu_solve n={n} nrhs={nrhs} trans={trans}")
    A_h = inputs.uniform_matrix(500 + n, 0, n, n)
    B_h = inputs.uniform_matrix(500 + n, 1, n, nrhs)
    dA = to_dev(A_h)
    _, ipiv, _ = api.lu_factor(dA, 64)
    dB = to_dev(B_h, ld=n + 2)
    api.lu_solve(dA, ipiv, dB, trans=bool(trans))
    torch.cuda.synchronize()
    X = dB.cpu().numpy()
    LU = dA.cpu().numpy()
    X_ref = oracle.getrs(LU, ipiv.cpu().numpy(), B_h, trans=bool(trans))
    Aop = A_h.T if trans else A_h
    assert checks.scaled_residual(Aop, X, B_h) < 16
    kappa = np.linalg.cond(A_h, np.inf)
    assert np.abs(X - X_ref).max() <= 64 * n * EPS * kappa * np.abs(X_ref).max()


def test_argument_errors(api):
    dA = api.fortran_empty(4, 4)
    with pytest.raises(ValueError):
        api.lu_factor(dA, 0)
    L = api.lib()
    assert L.lu_factor(-1, 8, None, 1, None, None) == -1
    assert L.lu_factor(4, 8, dA.data_ptr(), 2, None, None) == -4
    assert L.lu_solve(4, 1, dA.data_ptr(), 4, None, None, 4, 0, None) == -5
    assert L.lu_solve(4, 1, dA.data_ptr(), 4, dA.data_ptr(), dA.data_ptr(), 4, 2, None) == -8


# ------------------------------------------------- full size (bench workload)
@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_fp64_bench_configuration(api):
    """n = 32768, NB = 256, as timed by the bench: GPU residual, first-panel
    pivots against the oracle, sampled rows of PA - LU."""
    cfg = inputs.WORKLOADS["fp64_large"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size n={n} nb={nb}")
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    _, ipiv, info = api.lu_factor(dA, nb)
    x = api.lu_solve(dA, ipiv, db.clone())
    torch.cuda.synchronize()
    assert info == 0
    # residual against the regenerated original A (device, FP64)
    A0 = api.fortran_empty(n, n)
    api.fill_uniform(A0, seed, inputs.STREAM_A)
    rho = api.scaled_residual(A0, x, db)[0]
    anorm = A0.abs().sum(dim=1).max().item()          # ||A||_inf
    note(f"scaled residual {rho:.3e}")
    assert rho < 16
    del A0
    torch.cuda.empty_cache()
    piv = ipiv.cpu().numpy()
    # first panel: the oracle's GEPP of the n x nb leading panel
    P = inputs.uniform_matrix(seed, inputs.STREAM_A, n, nb)
    _, piv_ref, _ = oracle.panel_getrf(P)
    assert np.array_equal(piv[:nb], piv_ref)
    # sampled rows of P A - L U: max row 1-norm / (||A||_inf n eps), a lower
    # bound of the infinity-norm factorization ratio
    LU = dA.cpu().numpy()
    perm = checks.perm_from_ipiv(piv, n)
    worst = 0.0
    for i in (0, 1, nb - 1, nb, 12345, n - 1):
        arow = inputs.uniform_at(seed, inputs.STREAM_A,
                                 np.arange(n, dtype=np.uint64) * np.uint64(n) + np.uint64(perm[i]))
        lrow = LU[i, :i]
        urow = np.zeros(n)
        for c0 in range(0, n, 4096):
            c1 = min(n, c0 + 4096)
            Ub = LU[:i, c0:c1] * (np.arange(c0, c1)[None, :] >= np.arange(i)[:, None])
            urow[c0:c1] = lrow @ Ub
        urow[i:] += LU[i, i:]
        r = arow - urow
        worst = max(worst, np.abs(r).sum())
    ratio = worst / (anorm * n * EPS)
    note(f"sampled factorization ratio {ratio:.3e}")
    assert ratio < 10
