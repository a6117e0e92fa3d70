"""GPU parity of the FP64 path (Sec. III-A.1) against the CPU oracle, through
the C ABI.

Acceptance per factorization: pivots identical to the oracle's (a mismatch is
tolerated only at a certified near-tie, after which the rest is compared by
the unique measures), HPL scaled residual < 16 and
||PA - LU||_1 / (||A||_1 n eps) < 10 with eps = 2^-53.
"""

import os
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
GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_pivots.npz")


def full_factorization_ratio(api, A0, LU, piv, block=2048):
    """||P A - L U||_1 / (||A||_1 n eps) over the whole matrix, formed on the
    device in column blocks (torch FP64 products serve only as the test's
    independent comparator)."""
    n = A0.shape[0]
    perm = torch.from_numpy(checks.perm_from_ipiv(piv, n)).to(A0.device)
    L = torch.tril(LU, -1)
    L.diagonal().fill_(1.0)
    U = torch.triu(LU)
    worst = 0.0
    for c0 in range(0, n, block):
        c1 = min(n, c0 + block)
        R = A0[:, c0:c1].index_select(0, perm) - L[:, :c1] @ U[:c1, c0:c1]
        worst = max(worst, R.abs().sum(dim=0).max().item())
    anorm1 = A0.abs().sum(dim=0).max().item()
    del L, U
    return worst / (anorm1 * n * EPS)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_fp64_bench_configuration(api):
    """n = 32768, NB = 256, as timed by the bench: all 32768 pivots against
    the oracle's (stored by tests/golden/make_c2_pivots.py, with the gap of
    every pivot search for the near-tie rule), the first panel's values
    against the oracle's GEPP of the leading panel, the full factorization
    ratio and the scaled residual."""
    cfg = inputs.WORKLOADS["fp64_large"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size n={n} nb={nb}")
    gold = np.load(GOLDEN_C2)
    assert int(gold["n"]) == n and int(gold["nb"]) == nb and int(gold["seed"]) == seed
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    _, ipiv, info = api.lu_factor(dA, nb)
    x = api.lu_solve(dA, ipiv, db.clone())
    torch.cuda.synchronize()
    assert info == 0 == int(gold["info"])
    piv = ipiv.cpu().numpy()
    # every pivot; a first mismatch is legal only where the oracle's two best
    # candidates were within 1e-12 (relative), and then only that prefix is
    # comparable
    bad = checks.pivot_mismatches(piv, gold["ipiv"])
    if len(bad):
        j = int(bad[0])
        note(f"first pivot mismatch at column {j}, oracle gap {gold['gaps'][j]:.3e}")
        assert gold["gaps"][j] <= 1e-12, f"pivot mismatch at column {j} without a near-tie"
    else:
        note(f"all {n} pivots equal the oracle's (smallest oracle gap "
             f"{gold['gaps'].min():.2e})")
    A0 = api.fortran_empty(n, n)
    api.fill_uniform(A0, seed, inputs.STREAM_A)
    rho = api.scaled_residual(A0, x, db)[0]
    note(f"scaled residual {rho:.3e}")
    assert rho < 16
    ratio = full_factorization_ratio(api, A0, dA, piv)
    note(f"factorization ratio ||PA - LU||_1 / (||A||_1 n eps) = {ratio:.3e}")
    assert ratio < 10
    del A0
    torch.cuda.empty_cache()
    # the first panel: the oracle's GEPP of the n x nb leading panel.  Later
    # steps move the panel's rows, so rows are compared by original index.
    P = inputs.uniform_matrix(seed, inputs.STREAM_A, n, nb)
    Pref, piv_ref, _ = oracle.panel_getrf(P)
    assert np.array_equal(piv[:nb], piv_ref)
    F = dA[:, :nb].cpu().numpy()
    by_orig = np.empty_like(F)
    by_orig[checks.perm_from_ipiv(piv, n)] = F
    by_orig_ref = np.empty_like(Pref)
    by_orig_ref[checks.perm_from_ipiv(piv_ref, n)] = Pref
    d = np.abs(by_orig - by_orig_ref)
    note(f"first panel: max |dL| {d.max():.3e}, entries differing {(d > 0).sum()}")
    assert d.max() <= 1e-12 * max(1.0, np.abs(Pref).max())


# ------------------------------------------------------------ PFACT alone
@pytest.mark.parametrize("m,nb", [(70000, 256), (5000, 100), (3000, 32)])
def test_panel_factor_matches_oracle(api, m, nb):
    """The PFACT phase alone against the oracle's GEPP of the panel: pivots
    identical, values within rounding.  m = 70000 needs more than 256 groups
    of 256 rows, so the register leaf runs with two rows per thread; nb = 100
    ends with a 4-column leaf (the LDS form)."""
    note(f"panel factor m={m} nb={nb}")
    P = inputs.uniform_matrix(300 + nb, 0, m, nb)
    dP = to_dev(P)
    _, ipiv, info = api.panel_factor(dP)
    torch.cuda.synchronize()
    Pref, piv_ref, info_ref = oracle.panel_getrf(P)
    assert info == info_ref == 0
    assert np.array_equal(ipiv.cpu().numpy(), piv_ref)
    d = np.abs(dP.cpu().numpy() - Pref)
    note(f"  max |d| {d.max():.3e}")
    assert d.max() <= 1e-12 * max(1.0, np.abs(Pref).max())


# ------------------------------------------------------ expired-wait path
@pytest.mark.parametrize("depth", [0, 1])
def test_expired_waits_return_timeout_within_bounds(api, depth):
    """Forced from the host: every panel wait starts expired, so each gives
    up at its first check and every kernel runs to completion on stale
    exchange words.  lu_factor must return MXLU_E_TIMEOUT, every interchange
    must stay a row of the matrix, and nothing outside A and ipiv may
    change.  A factorization afterwards is normal again."""
    n, nb, pad = 1024, 128, 4096
    note(f"expired waits depth={depth}")
    buf = torch.full((pad + n * n + pad,), 12345.0, dtype=torch.float64, device="cuda")
    A = buf[pad:pad + n * n].view(n, n).t()
    api.fill_uniform(A, 7, 0)
    ibuf = torch.full((n + 128,), -7, dtype=torch.int32, device="cuda")
    ipiv = ibuf[64:64 + n]
    L = api.lib()
    api.set_lookahead(depth)
    api.debug_expire_waits(True)
    try:
        rc = L.lu_factor(n, nb, A.data_ptr(), n, ipiv.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        api.debug_expire_waits(False)
        api.set_lookahead(1)
    assert rc == -1005
    assert torch.all(buf[:pad] == 12345.0) and torch.all(buf[pad + n * n:] == 12345.0)
    assert torch.all(ibuf[:64] == -7) and torch.all(ibuf[64 + n:] == -7)
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    # the library is not left in a failed state
    A_h = inputs.uniform_matrix(7, 0, n, n)
    dA = to_dev(A_h)
    _, ipiv2, info = api.lu_factor(dA, nb)
    torch.cuda.synchronize()
    _, piv_ref, _ = oracle.getrf(A_h, nb)
    assert info == 0 and np.array_equal(ipiv2.cpu().numpy(), piv_ref)


def test_release_then_factor_again(api):
    """mxlu_release drops the cached look-ahead streams and events; the next
    factorization creates them again."""
    n, nb = 1024, 128
    A_h = inputs.uniform_matrix(8, 0, n, n)
    api.profile_enable(True)
    api.release()
    dA = to_dev(A_h)
    _, ipiv, info = api.lu_factor(dA, nb)
    torch.cuda.synchronize()
    api.profile_read()
    api.profile_enable(False)
    _, piv_ref, _ = oracle.getrf(A_h, nb)
    assert info == 0 and np.array_equal(ipiv.cpu().numpy(), piv_ref)


@pytest.mark.parametrize("lookahead", [0, 1])
def test_results_independent_of_scratch_contents(api, lookahead):
    """Determinism: the factorization and the solve on scratch memory that
    starts as zeros and on scratch that starts as NaN bytes (0xFF) give the
    same pivots, factors and solution bit for bit: no uninitialised scratch
    reaches a result."""
    n, nb = 2304, 128
    seed = 4242
    A0 = api.fortran_empty(n, n)
    api.fill_uniform(A0, seed, inputs.STREAM_A)
    b0 = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    api.set_lookahead(lookahead)
    try:
        out = []
        for byte in (0x00, 0xFF):
            api.debug_poison_scratch(byte)   # every scratch buffer starts as `byte`
            A = A0.clone()
            b = b0.clone()
            ipiv0 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            LU, ipiv, _ = api.lu_factor(A, nb=nb, ipiv=ipiv0)
            x = api.lu_solve(LU, ipiv, b)
            torch.cuda.synchronize()
            out.append((LU.cpu(), ipiv.cpu(), x.cpu()))
    finally:
        api.set_lookahead(1)
        api.debug_poison_scratch(None)
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][2], out[1][2])
