"""Pins of the mixed-precision oracle (Sec. III-A.2: low-precision factorization
and trailing updates without pivoting, FP64 residuals and corrections; Sec.
II-B: refinement based on GMRES) against independent facts: torch's own
format conversions, exact rational rounding, exactly representable
factorizations, adjoint identities and convergence properties.
"""

from fractions import Fraction
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import checks, refine
from paper_2604_09517_amd import inputs

FORMATS = {
    # name: (oracle id, p significand bits, emin, max finite, torch dtype)
    "bf16": (oracle.BF16, 8, -126, float.fromhex("0x1.fep127"), torch.bfloat16),
    "fp16": (oracle.FP16, 11, -14, 65504.0, torch.float16),
    "e4m3": (oracle.E4M3, 4, -6, 448.0, torch.float8_e4m3fn),
    "fp32": (oracle.FP32, 24, -126, float.fromhex("0x1.fffffep127"), torch.float32),
}


def exact_round(x, p, emin, maxfin, saturate):
    """Round-to-nearest-even of a double by integer arithmetic on its exact
    rational value (independent of the oracle's frexp/nearbyint method)."""
    if x == 0.0 or math.isnan(x):
        return x
    fx = Fraction(x)
    ax = abs(fx)
    E = math.floor(math.log2(ax))
    while Fraction(2) ** E > ax:
        E -= 1
    while Fraction(2) ** (E + 1) <= ax:
        E += 1
    E = max(E, emin)
    q = Fraction(2) ** (E - p + 1)
    t = ax / q
    fl = math.floor(t)
    rem = t - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    y = float(fl * q)
    if y > maxfin:
        y = maxfin if saturate else math.inf
    return math.copysign(y, x)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3"])
def test_rounding_matches_torch_casts_on_fp32_inputs(oracle_lib, fmt):
    fid, p, emin, maxfin, tdt = FORMATS[fmt]
    rng = np.random.default_rng(5)
    lim = maxfin * 0.95
    x32 = np.concatenate([
        rng.uniform(-lim, lim, 20000),
        rng.standard_normal(20000) * 2.0 ** rng.integers(emin - 6, 4, 20000),
    ]).astype(np.float32)
    got = oracle.round_lp(x32.astype(np.float64), fid)
    ref = torch.from_numpy(x32).to(tdt).to(torch.float64).numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3", "fp32"])
def test_rounding_is_correct_directly_from_fp64(oracle_lib, fmt):
    """Values that are not FP32 numbers: a path through FP32 would round twice."""
    fid, p, emin, maxfin, _ = FORMATS[fmt]
    rng = np.random.default_rng(6)
    xs = rng.standard_normal(3000) * 2.0 ** rng.integers(emin - 4, 6, 3000)
    # plus exact halfway points of the format nudged by one FP64 ulp: the
    # double-rounding trap
    q = 2.0 ** (0 - p + 1)
    half = 1.0 + q / 2
    xs = np.concatenate([xs, [half, np.nextafter(half, 2), np.nextafter(half, 0),
                              -half, 1.0 + 1.5 * q, 3 * 2.0 ** (emin - p)]])
    xs = xs[np.abs(xs) < maxfin]
    got = oracle.round_lp(xs, fid)
    ref = np.array([exact_round(float(v), p, emin, maxfin, fmt == "e4m3") for v in xs])
    assert np.array_equal(got, ref)
    # the nudged halfway values round differently from the exact halfway one
    if fmt != "e4m3":
        h = oracle.round_lp(np.array([half, np.nextafter(half, 2)]), fid)
        assert h[0] == 1.0 and h[1] == 1.0 + q


def test_fp32_rounding_is_the_ieee_cast(oracle_lib):
    """FP32 storage (the precision ladder's FP32 rung): rounding an FP64 value
    to FP32 is IEEE binary32 round-to-nearest-even, i.e. numpy's cast, over
    normal, subnormal and overflowing values."""
    rng = np.random.default_rng(8)
    xs = np.concatenate([
        rng.standard_normal(20000) * 2.0 ** rng.integers(-160, 130, 20000),
        [2.0 ** -149, 2.0 ** -150, 3 * 2.0 ** -151, 2.0 ** 128, -(2.0 ** 128),
         float.fromhex("0x1.ffffffp127"), float.fromhex("0x1.fffffe8p127")],
    ])
    got = oracle.round_lp(xs, oracle.FP32)
    with np.errstate(over="ignore"):
        ref = xs.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, ref)


def test_rounding_specials(oracle_lib):
    r = oracle.round_lp(np.array([np.inf, -np.inf, 0.0, -0.0, 1e300, 500.0]), oracle.E4M3)
    assert list(r) == [448.0, -448.0, 0.0, -0.0, 448.0, 448.0]
    r = oracle.round_lp(np.array([65520.0, 65519.0]), oracle.FP16)
    assert r[0] == np.inf and r[1] == 65504.0
    assert np.isnan(oracle.round_lp(np.array([np.nan]), oracle.BF16)[0])
    sub = oracle.round_lp(np.array([2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26]), oracle.FP16)
    assert list(sub) == [2.0 ** -24, 0.0, 2.0 ** -24]


def test_fp8_scale_is_minimal_power_of_two(oracle_lib):
    rng = np.random.default_rng(7)
    for amax in list(rng.uniform(1e-8, 1e4, 200)) + [448.0, 896.0, 1.0, 448.0 * 2.0 ** -20]:
        s = oracle.fp8_scale(amax)
        m, e = math.frexp(s)
        assert m == 0.5                              # power of two
        assert amax / s <= 448.0
        assert amax / (s / 2) > 448.0                # the next smaller one fails
    assert oracle.fp8_scale(0.0) == 1.0


def _exact_lu_pair(n, rng, dominant_l=True):
    """Unit-lower L with entries in {0, +-1/4, +-1/2} and upper U with small
    integer entries and power-of-two diagonal: every value the elimination
    produces is a short dyadic number, exact in bf16, fp16 and FP32."""
    L = np.tril(rng.choice([-0.5, -0.25, 0.0, 0.25, 0.5], (n, n)), -1) + np.eye(n)
    U = np.triu(rng.choice([-2.0, -1.0, 0.0, 1.0, 2.0, 3.0], (n, n)), 1)
    U += np.diag(rng.choice([4.0, 8.0, -4.0, 16.0], n))
    return L, U


@pytest.mark.parametrize("prec", [0, 1, 4])
def test_lp_lu_reproduces_exact_factors(oracle_lib, prec):
    rng = np.random.default_rng(11)
    n = 12
    L, U = _exact_lu_pair(n, rng)
    A = L @ U
    assert np.array_equal(oracle.round_lp(A, {0: 0, 1: 1, 4: oracle.FP32}[prec]), A)
    F, _, info = oracle.lp_getrf(A, nb=5, prec=prec, pivot=False)
    assert info == 0
    assert np.array_equal(np.tril(F, -1), np.tril(L, -1))
    assert np.array_equal(np.triu(F), U)


def test_lp_lu_fp8_update_exact_on_representable_operands(oracle_lib):
    """With L21 and U12 whose tile-scaled values are e4m3 numbers the FP8
    trailing update is exact, so the factors come back exactly."""
    rng = np.random.default_rng(12)
    n = 16
    L, U = _exact_lu_pair(n, rng)
    A = L @ U
    F, _, _ = oracle.lp_getrf(A, nb=4, prec=2, pivot=False, tile=8)
    assert np.array_equal(np.tril(F, -1), np.tril(L, -1))
    assert np.array_equal(np.triu(F), U)


def _tile_scaled_exact_lu(n, tile, seed):
    """Exact factors as in _exact_lu_pair, with rows and columns scaled by
    powers of two that are constant on each tile of `tile` rows (columns) and
    differ between neighbouring tiles: L' = Dr L Dr^-1, U' = Dr U Dc, so the
    rows of L21 and the columns of U12 fall into tiles whose largest entries
    differ by powers of two.  Every value stays a short dyadic number."""
    rng = np.random.default_rng(seed)
    L, U = _exact_lu_pair(n, rng)
    dr = 2.0 ** np.array([(i // tile) % 3 - 1 for i in range(n)], dtype=np.float64)
    dc = 2.0 ** np.array([1 - (j // tile) % 3 for j in range(n)], dtype=np.float64)
    L2 = (dr[:, None] * L) / dr[None, :]
    U2 = dr[:, None] * U * dc[None, :]
    return L2 @ U2, L2, U2


@pytest.mark.parametrize("n,nb,tile", [(24, 8, 4), (40, 16, 8), (36, 12, 12)])
def test_lp_lu_fp8_distinct_tile_scales_exact(oracle_lib, n, nb, tile):
    """FP8 update with one power-of-two scale per tile (Sec. III-A.2 reduced-
    precision trailing update; e4m3fn operands with per-tile scales): on
    factors whose tiles have different magnitudes every quantised operand is
    an e4m3 number times its own tile's scale, so the update is exact and the
    factors come back exactly -- but only when each row (column) is
    dequantised with the scale of its own tile."""
    A, L2, U2 = _tile_scaled_exact_lu(n, tile, seed=n + tile)
    assert np.array_equal(oracle.round_lp(A, oracle.FP16), A)
    # the tiles really carry different scales: the L21 row tiles of the first
    # step, and the U12 column tiles
    l21 = np.abs(np.tril(L2, -1)[nb:, :nb])
    amax_l = [l21[t:t + tile].max() for t in range(0, n - nb, tile)]
    u12 = np.abs(U2[:nb, nb:])
    amax_u = [u12[:, t:t + tile].max() for t in range(0, n - nb, tile)]
    assert len({oracle.fp8_scale(a) for a in amax_l}) > 1
    assert len({oracle.fp8_scale(a) for a in amax_u}) > 1
    assert any(oracle.fp8_scale(a) != oracle.fp8_scale(b) for a, b in zip(amax_l, amax_l[1:]))
    F, _, info = oracle.lp_getrf(A, nb=nb, prec=2, pivot=False, tile=tile)
    assert info == 0
    assert np.array_equal(np.tril(F, -1), np.tril(L2, -1))
    assert np.array_equal(np.triu(F), U2)


@pytest.mark.parametrize("n,nb", [(96, 64), (160, 128)])
def test_lp_lu_mx_block_scales_exact(oracle_lib, n, nb):
    """MX FP8 update (E8M0 scale per row of L21 / column of U12 and block of
    32 consecutive k): with the rows and columns scaled by powers of two
    that change every 32 indices, the blocks of one row of L21 (and of one
    column of U12) have different magnitudes; every quantised value is still
    an e4m3 number times its own block's scale, so the update is exact and
    the factors come back exactly -- only when each block is dequantised
    with its own scale."""
    A, L2, U2 = _tile_scaled_exact_lu(n, 32, seed=n + nb)
    assert np.array_equal(oracle.round_lp(A, oracle.FP16), A)
    l21 = np.abs(np.tril(L2, -1)[nb:, :nb])
    blocks = [l21[:, b:b + 32].max(axis=1) for b in range(0, nb, 32)]
    row = int(np.argmax([len({oracle.mx_scale(bk[r]) for bk in blocks}) for r in range(n - nb)]))
    assert len({oracle.mx_scale(bk[row]) for bk in blocks}) > 1   # one row, distinct scales
    F, _, info = oracle.lp_getrf(A, nb=nb, prec=3, pivot=False)
    assert info == 0
    assert np.array_equal(np.tril(F, -1), np.tril(L2, -1))
    assert np.array_equal(np.triu(F), U2)


def test_mx_scale_is_minimal_e8m0(oracle_lib):
    rng = np.random.default_rng(8)
    for amax in list(rng.uniform(1e-8, 1e4, 200)) + [448.0, 896.0, 1.0]:
        s = oracle.mx_scale(amax)
        assert s == oracle.fp8_scale(amax)
        assert amax / s <= 448.0 < amax / (s / 2)
    assert oracle.mx_scale(0.0) == 1.0
    assert oracle.mx_scale(1e-60) == 2.0 ** -127        # clamped to the E8M0 range
    assert oracle.mx_scale(1e60) == 2.0 ** 127


def test_lp_lu_pivoted_recovers_permutation(oracle_lib):
    rng = np.random.default_rng(13)
    n = 10
    L = np.tril(rng.choice([-0.5, -0.25, 0.0, 0.25, 0.5], (n, n)), -1) + np.eye(n)
    U = np.triu(rng.choice([-2.0, -1.0, 1.0, 2.0], (n, n)), 1) + np.diag(
        rng.choice([4.0, -8.0, 16.0], n))
    perm = rng.permutation(n)
    PA = L @ U
    A = np.empty_like(PA)
    A[perm, :] = PA                               # A = P^T (L U)
    F, ipiv, info = oracle.lp_getrf(A, nb=3, prec=0, pivot=True)
    assert info == 0
    assert np.array_equal(checks.perm_from_ipiv(ipiv, n), perm)
    assert np.array_equal(np.tril(F, -1), np.tril(L, -1))
    assert np.array_equal(np.triu(F), U)
    # the FP64 oracle picks the same pivots on this matrix
    _, ipiv64, _ = oracle.getrf(A, 3)
    assert np.array_equal(ipiv64, ipiv)


@pytest.mark.parametrize("prec,u", [(0, 2.0 ** -8), (1, 2.0 ** -11), (2, 2.0 ** -4),
                                    (3, 2.0 ** -4), (4, 2.0 ** -24)])
def test_lp_lu_backward_error_bound(oracle_lib, prec, u):
    n = 192
    A = inputs.diag_dominant_matrix(21, 0, n)
    F, _, info = oracle.lp_getrf(A, nb=32, prec=prec, pivot=False, tile=64)
    assert info == 0
    L, U = checks.unpack_lu(F)
    # storage rounding (u) plus the FP32 arithmetic of the k sums (n 2^-24),
    # which dominates only for FP32 storage
    u32 = 2.0 ** -24
    err = np.abs(L @ U - A).sum(1).max() / np.abs(A).sum(1).max()
    assert err <= 4 * u + n * u32
    # and close to the FP64 factors (the FP64 oracle pivots on the diagonal here)
    LU64, ipiv64, _ = oracle.getrf(A, 32)
    assert np.array_equal(ipiv64, np.arange(n))
    assert (np.abs(np.triu(F) - np.triu(LU64)).max()
            <= (8 * u + 2 * n * u32) * np.abs(np.triu(LU64)).max())


def test_dominant_matrix_pivots_on_diagonal(oracle_lib):
    for n in (64, 300):
        A = inputs.diag_dominant_matrix(2, 0, n)
        _, ipiv, _ = oracle.getrf(A, 64)
        assert np.array_equal(ipiv, np.arange(n))


def test_preconditioner_solves_with_factors_and_adjoint(oracle_lib):
    n = 150
    A = inputs.diag_dominant_matrix(31, 0, n)
    F, _, _ = oracle.lp_getrf(A, nb=32, prec=0, pivot=False)
    L, U = checks.unpack_lu(F)
    r = inputs.uniform_matrix(31, 1, n, 1)[:, 0]
    s = inputs.uniform_matrix(31, 2, n, 1)[:, 0]
    d = oracle.lp_precond(F, None, r)
    ref = np.linalg.solve(U, np.linalg.solve(L, r))
    assert np.abs(d - ref).max() <= 1e-5 * np.abs(ref).max()
    dt = oracle.lp_precond(F, None, s, trans=True)
    reft = np.linalg.solve(L.T, np.linalg.solve(U.T, s))
    assert np.abs(dt - reft).max() <= 1e-5 * np.abs(reft).max()
    # <M r, s> = <r, M^T s>
    assert abs(d @ s - r @ dt) <= 1e-5 * abs(d @ s)


def test_preconditioner_with_pivots_and_exact_factors(oracle_lib):
    rng = np.random.default_rng(17)
    n = 9
    L = np.tril(rng.choice([-0.5, 0.0, 0.5], (n, n)), -1) + np.eye(n)
    U = np.triu(rng.choice([-1.0, 1.0], (n, n)), 1) + np.diag(rng.choice([2.0, 4.0], n))
    perm = rng.permutation(n)
    A = np.empty((n, n))
    A[perm, :] = L @ U
    F, ipiv, _ = oracle.lp_getrf(A, nb=4, prec=0, pivot=True)
    x = rng.choice([-1.0, 1.0], n)
    # the vector is scaled by 1/||b||_inf before the FP32 solves, so the
    # result is exact to FP32 rounding of that scaling only
    b = A @ x
    assert np.abs(oracle.lp_precond(F, ipiv, b) - x).max() < 1e-6
    bt = A.T @ x
    assert np.abs(oracle.lp_precond(F, ipiv, bt, trans=True) - x).max() < 1e-6
    # with a power-of-two scale everything is exact
    b2 = b / np.abs(b).max()
    x2 = oracle.lp_precond(F, ipiv, b2 * 8.0)
    assert np.abs(x2 - 8.0 * x / np.abs(b).max()).max() < 1e-6
    assert np.array_equal(oracle.lp_precond(F, ipiv, np.zeros(n)), np.zeros(n))


def test_gmres_cycle_terminates_in_n_steps_unpreconditioned():
    n = 7
    A = inputs.uniform_matrix(3, 0, n, n) + 2 * np.eye(n)
    r = inputs.uniform_matrix(3, 1, n, 1)[:, 0]
    d, k, hist = refine._gmres_cycle(lambda v: A @ v, lambda v: v, r, n, 1e-14)
    assert k <= n
    assert np.abs(A @ d - r).max() <= 1e-12 * np.abs(r).max()
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))


def test_gmres_cycle_exact_preconditioner_one_step():
    n = 20
    A = inputs.uniform_matrix(4, 0, n, n) + 3 * np.eye(n)
    Ainv = np.linalg.inv(A)
    r = inputs.uniform_matrix(4, 1, n, 1)[:, 0]
    d, k, _ = refine._gmres_cycle(lambda v: A @ v, lambda v: Ainv @ v, r, 10, 1e-10)
    assert k == 1
    assert np.abs(d - np.linalg.solve(A, r)).max() < 1e-12


def test_refine_exact_factors_converge_immediately(oracle_lib):
    rng = np.random.default_rng(23)
    n = 12
    L, U = _exact_lu_pair(n, rng)
    A = L @ U
    F, _, _ = oracle.lp_getrf(A, nb=4, prec=0)
    x_true = rng.choice([-1.0, 1.0, 0.5], n)
    b = A @ x_true
    # M = A^-1 up to FP32 rounding of the scaled vectors: x0 has an error
    # of order u_fp32 and each classical step multiplies it by about u_fp32
    out = refine.refine(A, b, F, None, method="classical")
    assert out["converged"] and out["outer_iters"] == 1
    assert np.abs(out["x"] - x_true).max() <= 1e-12


@pytest.mark.parametrize("method,prec", [("classical", 0), ("gmres", 0), ("gmres", 2),
                                         ("classical", 1), ("gmres", 3), ("gmres", 4)])
def test_refine_reaches_fp64_accuracy_on_dominant_matrix(oracle_lib, method, prec):
    n = 256
    A = inputs.diag_dominant_matrix(inputs.config_seed(2), 0, n)
    b = inputs.uniform_matrix(inputs.config_seed(2), 1, n, 1)[:, 0]
    F, _, _ = oracle.lp_getrf(A, nb=64, prec=prec, pivot=False, tile=64)
    out = refine.refine(A, b, F, None, method=method)
    assert out["converged"]
    assert checks.scaled_residual(A, out["x"], b) < 16
    LU, ipiv, _ = oracle.getrf(A, 64)
    x64 = oracle.getrs(LU, ipiv, b)
    # rho < 16 bounds the forward error of each solution by about
    # 2 * 16 n eps kappa_inf (||b|| <= ||A|| ||x||); two such solutions differ by
    # at most twice that
    kappa = np.linalg.cond(A, np.inf)
    assert checks.forward_error(out["x"], x64) < 4 * 16 * n * checks.EPS * kappa
    # the residual history goes down
    assert out["history"][-1] < out["history"][0]


@pytest.mark.parametrize("method", ["classical", "gmres"])
def test_refine_stopping_measure_is_the_hpl_residual(oracle_lib, method):
    """The refinement's own stopping measure at every iterate equals the HPL
    scaled residual of the acceptance checks at that iterate."""
    n = 96
    A = inputs.diag_dominant_matrix(43, 0, n)
    b = inputs.uniform_matrix(43, 1, n, 1)[:, 0]
    F, _, _ = oracle.lp_getrf(A, nb=32, prec=0)
    full = refine.refine(A, b, F, None, method=method, threshold=0.0, max_outer=3)
    for k in range(4):
        out = refine.refine(A, b, F, None, method=method, threshold=0.0, max_outer=k)
        assert out["outer_iters"] == k
        rho = checks.scaled_residual(A, out["x"], b)
        assert abs(out["history"][-1] - rho) <= 1e-12 * rho
        assert abs(full["history"][k] - rho) <= 1e-12 * rho


def test_refine_transposed(oracle_lib):
    n = 128
    A = inputs.diag_dominant_matrix(41, 0, n)
    b = inputs.uniform_matrix(41, 1, n, 1)[:, 0]
    F, _, _ = oracle.lp_getrf(A, nb=32, prec=0)
    out = refine.refine(A, b, F, None, method="gmres", trans=True)
    assert out["converged"]
    assert checks.scaled_residual(A.T, out["x"], b) < 16


def test_refine_pivoted_bf16_on_uniform_matrix(oracle_lib):
    n = 128
    A = inputs.uniform_matrix(51, 0, n, n)
    b = inputs.uniform_matrix(51, 1, n, 1)[:, 0]
    F, ipiv, _ = oracle.lp_getrf(A, nb=32, prec=0, pivot=True)
    out = refine.refine(A, b, F, ipiv, method="gmres", restart=100)
    assert out["converged"]
    assert checks.scaled_residual(A, out["x"], b) < 16


def test_refine_reports_non_convergence(oracle_lib):
    n = 64
    A = inputs.diag_dominant_matrix(61, 0, n)
    b = inputs.uniform_matrix(61, 1, n, 1)[:, 0]
    F, _, _ = oracle.lp_getrf(A, nb=16, prec=0)
    out = refine.refine(A, b, F, None, method="classical", max_outer=0)
    assert not out["converged"] and out["outer_iters"] == 0
