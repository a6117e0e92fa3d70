"""Pins of the FP64 oracle (blocked GEPP + solve) against things other than
itself: exact rational elimination, closed forms, invariants, and LAPACK.

The method is the LU factorization with partial pivoting followed by
triangular solves of Sec. III-A.1 (phases PFACT, SWAP, DTRSM, DGEMM).
"""

from fractions import Fraction
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import checks
from paper_2604_09517_amd import inputs


def exact_gepp(A):
    """Textbook GEPP in exact rational arithmetic (unblocked)."""
    n = A.shape[0]
    M = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    piv = []
    gaps = []
    for j in range(n):
        mags = [abs(M[i][j]) for i in range(j, n)]
        best = max(mags)
        p = j + mags.index(best)
        s = sorted(mags, reverse=True)
        gaps.append((s[0] - s[1]) / s[0] if len(s) > 1 and s[0] != 0 else Fraction(1))
        piv.append(p)
        M[j], M[p] = M[p], M[j]
        if M[j][j] == 0:
            continue
        for i in range(j + 1, n):
            M[i][j] = M[i][j] / M[j][j]
            for c in range(j + 1, n):
                M[i][c] -= M[i][j] * M[j][c]
    return M, piv, gaps


@pytest.mark.parametrize("n,seed", [(n, s) for n in (1, 2, 3, 5, 8) for s in range(4)])
def test_pivots_and_factors_match_exact_rational(oracle_lib, n, seed):
    A = inputs.uniform_matrix(seed, 0, n, n)
    LU, ipiv, info = oracle.getrf(A, nb=3)
    M, piv, gaps = exact_gepp(A)
    assert info == 0
    for j in range(n):
        if gaps[j] > 1e-10:
            assert ipiv[j] == piv[j], (j, ipiv, piv)
    if list(ipiv) == piv:
        exact = np.array([[float(M[i][j]) for j in range(n)] for i in range(n)])
        scale = np.abs(exact).max()
        assert np.abs(LU - exact).max() <= 64 * n * 2.0 ** -53 * scale * 10


@pytest.mark.parametrize("n", [1, 4, 9, 33])
def test_permutation_matrix_closed_form(oracle_lib, n):
    rng = np.random.default_rng(n)
    perm = rng.permutation(n)
    A = np.zeros((n, n), order="F")
    A[perm, np.arange(n)] = 1.0          # column j has its 1 in row perm[j]
    LU, ipiv, info = oracle.getrf(A, nb=4)
    assert info == 0
    assert np.array_equal(LU, np.eye(n))
    p = checks.perm_from_ipiv(ipiv, n)
    assert np.array_equal(A[p, :], np.eye(n))


@pytest.mark.parametrize("n,nb", [(7, 3), (40, 16), (65, 64)])
def test_upper_triangular_closed_form(oracle_lib, n, nb):
    rng = np.random.default_rng(1)
    U = np.triu(rng.uniform(-1, 1, (n, n)))
    U[np.arange(n), np.arange(n)] += np.sign(U[np.arange(n), np.arange(n)]) + 0.5
    LU, ipiv, info = oracle.getrf(np.asfortranarray(U), nb)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(n))
    assert np.array_equal(LU, U)          # bitwise: nothing to eliminate


@pytest.mark.parametrize("n,nb", [(6, 2), (50, 16)])
def test_lower_triangular_dominant_closed_form(oracle_lib, n, nb):
    rng = np.random.default_rng(2)
    A = np.tril(rng.uniform(-1, 1, (n, n)))
    d = 2.0 + rng.uniform(0, 1, n)
    A[np.arange(n), np.arange(n)] = d    # |a_jj| > |a_ij| for i > j
    LU, ipiv, info = oracle.getrf(np.asfortranarray(A), nb)
    assert np.array_equal(ipiv, np.arange(n))
    L_expect = np.tril(A / d[None, :], -1)
    assert np.array_equal(np.tril(LU, -1), L_expect)
    assert np.array_equal(np.triu(LU), np.diag(d))


def test_two_by_two_formula(oracle_lib):
    a, b, c, d = 0.3, -2.0, 0.75, 1.25   # |c| > |a| -> swap
    A = np.array([[a, b], [c, d]], order="F")
    LU, ipiv, info = oracle.getrf(A, 1)
    assert list(ipiv) == [1, 1]
    l = a / c
    assert LU[0, 0] == c and LU[0, 1] == d and LU[1, 0] == l
    # one fused multiply-add: the exact value b - l d rounded once
    assert LU[1, 1] == float(Fraction(b) - Fraction(l) * Fraction(d))


def test_zero_pivot_info_like_lapack(oracle_lib):
    n = 6
    A = inputs.uniform_matrix(3, 0, n, n)
    A[:, 2] = 0.0                          # column 2 exactly zero
    LU, ipiv, info = oracle.getrf(A, 2)
    assert info == 3                       # 1-based first zero pivot
    assert ipiv[2] == 2                    # first index of an all-zero column
    assert np.all(LU[:, 2][3:] == 0.0)
    _, _, info_lapack = sla.lapack.dgetrf(A)
    assert info_lapack == 3


def test_determinant_against_laplace_expansion(oracle_lib):
    def det_laplace(M):
        n = len(M)
        if n == 1:
            return M[0][0]
        return sum((-1) ** c * M[0][c] * det_laplace([r[:c] + r[c + 1:] for r in M[1:]])
                   for c in range(n))

    for n in (2, 3, 5, 7):
        A = inputs.uniform_matrix(10 + n, 0, n, n)
        LU, ipiv, _ = oracle.getrf(A, 2)
        swaps = int(np.sum(ipiv != np.arange(n)))
        det = (-1) ** swaps * np.prod(np.diag(LU))
        exact = det_laplace([[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)])
        assert abs(det - float(exact)) <= 1e-12 * max(1e-300, abs(float(exact))) * 100


@pytest.mark.parametrize("n", [97, 200])
def test_pivots_invariant_in_block_size(oracle_lib, n):
    A = inputs.uniform_matrix(77, 0, n, n)
    ref_LU, ref_piv, _ = oracle.getrf(A, n)
    for nb in (1, 2, 3, 7, 64):
        LU, piv, _ = oracle.getrf(A, nb)
        assert np.array_equal(piv, ref_piv)
        assert np.abs(LU - ref_LU).max() < 1e-11


@pytest.mark.parametrize("n,nb", [(64, 8), (300, 64), (1024, 64)])
def test_invariants_and_lapack(oracle_lib, n, nb):
    A = inputs.uniform_matrix(inputs.config_seed(0), 0, n, n)
    b = inputs.uniform_matrix(inputs.config_seed(0), 1, n, 1)[:, 0]
    LU, ipiv, info = oracle.getrf(A, nb)
    assert info == 0
    assert np.abs(np.tril(LU, -1)).max() <= 1.0
    assert checks.factorization_ratio(A, LU, ipiv) < 10
    x = oracle.getrs(LU, ipiv, b)
    assert checks.scaled_residual(A, x, b) < 16
    xt = oracle.getrs(LU, ipiv, b, trans=True)
    assert checks.scaled_residual(A.T, xt, b) < 16
    lu2, piv2 = sla.lu_factor(A)
    assert np.array_equal(piv2, ipiv)                  # LAPACK getrf, 0-based
    assert np.abs(lu2 - LU).max() < 1e-9
    x2 = sla.lu_solve((lu2, piv2), b, trans=1)
    assert np.abs(x2 - xt).max() <= 1e-9 * np.abs(x2).max()


def test_first_pivot_is_first_argmax_on_ties(oracle_lib):
    A = np.array([[0.5, 1.0, 0.0], [-2.0, 0.0, 1.0], [2.0, 1.0, 1.0]], order="F")
    _, ipiv, _ = oracle.getrf(A, 3)
    assert ipiv[0] == 1                    # |-2| == |2|: the smaller row index


@pytest.mark.parametrize("n", [3, 5, 6])
def test_hilbert_inverse_closed_form(oracle_lib, n):
    from math import comb
    H = np.array([[1.0 / (i + j + 1) for j in range(n)] for i in range(n)], order="F")
    Hinv = np.array([[(-1) ** (i + j) * (i + j + 1) * comb(n + i, n - j - 1)
                      * comb(n + j, n - i - 1) * comb(i + j, i) ** 2
                      for j in range(n)] for i in range(n)], dtype=np.float64)
    LU, ipiv, _ = oracle.getrf(H, 2)
    X = oracle.getrs(LU, ipiv, np.eye(n))
    kappa = np.abs(H).sum(1).max() * np.abs(Hinv).sum(1).max()
    assert np.abs(X - Hinv).max() <= 50 * n * kappa * 2.0 ** -53 * np.abs(Hinv).max()


def test_multiple_rhs_and_leading_dimension(oracle_lib):
    n = 50
    A = inputs.uniform_matrix(5, 0, n, n)
    B = inputs.uniform_matrix(5, 1, n, 7)
    LU, ipiv, _ = oracle.getrf(A, 16)
    X = oracle.getrs(LU, ipiv, B)
    for c in range(7):
        x1 = oracle.getrs(LU, ipiv, B[:, c])
        assert np.array_equal(X[:, c], x1)
    assert checks.scaled_residual(A, X, B) < 16


def test_partial_steps_equal_full_run_prefix(oracle_lib):
    n, nb = 96, 16
    A = inputs.uniform_matrix(9, 0, n, n)
    LU_full, piv_full, _ = oracle.getrf(A, nb)
    LU2, piv2, _ = oracle.getrf(A, nb, max_steps=2)
    assert np.array_equal(piv2[:32], piv_full[:32])
    # after two steps rows 0..31 (U and the L11 blocks) are final
    assert np.array_equal(LU2[:32, :], LU_full[:32, :])


def test_scaled_residual_measure_itself():
    A = np.diag([2.0, 4.0, 8.0])
    b = np.array([1.0, 1.0, 1.0])
    assert checks.scaled_residual(A, np.array([0.5, 0.25, 0.125]), b) == 0.0
    x = np.array([0.5, 0.25, 0.125 + 2.0 ** -40])
    rho = checks.scaled_residual(A, x, b)
    assert rho == pytest.approx((8.0 * 2.0 ** -40) / (2.0 ** -53 * (8.0 * 0.5 + 1.0) * 3))


def test_perm_from_ipiv_roundtrip():
    ipiv = [2, 2, 3, 3]
    p = checks.perm_from_ipiv(ipiv)
    # rows: start 0123; swap 0,2 -> 2103; swap 1,2 -> 2013; swap 2,3 -> 2031
    assert list(p) == [2, 0, 3, 1]
    for combo in itertools.product(range(3), repeat=3):
        ip = [max(j, c) for j, c in enumerate(combo)]
        assert sorted(checks.perm_from_ipiv(ip)) == [0, 1, 2]


def test_panel_alone_equals_first_step(oracle_lib):
    n, nb = 200, 48
    A = inputs.uniform_matrix(12, 0, n, n)
    LU, ipiv, _ = oracle.getrf(A, nb, max_steps=1)
    P, pp, _ = oracle.panel_getrf(A[:, :nb])
    assert np.array_equal(pp, ipiv[:nb])
    assert np.array_equal(P, LU[:, :nb])


@pytest.mark.parametrize("n,seed", [(n, s) for n in (3, 5, 8) for s in range(3)])
def test_pivot_gaps_match_exact_rational(oracle_lib, n, seed):
    """The gap report of the gap-recording factorization equals the exact
    rational runner-up gap of textbook GEPP, and its factors and pivots are
    those of the plain factorization."""
    A = inputs.uniform_matrix(100 + seed, 0, n, n)
    _, piv, gaps_exact = exact_gepp(A)
    Ag = np.asfortranarray(A.copy())
    ipiv_g, gaps, info = oracle.getrf_gaps_inplace(Ag, 3)
    LU, ipiv, _ = oracle.getrf(A, 3)
    assert np.array_equal(ipiv_g, ipiv) and np.array_equal(Ag, LU)
    for j in range(n):
        assert abs(gaps[j] - float(gaps_exact[j])) <= 1e-9, (j, gaps[j], gaps_exact[j])
    # a planted exact tie in the first column has gap 0
    B = A.copy()
    B[1, 0] = -B[np.argmax(np.abs(B[:, 0])), 0] if np.argmax(np.abs(B[:, 0])) != 1 else B[1, 0]
    Bg = np.asfortranarray(B)
    _, gb, _ = oracle.getrf_gaps_inplace(Bg, 3)
    assert gb[0] == 0.0 or np.argmax(np.abs(B[:, 0])) == 1
