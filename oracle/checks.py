"""Acceptance measures of a solve -- TEST INFRASTRUCTURE ONLY (oracle side).

* scaled residual (the HPL acceptance test):
      rho = ||b - A x||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n),  pass < 16
* factorization ratio:
      ||P A - L U||_1 / (||A||_1 n eps),  pass < 10
with eps = 2^-53 (unit roundoff of FP64).
"""

from __future__ import annotations

import numpy as np

EPS = 2.0 ** -53


def perm_from_ipiv(ipiv, n=None):
    """Row order p with (P A)[i] = A[p[i]] for the interchange sequence ipiv."""
    ipiv = np.asarray(ipiv)
    n = len(ipiv) if n is None else n
    p = np.arange(n)
    for j, t in enumerate(ipiv):
        if t != j:
            p[j], p[t] = p[t], p[j]
    return p


def unpack_lu(LU):
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    U = np.triu(LU)
    return L, U


def scaled_residual(A, x, b):
    A = np.asarray(A)
    x = np.asarray(x).reshape(A.shape[1], -1)
    b = np.asarray(b).reshape(A.shape[0], -1)
    n = A.shape[0]
    r = b - A @ x
    anorm = np.abs(A).sum(axis=1).max()
    out = []
    for c in range(x.shape[1]):
        den = EPS * (anorm * np.abs(x[:, c]).max() + np.abs(b[:, c]).max()) * n
        out.append(np.abs(r[:, c]).max() / den)
    return max(out)


def factorization_ratio(A, LU, ipiv):
    n = A.shape[0]
    p = perm_from_ipiv(ipiv, n)
    L, U = unpack_lu(LU)
    R = A[p, :] - L @ U
    return np.abs(R).sum(axis=0).max() / (np.abs(A).sum(axis=0).max() * n * EPS)


def forward_error(x, x_ref):
    x = np.asarray(x)
    x_ref = np.asarray(x_ref)
    return np.abs(x - x_ref).max() / np.abs(x_ref).max()


def pivot_mismatches(ipiv_a, ipiv_b):
    """Indices where two interchange sequences differ."""
    a = np.asarray(ipiv_a)
    b = np.asarray(ipiv_b)
    return np.nonzero(a != b)[0]


def near_tie_at(A_orig, ipiv_ref, j, rel=1e-12):
    """True when, at elimination step j of the reference factorization, the
    two largest candidates |a_ij| differ by at most rel (relative): a place where
    rounding order may legally flip the pivot.  Uses the exact Schur
    complement of the first j pivots computed in FP64 by a direct solve."""
    A = np.asarray(A_orig, dtype=np.float64)
    p = perm_from_ipiv(ipiv_ref, A.shape[0])
    Ap = A[p, :]
    if j == 0:
        col = np.abs(Ap[:, 0])
    else:
        A11 = Ap[:j, :j]
        A21 = Ap[j:, :j]
        s = Ap[j:, j] - A21 @ np.linalg.solve(A11, Ap[:j, j])
        col = np.abs(s)
        col = np.concatenate([np.zeros(j), col])
    cand = np.sort(col[j:])[::-1]
    if len(cand) < 2:
        return False
    return (cand[0] - cand[1]) <= rel * cand[0]
