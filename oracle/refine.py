"""Iterative refinement in FP64 -- TEST INFRASTRUCTURE ONLY (oracle side).

The mixed-precision variant (Sec. III-A.2) factors in low precision and
restores FP64 accuracy by refinement whose residuals and corrections are FP64;
the refinement is "non-stationary ... based on GMRES" (Sec. II-B).  Two
methods, both preconditioned by the low-precision factors M = U^-1 L^-1 P:

  classical:  x <- x + M r
  GMRES-IR:   each outer step solves A d = r by left-preconditioned restarted
              GMRES (one cycle of at most `restart` Arnoldi steps, classical
              Gram-Schmidt applied twice, Givens rotations on the Hessenberg
              matrix), then x <- x + d.

The outer loop recomputes r = b - A x in FP64 and stops when the HPL scaled
residual drops below `threshold` (16).  x0 = M b.  ||A||_inf is computed once.
"""

from __future__ import annotations

import math

import numpy as np

from . import lp_precond
from .checks import EPS


def _gmres_cycle(matvec, prec, r, restart, inner_tol):
    z = prec(r)
    beta = float(np.linalg.norm(z))
    n = r.shape[0]
    if beta == 0.0:
        return np.zeros(n), 0, []
    V = np.zeros((n, restart + 1))
    H = np.zeros((restart + 1, restart))
    cs = np.zeros(restart)
    sn = np.zeros(restart)
    g = np.zeros(restart + 1)
    g[0] = beta
    V[:, 0] = z / beta
    k = 0
    resid_hist = [beta]
    for j in range(restart):
        w = prec(matvec(V[:, j]))
        h = V[:, :j + 1].T @ w            # classical Gram-Schmidt, twice
        w = w - V[:, :j + 1] @ h
        h2 = V[:, :j + 1].T @ w
        w = w - V[:, :j + 1] @ h2
        h = h + h2
        hn = float(np.linalg.norm(w))
        H[:j + 1, j] = h
        H[j + 1, j] = hn
        if hn > 0.0:
            V[:, j + 1] = w / hn
        for i in range(j):                # previous rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = math.hypot(H[j, j], H[j + 1, j])
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        resid_hist.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= inner_tol * beta or hn == 0.0:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):        # H[:k,:k] y = g[:k]
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    return V[:, :k] @ y, k, resid_hist


def refine(A, b, F, ipiv, method="gmres", trans=False, restart=30,
           max_outer=20, max_inner_total=300, inner_tol=1e-6, threshold=16.0):
    """Refine the solution of A x = b (or A^T x = b) with low-precision factors F.

    Returns dict(x, converged, outer_iters, inner_iters, history=[rho...])."""
    A = np.asarray(A, dtype=np.float64)
    Aop = A.T if trans else A
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[0]
    anorm = float(np.abs(Aop).sum(axis=1).max())
    bnorm = float(np.abs(b).max())

    def prec(v):
        return lp_precond(F, ipiv, v, trans=trans)

    def matvec(v):
        return Aop @ v

    x = prec(b)
    hist = []
    inner_total = 0
    increases = 0
    outer = 0
    converged = False
    while True:
        r = b - Aop @ x
        xn = float(np.abs(x).max())
        rho = float(np.abs(r).max()) / (EPS * (anorm * xn + bnorm) * n)
        hist.append(rho)
        if rho < threshold:
            converged = True
            break
        if len(hist) > 1 and hist[-1] > hist[-2]:
            increases += 1
        else:
            increases = 0
        if outer >= max_outer or increases >= 3 or inner_total >= max_inner_total:
            break
        if method == "classical":
            x = x + prec(r)
        elif method == "gmres":
            m = min(restart, max_inner_total - inner_total)
            d, k, _ = _gmres_cycle(matvec, prec, r, m, inner_tol)
            inner_total += k
            x = x + d
        else:
            raise ValueError(method)
        outer += 1
    return dict(x=x, converged=converged, outer_iters=outer,
                inner_iters=inner_total, history=hist)
