"""Gradient through the solve -- TEST INFRASTRUCTURE ONLY (oracle side).

For X = A^-1 B and a loss L(X) with upstream gradient G = dL/dX, differentiating
A X = B gives A dX = dB - dA X, hence

    Lambda = A^-T G,      dL/dB = Lambda,      dL/dA = -Lambda X^T.

The transposed solve reuses the factors of the forward solve.
"""

from __future__ import annotations

import numpy as np

from . import getrf, getrs


def solve_and_grad(A, B, G, nb=64):
    LU, ipiv, info = getrf(A, nb)
    X = getrs(LU, ipiv, B)
    Lam = getrs(LU, ipiv, G, trans=True)
    X2 = X.reshape(A.shape[0], -1)
    L2 = Lam.reshape(A.shape[0], -1)
    dA = -L2 @ X2.T
    return X, dA, Lam, info
