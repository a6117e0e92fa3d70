"""Pins of the oracle gradient through X = A^-1 B (loss = sum(W * X)):
closed form for diagonal A, central finite differences, and torch autograd of
torch.linalg.solve on the CPU."""

import numpy as np
import pytest
import torch

from oracle import grad
from paper_2604_09517_amd import inputs


def test_diagonal_closed_form(oracle_lib):
    d = np.array([2.0, -0.5, 4.0, 1.25])
    A = np.diag(d)
    b = np.array([1.0, 2.0, -3.0, 0.5])
    w = np.array([0.3, -1.0, 2.0, 0.25])
    X, dA, dB, _ = grad.solve_and_grad(A, b, w, nb=2)
    assert np.allclose(X, b / d, rtol=0, atol=1e-15)
    assert np.allclose(np.diag(dA), -w * b / d ** 2, rtol=1e-15)
    assert np.allclose(dB, w / d, rtol=1e-15)
    # dA = -Lambda X^T with Lambda = w / d and X = b / d
    assert np.allclose(dA, -np.outer(w / d, b / d), rtol=1e-15, atol=0)


def test_against_torch_autograd(oracle_lib):
    n, k = 48, 3
    A = inputs.uniform_matrix(8, 0, n, n)
    B = inputs.uniform_matrix(8, 1, n, k)
    W = inputs.normal_matrix(8, n, k)
    X, dA, dB, _ = grad.solve_and_grad(A, B, W, nb=16)
    At = torch.tensor(A, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    Xt = torch.linalg.solve(At, Bt)
    (Xt * torch.tensor(W)).sum().backward()
    assert np.abs(X - Xt.detach().numpy()).max() < 1e-10
    assert np.abs(dA - At.grad.numpy()).max() <= 1e-9 * np.abs(dA).max()
    assert np.abs(dB - Bt.grad.numpy()).max() <= 1e-9 * np.abs(dB).max()


def test_central_finite_differences(oracle_lib):
    n, k = 40, 2
    A = inputs.uniform_matrix(9, 0, n, n)
    B = inputs.uniform_matrix(9, 1, n, k)
    W = inputs.normal_matrix(9, n, k)
    _, dA, dB, _ = grad.solve_and_grad(A, B, W, nb=8)

    def loss(A_, B_):
        return float(np.sum(W * np.linalg.solve(A_, B_)))

    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(8):
        i, j = rng.integers(0, n, 2)
        Ap = A.copy(); Ap[i, j] += h
        Am = A.copy(); Am[i, j] -= h
        fd = (loss(Ap, B) - loss(Am, B)) / (2 * h)
        assert abs(fd - dA[i, j]) <= 1e-5 * max(1.0, abs(dA[i, j]))
    for _ in range(4):
        i, c = rng.integers(0, n), rng.integers(0, k)
        Bp = B.copy(); Bp[i, c] += h
        Bm = B.copy(); Bm[i, c] -= h
        fd = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
        assert abs(fd - dB[i, c]) <= 1e-5 * max(1.0, abs(dB[i, c]))


def test_gradcheck_tiny(oracle_lib):
    n = 6
    A0 = inputs.uniform_matrix(10, 0, n, n) + 2 * np.eye(n)
    B0 = inputs.uniform_matrix(10, 1, n, 2)
    W = inputs.normal_matrix(10, n, 2)

    class OracleSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, A, B):
            X, dA, dB, _ = grad.solve_and_grad(A.numpy(), B.numpy(), W, nb=2)
            ctx.save_for_backward(A, B, torch.tensor(X))
            return torch.tensor(X)

        @staticmethod
        def backward(ctx, g):
            A, B, X = ctx.saved_tensors
            _, dA, dB, _ = grad.solve_and_grad(A.numpy(), B.numpy(), g.numpy(), nb=2)
            return torch.tensor(dA), torch.tensor(dB)

    A = torch.tensor(A0, requires_grad=True)
    B = torch.tensor(B0, requires_grad=True)
    assert torch.autograd.gradcheck(OracleSolve.apply, (A, B), eps=1e-6, atol=1e-7)
