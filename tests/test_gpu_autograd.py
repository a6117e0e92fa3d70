"""GPU parity of the differentiable solve (autograd.Function): gradient of
loss = sum(W * X), X = A^-1 B, against the CPU oracle gradient
(Lambda = A^-T W, dA = -Lambda X^T, dB = Lambda), central finite
differences, and torch.autograd.gradcheck."""

import sys

import numpy as np
import pytest
import torch

from oracle import grad as ograd
from paper_2604_09517_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ag():
    from paper_2604_09517_amd import api, autograd
    api.lib()
    torch.cuda.set_device(0)
    return autograd


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grads(ag, A_h, B_h, W_h, mode, nb=64):
    A = torch.tensor(A_h, device="cuda", requires_grad=True)
    B = torch.tensor(B_h, device="cuda", requires_grad=True)
    X = ag.solve(A, B, mode=mode, nb=nb)
    loss = (X * torch.tensor(W_h, device="cuda")).sum()
    loss.backward()
    torch.cuda.synchronize()
    return X.detach().cpu().numpy(), A.grad.cpu().numpy(), B.grad.cpu().numpy()


@pytest.mark.parametrize("mode,n,k", [("fp64", 64, 3), ("fp64", 300, 16), ("bf16_ir", 256, 2)])
def test_gradient_matches_oracle(ag, mode, n, k):
    note(f"autograd {mode} n={n} k={k}")
    A = inputs.uniform_matrix(400 + n, 0, n, n)
    B = inputs.uniform_matrix(400 + n, 1, n, k)
    W = inputs.normal_matrix(400 + n, n, k)
    X, dA, dB = grads(ag, A, B, W, mode)
    Xr, dAr, dBr, _ = ograd.solve_and_grad(A, B, W, nb=64)
    tol = 1e-9 if mode == "fp64" else 1e-8
    assert np.abs(X - Xr).max() <= tol * np.abs(Xr).max()
    assert np.abs(dB - dBr).max() <= tol * np.abs(dBr).max()
    assert np.abs(dA - dAr).max() <= tol * np.abs(dAr).max()


def test_gradcheck_fp64(ag):
    n = 8
    A0 = inputs.uniform_matrix(7, 0, n, n) + 2 * np.eye(n)
    B0 = inputs.uniform_matrix(7, 1, n, 2)
    A = torch.tensor(A0, device="cuda", requires_grad=True)
    B = torch.tensor(B0, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: ag.solve(a, b, mode="fp64", nb=4), (A, B),
                                    eps=1e-6, atol=1e-7)


@pytest.mark.parametrize("mode", ["fp64", "bf16_ir"])
def test_full_size_gradient_finite_differences(ag, mode):
    """n = 8192, 16 right-hand sides, loss = sum(W * X) with W ~ N(0, 1):
    central differences on single entries of A and B.

    FP64 on the uniform matrix: step h = 1e-4, |fd - g| <= 1e-5 max(1, |g|).
    The central difference has truncation error O(h^2 |d3L/dh3|) and rounding
    error about eps kappa |L| / h (two independent factorizations); with
    kappa ~ 1e4 and |L| ~ 1e3, h = 1e-6 leaves ~1e-4 of rounding noise while
    h = 1e-4 brings both terms near 1e-6.

    Mixed precision on the diagonally dominant matrix of the mixed-precision
    benchmark (the class its refinement is meant for; on the uniform matrix
    BF16-preconditioned GMRES needs thousands of iterations at this size).
    The solve is only accurate to its stopping residual, so the step must be
    large: by Sherman-Morrison, L(A + h e_i e_j^T) - L(A) = -h lam_i x_j /
    (1 + h (A^-1)_ji), and |(A^-1)_ji| <~ 1e-7 off the diagonal (diagonal
    ~ n / 4), so h = 1 keeps truncation near 1e-14 relative, while the
    solver noise ~1e-13 |L| / h stays far below the gradient (~1e-7).
    Criterion: |fd - g| <= 1e-5 max(|g|, 1e-3 max|grad|)."""
    cfg = inputs.WORKLOADS["autograd"]
    n, k, nb, seed = cfg["n"], cfg["nrhs"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full-size autograd {mode} n={n} k={k}")
    from paper_2604_09517_amd import api
    A = api.fortran_empty(n, n)
    api.fill_uniform(A, seed, inputs.STREAM_A)
    if mode == "fp64":
        h = 1e-4
    else:
        api.make_diag_dominant(A)
        h = 1.0
    B = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, k)).cuda()
    W = torch.from_numpy(inputs.normal_matrix(seed, n, k)).cuda()
    Ar = A.clone().requires_grad_(True)
    Br = B.clone().requires_grad_(True)
    X = ag.solve(Ar, Br, mode=mode, nb=nb)
    (X * W).sum().backward()
    dA, dB = Ar.grad, Br.grad
    torch.cuda.synchronize()
    floor_a = 1.0 if mode == "fp64" else 1e-3 * float(dA.abs().max())
    floor_b = 1.0 if mode == "fp64" else 1e-3 * float(dB.abs().max())

    def loss(Ap, Bp):
        with torch.no_grad():
            return float((ag.solve(Ap, Bp, mode=mode, nb=nb) * W).sum())

    rng = np.random.default_rng(0)
    worst = 0.0
    for t in range(20):
        i, j = (int(v) for v in rng.integers(0, n, 2))
        Ap = A.clone(); Ap[i, j] += h
        Am = A.clone(); Am[i, j] -= h
        fd = (loss(Ap, B) - loss(Am, B)) / (2 * h)
        g = float(dA[i, j])
        worst = max(worst, abs(fd - g) / max(floor_a, abs(g)))
    for t in range(8):
        i, c = int(rng.integers(0, n)), int(rng.integers(0, k))
        Bp = B.clone(); Bp[i, c] += h
        Bm = B.clone(); Bm[i, c] -= h
        fd = (loss(A, Bp) - loss(A, Bm)) / (2 * h)
        g = float(dB[i, c])
        worst = max(worst, abs(fd - g) / max(floor_b, abs(g)))
    note(f"worst relative finite-difference mismatch {worst:.2e}")
    assert worst <= 1e-5


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_bf16_ir_form_on_configured_uniform_matrix(ag):
    """The mixed-precision form on the workload as configured: n = 8192
    uniform A, 16 right-hand sides, BF16 LU with partial pivoting on FP32
    panel values, FP64 GMRES refinement.

    Restart 100 does not converge on this matrix (kappa ~ 1e4 against the
    BF16 unit roundoff 2^-8: the preconditioned operator is far from the
    identity and a 100-step cycle stagnates); the library reports that as
    MXLU_E_NOTCONV with the iteration counts, which is what is checked.
    Restart 200 converges; then
      * every column's HPL scaled residual is < 16;
      * the gradient (transposed GMRES-IR with the same factors, and the
        outer-product update) agrees with the FP64 form's gradient within
        what two solutions meeting rho < 16 can differ by (~16 n eps kappa);
      * central differences on entries of B: the loss is linear in B, so any
        step h is exact up to the solves' own accuracy (single-column solves,
        since a change in column c of B moves only column c of X)."""
    from paper_2604_09517_amd import api
    cfg = inputs.WORKLOADS["autograd"]
    n, k, nb, seed = cfg["n"], cfg["nrhs"], cfg["nb"], inputs.config_seed(cfg["index"])
    A = api.fortran_empty(n, n)
    api.fill_uniform(A, seed, inputs.STREAM_A)
    B = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, k)).cuda()
    W = torch.from_numpy(inputs.normal_matrix(seed, n, k)).cuda()
    b0 = B[:, 0].contiguous()
    _, rep100, _, _ = api.mxp_solve(A, b0, prec="bf16", pivot=True, nb=nb, refine="gmres",
                                    restart=100, max_outer=30, max_inner_total=3000,
                                    allow_notconv=True)
    note(f"restart 100: status {rep100['status']}, outer {rep100['outer_iters']}, inner "
         f"{rep100['inner_iters']}, rho {rep100['scaled_residual']:.3e}")
    assert rep100["status"] in (0, -1004)
    assert rep100["outer_iters"] > 0 and rep100["inner_iters"] > 0
    kw = dict(restart=200, max_outer=30, max_inner_total=4000)
    Ar = A.clone().requires_grad_(True)
    Br = B.clone().requires_grad_(True)
    X = ag.solve(Ar, Br, mode="bf16_ir", nb=nb, **kw)
    (X * W).sum().backward()
    torch.cuda.synchronize()
    rho = max(api.scaled_residual(A, X.detach(), B))
    note(f"restart 200, 16 columns: max scaled residual {rho:.3e}")
    assert rho < 16
    A64 = A.clone().requires_grad_(True)
    B64 = B.clone().requires_grad_(True)
    X64 = ag.solve(A64, B64, mode="fp64", nb=nb)
    (X64 * W).sum().backward()
    torch.cuda.synchronize()
    ex = ((X.detach() - X64.detach()).abs().max() / X64.detach().abs().max()).item()
    ea = ((Ar.grad - A64.grad).abs().max() / A64.grad.abs().max()).item()
    eb = ((Br.grad - B64.grad).abs().max() / B64.grad.abs().max()).item()
    note(f"relative differences to the FP64 form: X {ex:.2e}, dA {ea:.2e}, dB {eb:.2e}")
    # rho < 16 on both sides bounds each solution's error by ~16 n eps kappa
    # relative (kappa_inf of this matrix is below 1e6): 16 * 8192 * 1.1e-16
    # * 1e6 = 1.5e-4
    assert ex < 1.5e-4 and ea < 1.5e-4 and eb < 1.5e-4
    rng = np.random.default_rng(1)
    worst = 0.0
    h = 1.0
    for t in range(4):
        i, c = int(rng.integers(0, n)), int(rng.integers(0, k))
        fd = 0.0
        for sgn in (1.0, -1.0):
            bc = B[:, c].clone()
            bc[i] += sgn * h
            xc, rep, _, _ = api.mxp_solve(A, bc, prec="bf16", pivot=True, nb=nb,
                                          refine="gmres", **kw)
            fd += sgn * float((xc * W[:, c]).sum())
        fd /= 2 * h
        g = float(Br.grad[i, c])
        worst = max(worst, abs(fd - g) / max(abs(g), 1e-3 * float(Br.grad.abs().max())))
    note(f"worst relative finite-difference mismatch on B entries {worst:.2e}")
    assert worst <= 1e-3
