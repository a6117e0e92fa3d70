"""lu_solve_noalloc (no device allocation, library-owned scratch) against
lu_solve, through the C ABI: the same kernels on the same data, so the
results must agree bit for bit.  Two calls in a row, the second on a smaller
system, so the second reuses the scratch the first left behind."""

import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2604_09517_amd import inputs

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2604_09517_amd import api as _api
    _api.lib()
    torch.cuda.set_device(0)
    return _api


def factor(api, n, nb, seed):
    A = api.fortran_empty(n, n)
    api.fill_uniform(A, seed, inputs.STREAM_A)
    _, ipiv, info = api.lu_factor(A, nb)
    assert info == 0
    return A, ipiv


def call_both(api, LU, ipiv, B, trans):
    n = LU.shape[0]
    L = api.lib()
    s = torch.cuda.current_stream().cuda_stream
    X1 = B.clone()
    X2 = B.clone()
    assert L.lu_solve(n, B.shape[1], LU.data_ptr(), LU.stride(1), ipiv.data_ptr(),
                      X1.data_ptr(), X1.stride(1), trans, s) == 0
    assert L.lu_solve_noalloc(n, B.shape[1], LU.data_ptr(), LU.stride(1), ipiv.data_ptr(),
                              X2.data_ptr(), X2.stride(1), trans, s) == 0
    torch.cuda.synchronize()
    return X1.cpu().numpy(), X2.cpu().numpy()


def test_noalloc_solve_matches_lu_solve_twice(api):
    # first call: n = 2000, 20 right-hand sides (two strips), A x = b
    note("no-alloc solve: n=2000 nrhs=20 trans=0")
    LU, ipiv = factor(api, 2000, 128, 41)
    B = api.fortran_empty(2000, 20)
    api.fill_uniform(B, 41, inputs.STREAM_B)
    X1, X2 = call_both(api, LU, ipiv, B, 0)
    assert np.array_equal(X1, X2)
    A_h = inputs.uniform_matrix(41, inputs.STREAM_A, 2000, 2000)
    r = B.cpu().numpy() - A_h @ X2
    assert np.abs(r).max() < 1e-9
    # second call, smaller: n = 300, one right-hand side, A^T x = b
    note("no-alloc solve: n=300 nrhs=1 trans=1")
    LU2, ipiv2 = factor(api, 300, 64, 42)
    B2 = api.fortran_empty(300, 1)
    api.fill_uniform(B2, 42, inputs.STREAM_B)
    X1, X2 = call_both(api, LU2, ipiv2, B2, 1)
    assert np.array_equal(X1, X2)
    A2 = inputs.uniform_matrix(42, inputs.STREAM_A, 300, 300)
    assert np.abs(B2.cpu().numpy() - A2.T @ X2).max() < 1e-10


def test_noalloc_rejects_sizes_beyond_its_scratch(api):
    L = api.lib()
    p = ctypes.c_void_p(16)   # nothing is enqueued: the size check comes first
    assert L.lu_solve_noalloc(65537, 1, p, 65537, p, p, 65537, 0, None) == -1006
    assert b"65536" in L.mxlu_last_error()
    assert L.lu_solve_noalloc(10, 1, p, 9, p, p, 10, 0, None) == -4
