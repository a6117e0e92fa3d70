"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This module holds no arithmetic of the solver: it only turns (seed, stream,
index) into numbers.  The HIP library carries its own device implementation of
the same counter-based generator (written separately from the same published
definition) so that large matrices can be produced in HBM; the GPU tests check
the two bit for bit.

Definition (SplitMix64 finaliser, Steele, Lea & Flood, OOPSLA 2014):

    mix(z)  = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^ (z >> 31)   (mod 2^64)
    key     = mix(seed + G * (stream + 1))            G = 0x9E3779B97F4A7C15
    h(idx)  = mix(key  + G * (idx + 1))
    u(idx)  = (h >> 32) * 2^-32 - 0.5                 exact in FP64, in [-0.5, 0.5)

A matrix element (i, j) of an n_rows x n_cols matrix uses idx = j * n_rows + i
(column-major linear index; independent of any leading dimension).

The paper's workloads use "random entries" (Sec. III-A.1); the uniform
[-0.5, 0.5) law and the diagonally dominant variant (diagonal = sum of the
absolute off-diagonal row entries) are the stated test problems.  Because every
value is a multiple of 2^-32 with magnitude <= 2^-1, any row sum of up to 2^20
such values is exact in FP64 in any order, so host and device agree bitwise.
"""

from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Stream ids: the matrix, the right-hand sides, two streams for normal weights.
STREAM_A = 0
STREAM_B = 1
STREAM_W1 = 2
STREAM_W2 = 3


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def _mix64_int(z: int) -> int:
    z &= MASK64
    z ^= z >> 30
    z = (z * M1) & MASK64
    z ^= z >> 27
    z = (z * M2) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """64-bit key of one (seed, stream) pair."""
    return _mix64_int((seed + GOLDEN * (stream + 1)) & MASK64)


def hash_at(seed: int, stream: int, idx) -> np.ndarray:
    """h(idx) as uint64 for an integer array of linear indices."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64_np(key + np.uint64(GOLDEN) * (idx + np.uint64(1)))


def uniform_at(seed: int, stream: int, idx) -> np.ndarray:
    """u(idx) in [-0.5, 0.5), exact multiples of 2^-32."""
    h = hash_at(seed, stream, idx)
    return (h >> np.uint64(32)).astype(np.float64) * (2.0 ** -32) - 0.5


def uniform_matrix(seed: int, stream: int, n_rows: int, n_cols: int,
                   chunk_cols: int = 4096, threads: int = 1) -> np.ndarray:
    """Column-major (Fortran-ordered) n_rows x n_cols FP64 matrix.  `threads`
    > 1 fills column chunks concurrently (numpy releases the GIL)."""
    out = np.empty((n_rows, n_cols), dtype=np.float64, order="F")
    rows = np.arange(n_rows, dtype=np.uint64)
    if threads > 1:
        chunk_cols = max(1, min(chunk_cols, (1 << 22) // max(1, n_rows)))

    def fill(c0):
        c1 = min(n_cols, c0 + chunk_cols)
        cols = np.arange(c0, c1, dtype=np.uint64)
        idx = cols[None, :] * np.uint64(n_rows) + rows[:, None]
        out[:, c0:c1] = uniform_at(seed, stream, idx)

    starts = range(0, n_cols, chunk_cols)
    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(fill, starts))
    else:
        for c0 in starts:
            fill(c0)
    return out


def diag_dominant_matrix(seed: int, stream: int, n: int) -> np.ndarray:
    """Off-diagonals u(idx); diagonal replaced by the sum of |off-diagonal| of its row."""
    a = uniform_matrix(seed, stream, n, n)
    np.fill_diagonal(a, 0.0)
    d = np.abs(a).sum(axis=1)
    np.fill_diagonal(a, d)
    return a


def normal_matrix(seed: int, n_rows: int, n_cols: int) -> np.ndarray:
    """N(0, 1) weights by Box-Muller (1958) from streams W1 and W2 (host only)."""
    idx = np.arange(n_rows * n_cols, dtype=np.uint64)
    h1 = hash_at(seed, STREAM_W1, idx)
    h2 = hash_at(seed, STREAM_W2, idx)
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)  # (0, 1]
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)          # [0, 1)
    w = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return np.asfortranarray(w.reshape(n_cols, n_rows).T)


def config_seed(config_index: int) -> int:
    """Seed used for workload number `config_index` (matrix stream 0, rhs stream 1)."""
    return 1000 + int(config_index)


# The five workloads: sizes and recipes (see the configuration table in the
# design notes).  `kind` is "uniform" (i.i.d. u) or "dominant".
WORKLOADS = {
    "fp64_small": dict(index=0, n=1024, nb=64, kind="uniform", nrhs=1),
    "fp64_large": dict(index=1, n=32768, nb=256, kind="uniform", nrhs=1),
    "bf16_ir": dict(index=2, n=65536, nb=512, kind="dominant", nrhs=1),
    "fp8_ir": dict(index=3, n=131072, nb=1024, kind="dominant", nrhs=1),
    "autograd": dict(index=4, n=8192, nb=256, kind="uniform", nrhs=16),
}
