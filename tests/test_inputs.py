"""The seeded input generator: published SplitMix64 outputs, value lattice,
and the properties the workloads rely on."""

import numpy as np

from paper_2604_09517_amd import inputs


def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0 emits mix(G), mix(2G), mix(3G), ...
    assert inputs._mix64_int(inputs.GOLDEN) == 0xE220A8397B1DCDAF
    assert inputs._mix64_int(2 * inputs.GOLDEN) == 0x6E789E6AA1B965F4
    assert inputs._mix64_int(3 * inputs.GOLDEN) == 0x06C45D188009454F
    # the vectorised form agrees with the integer form
    z = np.array([inputs.GOLDEN, 2 * inputs.GOLDEN & inputs.MASK64], dtype=np.uint64)
    with np.errstate(over="ignore"):
        got = inputs._mix64_np(z)
    assert int(got[0]) == 0xE220A8397B1DCDAF and int(got[1]) == 0x6E789E6AA1B965F4


def test_uniform_values_on_lattice_and_range():
    a = inputs.uniform_matrix(1000, 0, 300, 200)
    assert a.flags["F_CONTIGUOUS"]
    assert a.min() >= -0.5 and a.max() < 0.5
    k = (a + 0.5) * 2.0 ** 32
    assert np.array_equal(k, np.round(k))
    assert abs(a.mean()) < 0.01 and abs(a.var() - 1 / 12) < 0.005


def test_column_major_index_definition():
    n_rows, n_cols = 37, 5
    a = inputs.uniform_matrix(4, 1, n_rows, n_cols, chunk_cols=2)
    i, j = 11, 3
    assert a[i, j] == inputs.uniform_at(4, 1, np.array([j * n_rows + i]))[0]
    b = inputs.uniform_matrix(4, 2, n_rows, n_cols)
    assert not np.array_equal(a, b)


def test_dominant_diagonal_is_exact_row_sum():
    n = 257
    a = inputs.diag_dominant_matrix(7, 0, n)
    off = a - np.diag(np.diag(a))
    for i in (0, 100, 256):
        s = sum(abs(float(v)) for v in off[i])       # sequential Python sum
        assert a[i, i] == s                           # order does not matter
    assert np.all(np.diag(a) >= np.abs(off).sum(1))


def test_normals_moments():
    w = inputs.normal_matrix(3, 4000, 4)
    assert w.shape == (4000, 4)
    assert abs(w.mean()) < 0.03 and abs(w.std() - 1) < 0.03
