"""Planted mistakes: each mutant is a copy of the oracle's C source with one
plausible error (a dropped term, a wrong sign, a transposed index, a wrong
tie-break, a wrong order).  The pins in the other oracle test modules must
fail on every mutant; this shows they constrain the oracle rather than
restate it.  Everything here runs on the CPU."""

import os

import pytest

import oracle
from tests import test_oracle_getrf as G
from tests import test_oracle_lowprec as P

SRC = open(oracle.SRC_PATH).read()

# (name, exact text in the source, replacement, occurrence index)
MUTANTS = [
    ("tie_break_last_index", "if (v > best) { best = v; p = i; }",
     "if (v >= best) { best = v; p = i; }", 0),
    ("panel_rank1_dropped",
     "A[IDX(i, c, lda)] = fma(-A[IDX(i, j, lda)], u, A[IDX(i, c, lda)]);",
     "(void)u;", 0),
    ("trsm_sign", "A[IDX(i, c, lda)] = fma(-A[IDX(i, k, lda)], x, A[IDX(i, c, lda)]);",
     "A[IDX(i, c, lda)] = fma(A[IDX(i, k, lda)], x, A[IDX(i, c, lda)]);", 0),
    ("gemm_transposed_u",
     "double u = A[IDX(k, c, lda)];\n            for (int64_t i = c1; i < n; ++i)",
     "double u = A[IDX(c, k, lda)];\n            for (int64_t i = c1; i < n; ++i)", 0),
    ("gemm_k_range_short", "for (int64_t k = k0; k < c1; ++k) {\n            double u",
     "for (int64_t k = k0; k < c1 - 1; ++k) {\n            double u", 0),
    ("swap_skips_left_columns", "if (c >= k0 && c < k0 + kb) continue;",
     "if (c < k0 + kb) continue;", 0),
    ("getrs_no_interchanges",
     "if (p != j) { double t = b[j]; b[j] = b[p]; b[p] = t; }",
     "(void)p;", 0),
    ("getrs_trans_interchanges_forward",
     "for (int64_t j = n - 1; j >= 0; --j) {     /* x = P^T z */",
     "for (int64_t j = 0; j < n; ++j) {     /* x = P^T z */", 0),
    ("getrs_upper_index",
     "b[i] = fma(-LU[IDX(i, k, lda)], x, b[i]);\n            }\n        } else",
     "b[i] = fma(-LU[IDX(k, i, lda)], x, b[i]);\n            }\n        } else", 0),
    ("round_ties_away", "double y = nearbyint(x / q) * q;", "double y = round(x / q) * q;", 0),
    ("round_bf16_precision", "case ORACLE_BF16: p = 8;", "case ORACLE_BF16: p = 9;", 0),
    ("fp8_scale_not_minimal", "int k = (f == 0.5) ? e2 - 1 : e2;", "int k = e2;", 0),
    ("lp_update_sign", "acc = fmaf(-to_f32(S[IDX(i, k0 + k, lds)]),",
     "acc = fmaf(to_f32(S[IDX(i, k0 + k, lds)]),", 0),
    ("lp_fp8_missing_u_scale", "upd = (float)((double)upd * su);", "upd = upd;", 0),
    ("lp_fp8_neighbour_row_tile_scale", "double sl = sL[(i - c1) / tile];",
     "double sl = sL[(i - c1) / tile > 0 ? (i - c1) / tile - 1 : 1];", 0),
    ("lp_fp8_first_column_tile_scale", "double su = sU[(c - c1) / tile];",
     "double su = sU[0];", 0),
    ("lp_mx_neighbour_block_scale", "sL[(i - c1) * nblk + k / 32]);   /* exact */",
     "sL[(i - c1) * nblk + ((k / 32) ^ 1) % nblk]);", 0),
    ("lp_mx_u_first_block_scale", "sU[(c - c1) * nblk + k / 32]);   /* exact */",
     "sU[(c - c1) * nblk]);", 0),
    ("lp_fp32_storage_rounds_to_fp16",
     "int sfmt = (prec == 0) ? ORACLE_BF16 : (prec == 4) ? ORACLE_FP32 : ORACLE_FP16;",
     "int sfmt = (prec == 0) ? ORACLE_BF16 : (prec == 4) ? ORACLE_FP16 : ORACLE_FP16;", 0),
    ("round_fp32_precision", "case ORACLE_FP32: p = 24;", "case ORACLE_FP32: p = 23;", 0),
    ("lp_trsm_wrong_factor", "uu[i] = fmaf(-P[IDX(i, k, m)], uu[k], uu[i]);",
     "uu[i] = fmaf(-P[IDX(k, i, m)], uu[k], uu[i]);", 0),
    ("precond_no_forward_solve",
     "v[i] = fmaf(-(float)F[IDX(i, k, ldf)], v[k], v[i]);\n        for",
     "(void)v;\n        for", 0),
    ("precond_trans_pivots_forward",
     "for (int64_t j = n - 1; j >= 0; --j) {\n                int64_t p = ipiv[j];\n                if (p != j) { float t",
     "for (int64_t j = 0; j < n; ++j) {\n                int64_t p = ipiv[j];\n                if (p != j) { float t", 0),
]

# The pins run against each mutant (a subset that runs in a second or two).
PINS = [
    lambda: [G.test_pivots_and_factors_match_exact_rational(None, n, s)
             for n in (3, 5, 8) for s in range(4)],
    lambda: G.test_first_pivot_is_first_argmax_on_ties(None),
    lambda: G.test_two_by_two_formula(None),
    lambda: G.test_invariants_and_lapack(None, 64, 8),
    lambda: G.test_invariants_and_lapack(None, 300, 64),
    lambda: G.test_hilbert_inverse_closed_form(None, 5),
    lambda: [P.test_rounding_matches_torch_casts_on_fp32_inputs(None, f)
             for f in ("bf16", "fp16", "e4m3")],
    lambda: P.test_fp8_scale_is_minimal_power_of_two(None),
    lambda: [P.test_lp_lu_reproduces_exact_factors(None, p) for p in (0, 1)],
    lambda: P.test_fp32_rounding_is_the_ieee_cast(None),
    lambda: P.test_lp_lu_backward_error_bound(None, 4, 2.0 ** -24),
    lambda: P.test_lp_lu_fp8_update_exact_on_representable_operands(None),
    lambda: [P.test_lp_lu_fp8_distinct_tile_scales_exact(None, n, nb, t)
             for n, nb, t in ((24, 8, 4), (40, 16, 8), (36, 12, 12))],
    lambda: [P.test_lp_lu_mx_block_scales_exact(None, n, nb) for n, nb in ((96, 64), (160, 128))],
    lambda: P.test_lp_lu_pivoted_recovers_permutation(None),
    lambda: P.test_preconditioner_solves_with_factors_and_adjoint(None),
    lambda: P.test_preconditioner_with_pivots_and_exact_factors(None),
]


def test_mutations_apply_cleanly():
    for name, old, new, occ in MUTANTS:
        assert SRC.count(old) >= occ + 1, name


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new, occ):
    pos = -1
    for _ in range(occ + 1):
        pos = SRC.index(old, pos + 1)
    mutated = SRC[:pos] + new + SRC[pos + len(old):]
    src = tmp_path / "mutant.c"
    src.write_text(mutated)
    lib_path = str(tmp_path / "libmutant.so")
    oracle.build_variant(str(src), lib_path)
    saved = oracle.load(lib_path)
    caught = []
    try:
        for k, pin in enumerate(PINS):
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError, IndexError):
                caught.append(k)
    finally:
        oracle.restore(saved)
    assert caught, f"no pin failed for mutant {name}"
