"""GPU parity of the mixed-precision path (Sec. III-A.2: low-precision LU
without pivoting and FP64 refinement; Sec. II-B: GMRES-based refinement)
against the CPU oracle, through the C ABI.

What is compared, and how:
  * conversion FP64 -> bf16/fp16: bit for bit;
  * factors: the first panel step (panel and U12 block row, FP32 arithmetic in
    the same operation order) bit for bit; after one panel step every entry
    of the updated trailing block within one storage ulp (same operands, only
    the FP32 summation order differs); the whole factorization within a
    componentwise bound of two summation orders, and the backward error
    ||LU - A|| / ||A|| within 4 u (u = 2^-8 bf16, 2^-11 fp16, 2^-4 for the
    FP8 update); FP8 at nb 128, 256 and 1024 (1, 2 and 8 K chunks in the
    update kernel) and on inputs whose scale tiles all differ;
  * preconditioner M b on identical (oracle) factors: bit for bit;
  * solves: the HPL scaled residual < 16 (the acceptance threshold), the
    forward error against the FP64 oracle solution within the bound that
    rho < 16 implies, iteration counts close to the oracle refinement's.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import checks, refine
from paper_2604_09517_amd import inputs

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53
U_LP = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp8": 2.0 ** -4, "fp8_mx": 2.0 ** -4,
        "fp32": 2.0 ** -24}
PREC_ID = {"bf16": 0, "fp16": 1, "fp8": 2, "fp8_mx": 3, "fp32": 4}


@pytest.fixture(scope="module")
def api():
    from paper_2604_09517_amd import api as _api
    _api.lib()
    torch.cuda.set_device(0)
    return _api


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a, ld=None):
    from paper_2604_09517_amd import api as _api
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    t = _api.fortran_empty(a.shape[0], a.shape[1], ld=ld)
    t.copy_(torch.from_numpy(a))
    return t


def factors_to_host(api, work, n, prec):
    return api.mxp_factors(work, n, prec).to(torch.float64).cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_convert_bitwise(api, prec):
    rng = np.random.default_rng(1)
    rows, cols = 300, 7
    A = rng.standard_normal((rows, cols)) * 2.0 ** rng.integers(-30, 20, (rows, cols))
    A[0, 0] = 1.0 + 2.0 ** -8 + 2.0 ** -40      # above a bf16 halfway point
    A[1, 0] = 1.0 + 2.0 ** -8                    # exact halfway: ties to even
    A[2, 0] = 65520.0                            # fp16 overflow to inf
    A[3, 0] = 2.0 ** -25 * 3                     # fp16 subnormal rounding
    out = api.mxp_convert(to_dev(A, ld=rows + 3), prec)
    torch.cuda.synchronize()
    got = out.to(torch.float64).cpu().numpy()
    ref = oracle.round_lp(A, oracle.BF16 if prec == "bf16" else oracle.FP16)
    assert np.array_equal(got, ref)


def run_mxp(api, A_h, b_h, **kw):
    dA = to_dev(A_h)
    db = to_dev(b_h)
    X, rep, work, ipiv = api.mxp_solve(dA, db, allow_notconv=True, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), rep, work, dA


def tile_scaled(A, tile):
    """D_r A D_c with power-of-two factors constant on each tile of `tile`
    rows (columns) and different between neighbouring tiles.  The no-pivot
    LU of the result is D_r L D_r^-1 times D_r U D_c (exact scalings), so the
    factorization is as stable as A's, while the FP8 tile scales of L21 rows
    and U12 columns differ from tile to tile."""
    n = A.shape[0]
    kr = np.array([(i // tile) % 5 - 2 for i in range(n)], dtype=np.float64)
    kc = np.array([2 - (j // tile) % 5 for j in range(n)], dtype=np.float64)
    return (2.0 ** kr)[:, None] * A * (2.0 ** kc)[None, :]


def lp_input(kind, n, seed, tile=128, l21_boost=0, nb=0):
    A = inputs.diag_dominant_matrix(seed, 0, n)
    if l21_boost:
        # larger multipliers below the first panel (a power of two, exact):
        # the first trailing update then moves A22 by much more than a
        # storage ulp, so a dropped or misplaced term shows at once
        A[nb:, :nb] *= 2.0 ** l21_boost
    if kind == "scaled":
        A = tile_scaled(A, tile)
    return A


def ordered_bits(F, prec):
    """Storage words of F (FP64 holding storage values) as integers ordered
    like the values: adjacent representable numbers differ by 1."""
    dt = torch.bfloat16 if prec == "bf16" else torch.float16
    w = torch.from_numpy(np.ascontiguousarray(F)).to(dt).view(torch.int16).numpy()
    w = w.astype(np.int64) & 0xFFFF
    mag = w & 0x7FFF
    return np.where(w & 0x8000, -mag, mag)


def componentwise_bound(A, F_ref, nb, prec):
    """Bound on |F - F_ref| for two executions of the same blocked algorithm
    that differ only in the FP32 summation order of the trailing updates.
    Each update step can move a stored Schur-complement entry by one storage
    rounding (u_s |value|), and a changed stored operand changes later update
    terms l_ik u_kj by a relative u_s -- by one e4m3 step (2^-3) when the FP8
    quantisation of the changed operand flips.  Summed over the steps that
    touch entry (i, j):
      |dF_ij| <= 4 s_ij (u_s (|F_ij| + |A_ij|) + u_q (|L||U|)'_ij)
    with s_ij = min(i, j) // nb + 1 and (|L||U|)' the sum over k < min(i, j)
    of |l_ik| |u_kj| (the update terms)."""
    n = A.shape[0]
    L, U = checks.unpack_lu(F_ref)
    aL, aU = np.abs(L), np.abs(U)
    full = aL @ aU
    last = np.where(np.tri(n, dtype=bool), aL * np.diag(aU)[None, :], aU)
    upd = full - last
    us = U_LP["bf16"] if prec == "bf16" else U_LP["fp16"]
    uq = 2.0 ** -3 if prec.startswith("fp8") else us
    steps = np.minimum.outer(np.arange(n), np.arange(n)) // nb + 1
    return 4 * steps * (us * (np.abs(F_ref) + np.abs(A)) + uq * upd)


@pytest.mark.parametrize("prec,n,nb,kind,tile", [
    ("bf16", 256, 64, "dominant", 64), ("fp16", 300, 64, "dominant", 64),
    ("bf16", 640, 128, "dominant", 64), ("fp8", 512, 128, "dominant", 64),
    ("fp8", 700, 128, "dominant", 64), ("fp8", 680, 256, "dominant", 128),
    ("fp8", 2216, 1024, "dominant", 128), ("fp8", 500, 128, "scaled", 12),
    ("fp8", 680, 256, "scaled", 128), ("bf16", 680, 256, "scaled", 128),
    ("fp8_mx", 700, 128, "dominant", 32), ("fp8_mx", 680, 256, "scaled", 32),
    ("fp8_mx", 2216, 1024, "scaled", 32)])
def test_lp_factors_against_oracle(api, prec, n, nb, kind, tile):
    """Whole factorization: first panel and block row bit for bit, every
    other entry within the componentwise bound of two summation orders."""
    note(f"lp factors prec={prec} n={n} nb={nb} input={kind} tile={tile}")
    A = lp_input(kind, n, 31 + n, tile)
    b = inputs.uniform_matrix(31 + n, 1, n, 1)[:, 0]
    _, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, max_outer=0, scale_tile=tile)
    F = factors_to_host(api, work, n, prec)
    F_ref, _, info = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=tile)
    assert rep["info"] == info == 0
    # first panel and first block row: FP32 arithmetic in the same order
    assert np.array_equal(F[:, :nb], F_ref[:, :nb])
    assert np.array_equal(F[:nb, :], F_ref[:nb, :])
    d = np.abs(F - F_ref)
    bound = componentwise_bound(A, F_ref, nb, prec)
    worst = np.unravel_index(np.argmax(d / np.maximum(bound, 1e-300)), d.shape)
    note(f"  entries differing {(d > 0).sum()}, max |dF| {d.max():.3e}, "
         f"worst ratio to bound {d[worst] / bound[worst]:.3f} at {worst}")
    assert np.all(d <= bound)
    u = U_LP[prec]
    L, U = checks.unpack_lu(F)
    err = np.abs(L @ U - A).sum(1).max() / np.abs(A).sum(1).max()
    assert err <= 4 * u


@pytest.mark.parametrize("prec,n,nb,kind,tile,steps", [
    ("bf16", 2216, 512, "dominant", 128, 0), ("fp16", 1100, 256, "dominant", 64, 0),
    ("fp16", 700, 128, "dominant", 64, 0),
    ("bf16", 1064, 256, "scaled", 128, 2), ("fp8", 2216, 1024, "dominant", 128, 0),
    ("fp8", 1064, 256, "scaled", 128, 0), ("fp8", 1064, 256, "scaled", 64, 3),
    ("fp8", 500, 128, "scaled", 12, 0), ("fp8_mx", 2216, 1024, "scaled", 32, 0),
    ("fp8_mx", 1064, 256, "scaled", 32, 2)])
def test_lp_lookahead_equals_depth0(api, prec, n, nb, kind, tile, steps):
    """Look-ahead depth 1 (the next panel factored on a second stream while
    the rest of the update runs) gives the same factors as depth 0 bit for
    bit: the update is split at a tile boundary, so every element takes the
    same operations in the same order.  Covers a ragged last panel (n = 2216,
    nb = 1024: the last update is narrower than a panel), factorizations
    stopped after a few steps (the panel after the last step stays
    unfactored), and a scale tile that does not divide nb or a 16-bit panel
    narrower than the 256-row tile (depth 0 is used)."""
    note(f"look-ahead vs depth 0 prec={prec} n={n} nb={nb} input={kind} tile={tile} "
         f"steps={steps}")
    A = lp_input(kind, n, 91 + n, tile)
    b = inputs.uniform_matrix(91 + n, 1, n, 1)[:, 0]
    got = []
    try:
        for depth in (0, 1):
            api.set_lookahead(depth)
            _, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, max_outer=0,
                                      scale_tile=tile, factor_steps=steps)
            got.append(api.mxp_factors(work, n, prec).cpu().clone())
            assert rep["info"] == 0
    finally:
        api.set_lookahead(1)
    assert torch.equal(got[0].view(torch.int16), got[1].view(torch.int16))
    if steps:   # the block after the last step is the updated, unfactored Schur complement
        F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=tile,
                                      max_steps=steps)
        F = got[1].to(torch.float64).numpy()
        assert np.all(np.abs(F - F_ref) <= componentwise_bound(A, F_ref, nb, prec))


@pytest.mark.parametrize("prec,n,nb,kind,tile", [
    ("bf16", 680, 256, "dominant", 128), ("fp16", 700, 128, "dominant", 64),
    ("bf16", 2216, 512, "dominant", 128),
    ("fp8", 700, 128, "dominant", 64), ("fp8", 680, 256, "dominant", 128),
    ("fp8", 2216, 1024, "dominant", 128), ("fp8", 500, 128, "scaled", 12),
    ("fp8", 1064, 256, "scaled", 128), ("fp8", 1064, 256, "scaled", 36),
    ("fp8_mx", 700, 128, "dominant", 32), ("fp8_mx", 1064, 256, "scaled", 32),
    ("fp8_mx", 2216, 1024, "scaled", 32)])
def test_lp_one_update_within_one_ulp(api, prec, n, nb, kind, tile):
    """One panel step (partial factorization): the panel and U12 bit for bit,
    and every updated entry of the trailing block within one storage ulp of
    the oracle's -- the operands are identical, so only the FP32 summation
    order differs, and with FP8 operands the products and their partial sums
    are mostly exact in FP32.  nb 256 and 1024 run the FP8 update's K loop
    over 2 and 8 chunks; the scaled inputs give every scale tile its own
    power-of-two scale (tile 12: rows of one lane's 8-row group fall into two
    scale tiles)."""
    note(f"one update prec={prec} n={n} nb={nb} input={kind} tile={tile}")
    A = lp_input(kind, n, 57 + n, tile, l21_boost=4, nb=nb)
    b = inputs.uniform_matrix(57 + n, 1, n, 1)[:, 0]
    _, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, max_outer=0, scale_tile=tile,
                              factor_steps=1)
    F = factors_to_host(api, work, n, prec)
    F_ref, _, info = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=tile, max_steps=1)
    assert rep["info"] == info == 0
    assert np.array_equal(F[:, :nb], F_ref[:, :nb])
    assert np.array_equal(F[:nb, :], F_ref[:nb, :])
    A22, R22 = F[nb:, nb:], F_ref[nb:, nb:]
    diff = np.abs(ordered_bits(A22, prec) - ordered_bits(R22, prec))
    # the update is not trivially small: it moved most entries by many ulps
    sfmt = oracle.BF16 if prec == "bf16" else oracle.FP16
    S22 = oracle.round_lp(A[nb:, nb:], sfmt)
    moved = np.abs(ordered_bits(R22, prec) - ordered_bits(S22, prec))
    # where the update cancels to a result far below its terms, two FP32
    # summation orders may differ by more than one storage ulp: there the
    # difference stays within the FP32 dot-product bound 2 gamma_K T,
    # T = |a_ij| + sum_k |l_ik u_kj|, gamma_K = K 2^-24 (plus one ulp)
    T = np.abs(S22) + np.abs(F_ref[nb:, :nb]) @ np.abs(F_ref[:nb, nb:])
    ulp = np.abs(R22) * (2.0 ** -7 if prec == "bf16" else 2.0 ** -10) + 2.0 ** -24
    cancel_ok = np.abs(A22 - R22) <= 2 * nb * 2.0 ** -24 * T + ulp
    note(f"  entries off by one ulp {(diff == 1).sum()}, by more (cancellation) "
         f"{(diff > 1).sum()} of {diff.size}; median ulps moved by the update "
         f"{np.median(moved):.0f}")
    assert np.median(moved) >= 4
    assert np.all((diff <= 1) | cancel_ok)


@pytest.mark.parametrize("prec,trans", [("bf16", 0), ("fp16", 0), ("bf16", 1)])
def test_preconditioner_bitwise_on_oracle_factors(api, prec, trans):
    n, nb = 600, 64
    A = inputs.diag_dominant_matrix(77, 0, n)
    b = inputs.uniform_matrix(77, 1, n, 1)[:, 0]
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False)
    dA, db = to_dev(A), to_dev(b)
    opts = api.mxp_options(prec=prec, nb=nb, max_outer=0, reuse_factors=True, trans=bool(trans))
    work = torch.zeros(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8, device="cuda")
    api.mxp_factors(work, n, prec).copy_(torch.from_numpy(F_ref).to(
        torch.bfloat16 if prec == "bf16" else torch.float16))
    X, rep, _, _ = api.mxp_solve(dA, db, work=work, opts=opts, allow_notconv=True)
    torch.cuda.synchronize()
    x0 = X.cpu().numpy()
    ref = oracle.lp_precond(F_ref, None, b, trans=bool(trans))
    if trans == 0:
        assert np.array_equal(x0, ref)
    else:
        assert np.abs(x0 - ref).max() <= 1e-5 * np.abs(ref).max()


def test_preconditioner_bitwise_outside_the_reciprocal_range(api):
    """The U solve's diagonal steps divide through a reciprocal only while
    every value is in the normal range; with some diagonal entries of U scaled
    by 2^110 (exact in BF16) the quotients of those rows fall below 2^-99, so
    their 64-row sub-blocks are solved again with the division -- and the
    preconditioner is still the oracle's bit for bit."""
    n, nb = 600, 64
    A = inputs.diag_dominant_matrix(78, 0, n)
    b = inputs.uniform_matrix(78, 1, n, 1)[:, 0]
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID["bf16"], pivot=False)
    F = F_ref.copy()
    for k in (3, 64, 130, 200, 300, 450, 599):
        F[k, k] *= 2.0 ** 110
    dA, db = to_dev(A), to_dev(b)
    opts = api.mxp_options(prec="bf16", nb=nb, max_outer=0, reuse_factors=True)
    work = torch.zeros(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8, device="cuda")
    api.mxp_factors(work, n, "bf16").copy_(torch.from_numpy(F).to(torch.bfloat16))
    X, rep, _, _ = api.mxp_solve(dA, db, work=work, opts=opts, allow_notconv=True)
    torch.cuda.synchronize()
    x0 = X.cpu().numpy()
    ref = oracle.lp_precond(F, None, b)
    assert np.all(np.isfinite(ref)) and np.abs(ref[[3, 130, 450]]).max() < 2.0 ** -99
    assert np.array_equal(x0, ref)


@pytest.mark.parametrize("prec,method,n,nb", [
    ("bf16", "gmres", 512, 128), ("bf16", "classical", 512, 128), ("fp16", "gmres", 777, 64),
    ("fp8", "gmres", 1024, 128), ("bf16", "gmres", 2048, 256), ("fp8", "classical", 640, 128),
    ("fp8_mx", "gmres", 1024, 128), ("fp8_mx", "classical", 896, 256)])
def test_mxp_solve_matches_oracle(api, prec, method, n, nb):
    note(f"mxp_solve prec={prec} refine={method} n={n} nb={nb}")
    seed = inputs.config_seed(2) + n
    A = inputs.diag_dominant_matrix(seed, 0, n)
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    x, rep, work, _ = run_mxp(api, A, b, prec=prec, nb=nb, refine=method, scale_tile=128)
    assert rep["status"] == 0 and rep["converged"] == 1
    rho = checks.scaled_residual(A, x, b)
    assert rho < 16 and rep["scaled_residual"] < 16
    # oracle: the same algorithm on the oracle's factors
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=128)
    out = refine.refine(A, b, F_ref, None, method=method)
    assert out["converged"]
    LU, ipiv, _ = oracle.getrf(A, nb)
    x64 = oracle.getrs(LU, ipiv, b)
    kappa = np.linalg.cond(A, np.inf)
    fe = checks.forward_error(x, x64)
    note(f"  outer {rep['outer_iters']} (oracle {out['outer_iters']}), inner "
         f"{rep['inner_iters']} (oracle {out['inner_iters']}), rho {rho:.2f}, fwd err {fe:.2e}")
    assert abs(rep["outer_iters"] - out["outer_iters"]) <= 1
    # GMRES: each cycle may end one Arnoldi step earlier or later (its stopping
    # test compares a rounding-sensitive estimate with inner_tol * beta)
    assert abs(rep["inner_iters"] - out["inner_iters"]) <= out["outer_iters"] + 1
    assert fe < 4 * 16 * n * EPS * kappa


@pytest.mark.parametrize("prec,n,nb,tile", [("fp8", 896, 128, 12), ("bf16", 1000, 256, 128)])
def test_mxp_solve_tile_scaled_matrix(api, prec, n, nb, tile):
    """A harder system for the refinement: the tile-scaled matrix has
    condition number about 2^8 times that of the dominant matrix, and its
    FP8 factors carry a different scale on every tile."""
    seed = 71 + n
    A = lp_input("scaled", n, seed, tile)
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    x, rep, _, _ = run_mxp(api, A, b, prec=prec, nb=nb, refine="gmres", scale_tile=tile)
    F_ref, _, _ = oracle.lp_getrf(A, nb, PREC_ID[prec], pivot=False, tile=tile)
    out = refine.refine(A, b, F_ref, None, method="gmres")
    rho = checks.scaled_residual(A, x, b)
    note(f"tile-scaled {prec} n={n}: outer {rep['outer_iters']} (oracle {out['outer_iters']}), "
         f"inner {rep['inner_iters']} (oracle {out['inner_iters']}), rho {rho:.2f}")
    assert out["converged"] and rep["converged"] == 1 and rho < 16
    assert abs(rep["outer_iters"] - out["outer_iters"]) <= 1
    assert abs(rep["inner_iters"] - out["inner_iters"]) <= out["outer_iters"] + 1


def test_mxp_transposed_and_multiple_rhs(api):
    n, nb = 500, 64
    A = inputs.diag_dominant_matrix(5, 0, n)
    B = inputs.uniform_matrix(5, 1, n, 3)
    dA, dB = to_dev(A), to_dev(B)
    X, rep, work, _ = api.mxp_solve(dA, dB, prec="bf16", nb=nb)
    torch.cuda.synchronize()
    assert rep["converged"] == 1
    assert checks.scaled_residual(A, X.cpu().numpy(), B) < 16
    # A^T X = B with the same factors
    Xt, rep2, _, _ = api.mxp_solve(dA, dB, work=work, prec="bf16", nb=nb, trans=True,
                                   reuse_factors=True)
    torch.cuda.synchronize()
    assert rep2["converged"] == 1
    assert checks.scaled_residual(A.T, Xt.cpu().numpy(), B) < 16


def test_mxp_nonconvergence_reported(api):
    n = 256
    A = inputs.diag_dominant_matrix(9, 0, n)
    b = inputs.uniform_matrix(9, 1, n, 1)[:, 0]
    _, rep, _, _ = run_mxp(api, A, b, prec="bf16", nb=64, refine="classical", max_outer=0)
    assert rep["status"] == -1004 and rep["converged"] == 0
    assert rep["outer_iters"] == 0 and rep["scaled_residual"] >= 16


def test_mxp_argument_errors(api):
    dA = api.fortran_empty(64, 64)
    db = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        api.mxp_solve(dA, db, nb=48)          # not a multiple of 32
    with pytest.raises(ValueError):
        api.mxp_solve(dA, db, prec="fp8", nb=64)   # FP8 needs nb % 128 == 0
    opts = api.mxp_options(nb=64)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        api.mxp_solve(dA, db, work=small, opts=opts)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_bf16_configuration(api):
    """N = 65536 diagonally dominant, BF16 storage, NB = 512, GMRES-IR."""
    cfg = inputs.WORKLOADS["bf16_ir"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size bf16 n={n} nb={nb}")
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    api.make_diag_dominant(dA)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    X, rep, work, _ = api.mxp_solve(dA, db, prec="bf16", nb=nb, refine="gmres")
    torch.cuda.synchronize()
    note(f"report {rep}")
    assert rep["converged"] == 1 and rep["info"] == 0
    rho = api.scaled_residual(dA, X, db)[0]
    note(f"independent scaled residual {rho:.3e}")
    assert rho < 16
    # sampled rows: x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii on the host
    x = X.cpu().numpy()
    b = db.cpu().numpy()
    for i in (0, 1, 4097, n - 1):
        arow = inputs.uniform_at(seed, inputs.STREAM_A,
                                 np.arange(n, dtype=np.uint64) * np.uint64(n) + np.uint64(i))
        arow[i] = np.abs(arow).sum() - np.abs(arow[i])
        r_i = b[i] - arow @ x
        assert abs(r_i) <= 16 * EPS * n * (np.abs(arow).sum() * np.abs(x).max() + np.abs(b).max())


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_fp8_configuration(api):
    """N = 131072 diagonally dominant, FP8 e4m3 updates with per-tile scales,
    FP16 storage, NB = 1024, GMRES-IR: converged, independent scaled residual
    and sampled rows below the threshold, and the seeded form (A regenerated
    inside the conversion and every residual, no FP64 copy) gives the same X
    bit for bit."""
    cfg = inputs.WORKLOADS["fp8_ir"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size fp8 n={n} nb={nb}")
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    api.make_diag_dominant(dA)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    X, rep, work, _ = api.mxp_solve(dA, db, prec="fp8", nb=nb, refine="gmres", scale_tile=128)
    torch.cuda.synchronize()
    note(f"report {rep}")
    assert rep["converged"] == 1 and rep["info"] == 0
    rho = api.scaled_residual(dA, X, db)[0]
    note(f"independent scaled residual {rho:.3e}")
    assert rho < 16
    x = X.cpu().numpy()
    b = db.cpu().numpy()
    for i in (0, 1, 65537, n - 1):
        arow = inputs.uniform_at(seed, inputs.STREAM_A,
                                 np.arange(n, dtype=np.uint64) * np.uint64(n) + np.uint64(i))
        arow[i] = np.abs(arow).sum() - np.abs(arow[i])
        r_i = b[i] - arow @ x
        assert abs(r_i) <= 16 * EPS * n * (np.abs(arow).sum() * np.abs(x).max() + np.abs(b).max())
    del dA
    torch.cuda.empty_cache()
    Xs, reps, _, _ = api.mxp_solve_seeded(n, seed, inputs.STREAM_A, db, dominant=True, work=work,
                                          prec="fp8", nb=nb, refine="gmres", scale_tile=128)
    torch.cuda.synchronize()
    note(f"seeded report {reps}")
    assert reps["outer_iters"] == rep["outer_iters"] and reps["inner_iters"] == rep["inner_iters"]
    assert torch.equal(Xs, X)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_full_size_fp8_lookahead_equals_depth0(api):
    """N = 131072, NB = 1024 FP8 factorization: look-ahead depth 1 (the next
    panel factored on a second stream) gives the depth-0 factors bit for bit
    at full size, where the panel's leaves run hundreds of workgroups.  (A
    leaf that let one workgroup write the factored diagonal block back while
    others might still read it flipped a few hundred FP16 entries by one unit
    here once the panel's workgroups were scheduled differently.)"""
    cfg = inputs.WORKLOADS["fp8_ir"]
    n, nb, seed = cfg["n"], cfg["nb"], inputs.config_seed(cfg["index"])
    note(f"full size fp8 look-ahead vs depth 0 n={n} nb={nb}")
    dA = api.fortran_empty(n, n)
    api.fill_uniform(dA, seed, inputs.STREAM_A)
    api.make_diag_dominant(dA)
    db = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    opts = api.mxp_options(prec="fp8", nb=nb, scale_tile=128, max_outer=0)
    work = torch.empty(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8, device="cuda")
    F0 = None
    try:
        for depth in (0, 1):
            api.set_lookahead(depth)
            _, rep, work, _ = api.mxp_solve(dA, db, work=work, opts=opts, allow_notconv=True)
            torch.cuda.synchronize()
            assert rep["info"] == 0
            F = api.mxp_factors(work, n, "fp8").view(torch.int16)
            if F0 is None:
                F0 = F.clone()
    finally:
        api.set_lookahead(1)
    del dA
    torch.cuda.empty_cache()
    differ = 0
    for j0 in range(0, n, 8192):   # column slabs bound the temporaries
        differ += int((F[:, j0:j0 + 8192] != F0[:, j0:j0 + 8192]).sum())
    note(f"  entries differing: {differ}")
    assert differ == 0


def test_lp_pivoted_first_panel_matches_oracle(api):
    """Partial pivoting on FP32 panel values: the first panel (same FP32
    operation order) gives the oracle's pivots and values bit for bit."""
    n, nb = 320, 64
    A = inputs.uniform_matrix(91, 0, n, n)
    b = inputs.uniform_matrix(91, 1, n, 1)[:, 0]
    dA, db = to_dev(A), to_dev(b)
    X, rep, work, ipiv = api.mxp_solve(dA, db, prec="bf16", pivot=True, nb=nb, max_outer=0,
                                       allow_notconv=True)
    torch.cuda.synchronize()
    F = factors_to_host(api, work, n, "bf16")
    F_ref, piv_ref, info = oracle.lp_getrf(A, nb, 0, pivot=True)
    piv = ipiv.cpu().numpy()
    assert rep["info"] == info == 0
    assert np.array_equal(piv[:nb], piv_ref[:nb])
    # later panels may legitimately pick other pivots (their inputs passed
    # through the MFMA update) and move the first panel's rows differently:
    # compare the first panel row by row of the original matrix
    by_orig = np.empty_like(F[:, :nb])
    by_orig[checks.perm_from_ipiv(piv, n)] = F[:, :nb]
    by_orig_ref = np.empty_like(F_ref[:, :nb])
    by_orig_ref[checks.perm_from_ipiv(piv_ref, n)] = F_ref[:, :nb]
    assert np.array_equal(by_orig, by_orig_ref)
    # whole factorization: a valid interchange sequence and a small backward error
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    p = checks.perm_from_ipiv(piv, n)
    L, U = checks.unpack_lu(F)
    err = np.abs(L @ U - A[p, :]).sum(1).max() / np.abs(A).sum(1).max()
    assert err <= 64 * U_LP["bf16"]


@pytest.mark.parametrize("n,nb", [(512, 128), (1000, 64)])
def test_mxp_pivoted_solve_uniform_matrix(api, n, nb):
    A = inputs.uniform_matrix(93 + n, 0, n, n)
    b = inputs.uniform_matrix(93 + n, 1, n, 1)[:, 0]
    x, rep, work, _ = run_mxp(api, A, b, prec="bf16", pivot=True, nb=nb, refine="gmres",
                              restart=100, max_outer=30, max_inner_total=1000)
    note(f"pivoted bf16 n={n}: {rep}")
    assert rep["converged"] == 1
    assert checks.scaled_residual(A, x, b) < 16


@pytest.mark.parametrize("prec,n,nb,pivot,dominant,trans", [
    ("bf16", 1500, 128, False, True, 0), ("fp8", 1100, 128, False, True, 0),
    ("bf16", 900, 64, False, True, 1), ("bf16", 700, 64, True, False, 0),
    ("fp32", 800, 64, False, True, 0)])
def test_seeded_solve_equals_stored_matrix(api, prec, n, nb, pivot, dominant, trans):
    """mxp_solve_seeded regenerates A from its counter in the conversion and
    in every FP64 residual; the operations and their order are those of
    mxp_solve on the stored matrix, so factors, solution and counts agree
    bit for bit."""
    seed = 5000 + n
    note(f"seeded solve prec={prec} n={n} pivot={pivot} dominant={dominant} trans={trans}")
    A = api.fortran_empty(n, n)
    api.fill_uniform(A, seed, inputs.STREAM_A)
    if dominant:
        api.make_diag_dominant(A)
    b = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    kw = dict(prec=prec, nb=nb, pivot=pivot, refine="gmres", trans=bool(trans), scale_tile=128,
              restart=100 if pivot else 30, max_outer=30, max_inner_total=1000)
    X1, r1, w1, p1 = api.mxp_solve(A, b, allow_notconv=True, **kw)
    X2, r2, w2, p2 = api.mxp_solve_seeded(n, seed, inputs.STREAM_A, b, dominant=dominant,
                                          allow_notconv=True, **kw)
    torch.cuda.synchronize()
    note(f"  stored: {r1['outer_iters']}/{r1['inner_iters']} rho {r1['scaled_residual']:.3e}; "
         f"seeded: {r2['outer_iters']}/{r2['inner_iters']} rho {r2['scaled_residual']:.3e}")
    assert r1["status"] == r2["status"] == 0
    assert (r1["outer_iters"], r1["inner_iters"]) == (r2["outer_iters"], r2["inner_iters"])
    assert r1["scaled_residual"] == r2["scaled_residual"]
    assert torch.equal(api.mxp_factors(w1, n, prec), api.mxp_factors(w2, n, prec))
    if pivot:
        assert torch.equal(p1, p2)
    assert torch.equal(X1, X2)
    rho = api.scaled_residual(A, X2, b, trans=bool(trans))[0]
    assert rho < 16


@pytest.mark.parametrize("n,nb,pivot", [(300, 64, False), (700, 128, False), (1100, 256, False),
                                        (520, 64, True), (900, 128, True)])
def test_fp32_storage_factors_bitwise(api, n, nb, pivot):
    """FP32 factor storage: panel, TRSM and trailing update take the oracle's
    operations in the oracle's order (one fused multiply-add per term, k
    ascending, nothing rounded to a narrower format), so the whole
    factorization -- and with pivoting every interchange -- is bit for bit
    the oracle's.  Pivoted cases use the uniform (not dominant) matrix."""
    note(f"fp32 storage n={n} nb={nb} pivot={pivot}")
    seed = 91 + n
    A = (inputs.uniform_matrix(seed, 0, n, n) if pivot
         else inputs.diag_dominant_matrix(seed, 0, n))
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    dA, db = to_dev(A), to_dev(b)
    X, rep, work, ipiv = api.mxp_solve(dA, db, prec="fp32", nb=nb, pivot=pivot, max_outer=0,
                                       allow_notconv=True)
    torch.cuda.synchronize()
    F = factors_to_host(api, work, n, "fp32")
    F_ref, ipiv_ref, info = oracle.lp_getrf(A, nb, 4, pivot=pivot)
    assert rep["info"] == info == 0
    if pivot:
        assert np.array_equal(ipiv.cpu().numpy(), ipiv_ref)
    assert np.array_equal(F, F_ref)


@pytest.mark.parametrize("n,nb,steps,pivot", [(3200, 128, 1, False), (3200, 96, 1, False),
                                               (3400, 256, 2, False), (3200, 128, 1, True)])
def test_fp32_matrix_core_update_bitwise(api, n, nb, steps, pivot):
    """The FP32 trailing update at sizes that take the matrix-core GEMM
    (v_mfma_f32_16x16x4f32, four fused multiply-adds in ascending k per
    instruction): after `steps` panel steps the whole partial factorization is
    bit for bit the oracle's."""
    note(f"fp32 matrix-core update n={n} nb={nb} steps={steps} pivot={pivot}")
    seed = 313 + n + nb
    A = (inputs.uniform_matrix(seed, 0, n, n) if pivot
         else inputs.diag_dominant_matrix(seed, 0, n))
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    X, rep, work, ipiv = api.mxp_solve(to_dev(A), to_dev(b), prec="fp32", nb=nb, pivot=pivot,
                                       max_outer=0, factor_steps=steps, allow_notconv=True)
    torch.cuda.synchronize()
    F = factors_to_host(api, work, n, "fp32")
    F_ref, ipiv_ref, info = oracle.lp_getrf(A, nb, 4, pivot=pivot, max_steps=steps)
    assert rep["info"] == info == 0
    if pivot:
        k = steps * nb
        assert np.array_equal(ipiv.cpu().numpy()[:k], ipiv_ref[:k])
    assert np.array_equal(F, F_ref)


@pytest.mark.parametrize("pivot", [False, True])
def test_fp32_storage_preconditioner_bitwise(api, pivot):
    """x0 = M b from FP32 factors: the block solves take every term in the
    substitution's order (k ascending for L, descending for U, then the
    division), so x0 equals the oracle's preconditioner bit for bit."""
    n, nb = 650, 64
    A = (inputs.uniform_matrix(83, 0, n, n) if pivot else inputs.diag_dominant_matrix(83, 0, n))
    b = inputs.uniform_matrix(83, 1, n, 1)[:, 0]
    F_ref, ipiv_ref, _ = oracle.lp_getrf(A, nb, 4, pivot=pivot)
    dA, db = to_dev(A), to_dev(b)
    opts = api.mxp_options(prec="fp32", nb=nb, pivot=pivot, max_outer=0, reuse_factors=True)
    work = torch.zeros(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8, device="cuda")
    api.mxp_factors(work, n, "fp32").copy_(torch.from_numpy(F_ref).to(torch.float32))
    ipiv = torch.from_numpy(ipiv_ref.astype(np.int32)).cuda() if pivot else None
    X, rep, _, _ = api.mxp_solve(dA, db, work=work, ipiv=ipiv, opts=opts, allow_notconv=True)
    torch.cuda.synchronize()
    ref = oracle.lp_precond(F_ref, ipiv_ref if pivot else None, b)
    assert np.array_equal(X.cpu().numpy(), ref)


@pytest.mark.parametrize("method,pivot,n,nb", [("gmres", False, 1024, 128),
                                               ("classical", False, 700, 64),
                                               ("gmres", True, 900, 128)])
def test_fp32_storage_solve(api, method, pivot, n, nb):
    """FP32 storage through refinement: converged below the threshold, outer
    iterations as the oracle refinement's on the oracle's factors."""
    seed = inputs.config_seed(2) + n
    A = (inputs.uniform_matrix(seed, 0, n, n) if pivot
         else inputs.diag_dominant_matrix(seed, 0, n))
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    dA, db = to_dev(A), to_dev(b)
    X, rep, _, _ = api.mxp_solve(dA, db, prec="fp32", nb=nb, pivot=pivot, refine=method)
    torch.cuda.synchronize()
    x = X.cpu().numpy()
    rho = checks.scaled_residual(A, x, b)
    F_ref, ipiv_ref, _ = oracle.lp_getrf(A, nb, 4, pivot=pivot)
    out = refine.refine(A, b, F_ref, ipiv_ref if pivot else None, method=method)
    note(f"fp32 storage {method} pivot={pivot} n={n}: outer {rep['outer_iters']} "
         f"(oracle {out['outer_iters']}), inner {rep['inner_iters']} "
         f"(oracle {out['inner_iters']}), rho {rho:.2f}")
    assert rep["converged"] == 1 and out["converged"] and rho < 16
    assert abs(rep["outer_iters"] - out["outer_iters"]) <= 1


def test_fp32_storage_rejects_transposed_solve(api):
    n = 128
    A = inputs.diag_dominant_matrix(3, 0, n)
    b = inputs.uniform_matrix(3, 1, n, 1)[:, 0]
    with pytest.raises(ValueError, match="argument 12"):   # the options
        api.mxp_solve(to_dev(A), to_dev(b), prec="fp32", nb=64, trans=True)


@pytest.mark.parametrize("prec,pivot", [("bf16", False), ("fp8", False), ("fp8_mx", False),
                                        ("bf16", True), ("fp32", False)])
def test_mxp_results_independent_of_workspace_contents(api, prec, pivot):
    """Determinism: the caller's workspace and the library's scratch starting
    as zeros or as NaN bytes (0xFF) give the same factors, pivots, solution
    and iteration counts bit for bit."""
    n, nb = 1100, 128 if prec.startswith("fp8") else 64
    seed = 777 + n
    A = (inputs.uniform_matrix(seed, 0, n, n) if pivot
         else inputs.diag_dominant_matrix(seed, 0, n))
    b = inputs.uniform_matrix(seed, 1, n, 1)[:, 0]
    dA, db = to_dev(A), to_dev(b)
    opts = api.mxp_options(prec=prec, nb=nb, pivot=pivot, restart=60)
    res = []
    try:
        for byte in (0x00, 0xFF):
            api.debug_poison_scratch(byte)   # every scratch buffer starts as `byte`
            work = torch.empty(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8,
                               device="cuda")
            work.fill_(byte)
            X = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            ipiv = torch.full((n,), -7, dtype=torch.int32, device="cuda") if pivot else None
            X, rep, work, ipiv = api.mxp_solve(dA, db, X=X, work=work, ipiv=ipiv, opts=opts)
            torch.cuda.synchronize()
            res.append((api.mxp_factors(work, n, prec).cpu().clone(), X.cpu(),
                        None if ipiv is None else ipiv.cpu(), rep["outer_iters"],
                        rep["inner_iters"]))
    finally:
        api.debug_poison_scratch(None)
    assert torch.equal(res[0][0].view(torch.int16 if prec != "fp32" else torch.int32),
                       res[1][0].view(torch.int16 if prec != "fp32" else torch.int32))
    assert torch.equal(res[0][1], res[1][1])
    if pivot:
        assert torch.equal(res[0][2], res[1][2])
    assert res[0][3:] == res[1][3:]
