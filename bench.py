#!/usr/bin/env python3
"""Benchmark of the dense LU solver on one MI355X.

Metric: effective TFLOP/s = (2/3 N^3) / time of one step, the operation count
of the paper's benchmarks (Sec. III-A.1) without the O(N^2) term.  A step is
one pass of the whole path over one resident N x N matrix:

  fp64 workloads:  lu_factor (PFACT, SWAP, DTRSM, DGEMM for every panel) +
                   lu_solve for one right-hand side
  mixed precision: conversion + low-precision LU + x0 + FP64 refinement to an
                   HPL scaled residual below 16 (the FP64-equivalent rate)

Inputs are generated in HBM before the timed region (one pristine matrix per
step for the in-place FP64 factorization).  Exactly `--steps` steps are timed
between two device synchronisations.

Default run: the headline is the FP64 workload (N = 32768, NB = 256); after
its matrices are freed, the two mixed-precision workloads (BF16, N = 65536;
FP8 updates, N = 131072) run as `legs` of the same JSON line with fewer steps,
each with its own roofline, residual, refinement counts, forward error against
an FP64 reference and CPU-oracle baseline.

Output: one JSON line.  `roofline` covers the dominant kernel (the FP64 MFMA
trailing update for the fp64 workloads, the low-precision trailing update for
the others): its algorithmic work per launch over its average launch time,
both from HIP events recorded on the kernel's stream during the timed steps.
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.

`--phase-model PATH` instead times every panel step's phases (PFACT, SWAP,
DTRSM, DGEMM) at N = 32768 for NB in {128, 256, 384, 512}, fits the per-step
cost model of Sec. III-A.1 and writes a markdown summary to PATH.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Effective TFLOP/s (2N³/3): FP64 LU vs BF16/FP8 LU+FP64 IR at residual<16"
PEAK_TFLOPS = {"f64": 78.6, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0}
HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
GEMM_SRC = os.path.join(ROOT, "paper_2604_09517_amd", "csrc", "gemm_f64.hip")
LP_SRC = os.path.join(ROOT, "paper_2604_09517_amd", "csrc", "lp_gemm.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def file_sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(name, src):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary, or None when missing or taken on other kernel source."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_t or m_sha.group(1) != file_sha(src):
        return None
    return float(m_t.group(1))


def fp64_first_step_flops(n, nb):
    """Flops of the oracle's first panel step (PFACT + DTRSM + DGEMM)."""
    m = n
    pf = sum((m - j - 1) + 2 * (m - j - 1) * (nb - j - 1) for j in range(nb))
    trsm = (n - nb) * nb * (nb - 1)
    gemm = 2 * (n - nb) ** 2 * nb
    return pf + trsm + gemm


def cpu_baseline_fp64(n, nb, seed):
    """Time the oracle on the first panel step of the same N, NB factorization."""
    import oracle
    from paper_2604_09517_amd import inputs

    threads = oracle.threads()
    t0 = time.perf_counter()
    A = inputs.uniform_matrix(seed, inputs.STREAM_A, n, n, threads=max(1, threads))
    log(f"cpu baseline: generated {n}x{n} on the host in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    oracle.getrf_inplace(A, nb, max_steps=1)
    dt = time.perf_counter() - t0
    flops = fp64_first_step_flops(n, nb)
    del A
    return {
        "value": flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first panel step (PFACT+SWAP+DTRSM+DGEMM, {flops:.3e} flop) of the "
                   f"N={n}, NB={nb} FP64 factorization, plain C oracle, {dt:.1f} s"),
    }


def run_fp64(args, cfg, steps, warmup, nb=None):
    import torch

    from paper_2604_09517_amd import api, inputs

    n = cfg["n"]
    nb = nb or cfg["nb"]
    seed = inputs.config_seed(cfg["index"])
    total = warmup + steps
    api.set_lookahead(args.lookahead)
    log(f"workload fp64 n={n} nb={nb} lookahead={args.lookahead}: "
        f"generating {total} matrices in HBM")
    mats = []
    for _ in range(total):
        A = api.fortran_empty(n, n)
        api.fill_uniform(A, seed, inputs.STREAM_A)
        mats.append(A)
    b = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    rhs = [b.clone() for _ in range(total)]
    piv = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(total)]
    torch.cuda.synchronize()

    for w in range(warmup):
        api.lu_factor(mats[w], nb, piv[w])
        api.lu_solve(mats[w], piv[w], rhs[w])
        torch.cuda.synchronize()
        log(f"warmup step {w} done")

    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(warmup, total):
        _, _, info = api.lu_factor(mats[k], nb, piv[k])
        api.lu_solve(mats[k], piv[k], rhs[k])
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    prof = api.profile_read()
    ms = (t1 - t0) * 1e3 / steps
    log(f"timed {steps} steps: {ms:.1f} ms/step")

    # verification (untimed): residual of the last solve against a fresh A
    A0 = mats[0]
    api.fill_uniform(A0, seed, inputs.STREAM_A)
    rho = api.scaled_residual(A0, rhs[-1], b)[0]
    log(f"scaled residual {rho:.3e}, info {infos}")

    gms, gflop, gcnt = prof["gemm"]        # (milliseconds, flops, launches)
    achieved = gflop / (gms * 1e-3) / 1e12 if gms > 0 else 0.0
    traffic = traffic_from_profile("gemm_f64_fp64_large.md", GEMM_SRC)
    roofline = {
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f64"],
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f64"], 4),
        "traffic": traffic, "kernel": "gemm_f64_direct_kernel (trailing update)",
        "launches": gcnt, "avg_launch_ms": round(gms / max(1, gcnt), 4),
    }
    phases = {p: round(v[0] / steps, 3) for p, v in prof.items() if v[2] > 0}
    value = (2.0 / 3.0) * n ** 3 / (ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "ms_per_step": round(ms, 3),
        "dtype": "f64",
        "config": {"workload": "fp64_lu_partial_pivoting_plus_solve", "n": n, "nb": nb,
                   "nrhs": 1, "matrix": "i.i.d. uniform[-0.5,0.5), column-major, lda=n",
                   "lookahead": args.lookahead,
                   "peak_frac_f64_mfma": round(value / PEAK_TFLOPS["f64"], 4)},
        "roofline": roofline,
        "scaled_residual": rho,
        "phases_ms_per_step": phases,
    }
    del A0, A
    mats.clear()
    rhs.clear()
    piv.clear()
    torch.cuda.empty_cache()
    return out, (lambda: cpu_baseline_fp64(n, nb, seed))


def cpu_baseline_mxp(cfg, seed, prec_id, n_sample=4096):
    """Time the oracle's mixed-precision solve (low-precision LU + GMRES-IR)
    on the same recipe at a smaller order."""
    import oracle
    from oracle import refine
    from paper_2604_09517_amd import inputs

    nb = min(cfg["nb"], n_sample)
    A = inputs.diag_dominant_matrix(seed, inputs.STREAM_A, n_sample)
    b = inputs.uniform_matrix(seed, inputs.STREAM_B, n_sample, 1)[:, 0]
    t0 = time.perf_counter()
    F, _, _ = oracle.lp_getrf(A, nb, prec_id, pivot=False, tile=128)
    out = refine.refine(A, b, F, None, method="gmres")
    dt = time.perf_counter() - t0
    return {
        "value": (2.0 / 3.0) * n_sample ** 3 / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"full mixed-precision solve (low-precision LU NB={nb} + GMRES-IR, "
                   f"converged={out['converged']}) of the same recipe at N={n_sample}, "
                   f"{dt:.1f} s"),
    }


def jacobi_reference(A, b, sweeps=40):
    """FP64 reference solution of the diagonally dominant system by Jacobi
    sweeps x <- x + D^-1 (b - A x) with torch's FP64 matrix-vector product
    (a comparator independent of the solver's kernels; untimed).  The
    iteration matrix has spectral radius about 1.16 / sqrt(N) here, so the
    error after the last sweep is about that times the last step."""
    import torch

    d = A.diagonal().clone()
    x = b / d
    step = float("inf")
    k = 0
    for k in range(sweeps):
        r = b - torch.mv(A, x)
        dx = r / d
        x = x + dx
        step = (dx.abs().max() / x.abs().max()).item()
        if step < 1e-17:
            break
    return x, step, k + 1


def run_mxp(args, cfg, name, steps, warmup):
    import torch

    from paper_2604_09517_amd import api, inputs

    n, nb = cfg["n"], cfg["nb"]
    prec = {"bf16_ir": "bf16", "fp8_ir": "fp8"}[name]
    seed = inputs.config_seed(cfg["index"])
    log(f"workload {name} n={n} nb={nb}: generating A in HBM")
    A = api.fortran_empty(n, n)
    api.fill_uniform(A, seed, inputs.STREAM_A)
    api.make_diag_dominant(A)
    b = torch.from_numpy(inputs.uniform_matrix(seed, inputs.STREAM_B, n, 1)[:, 0]).cuda()
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    opts = api.mxp_options(prec=prec, nb=nb, refine="gmres", scale_tile=128)
    work = torch.empty(api.mxp_workspace_bytes(n, opts, n), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for w in range(warmup):
        _, rep, _, _ = api.mxp_solve(A, b, X=X, work=work, opts=opts)
        torch.cuda.synchronize()
        log(f"warmup step {w}: {rep}")
    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(steps):
        _, rep, _, _ = api.mxp_solve(A, b, X=X, work=work, opts=opts)
        reps.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    prof = api.profile_read()
    ms = (t1 - t0) * 1e3 / steps
    rho = api.scaled_residual(A, X, b)[0]
    log(f"timed {steps} steps: {ms:.1f} ms/step, residual {rho:.3e}, last report {reps[-1]}")
    # forward error against an FP64 reference (untimed)
    del work
    torch.cuda.empty_cache()
    x_ref, jstep, sweeps = jacobi_reference(A, b)
    fwd = ((X - x_ref).abs().max() / x_ref.abs().max()).item()
    log(f"forward error {fwd:.3e} against FP64 Jacobi ({sweeps} sweeps, last step {jstep:.1e})")
    sms, sbytes, scnt = prof["lp_schur"]   # (milliseconds, bytes, launches)
    achieved = sbytes / (sms * 1e-3) / 1e9 if sms > 0 else 0.0
    schur_flops = sum(2.0 * (n - k0 - nb) ** 2 * nb for k0 in range(0, n - nb, nb))
    mma_peak = PEAK_TFLOPS["bf16" if prec == "bf16" else "fp8"]
    value = (2.0 / 3.0) * n ** 3 / (ms * 1e-3) / 1e12
    phases = {p: round(v[0] / steps, 3) for p, v in prof.items() if v[2] > 0}
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "ms_per_step": round(ms, 3),
        "dtype": "bf16" if prec == "bf16" else "fp8",
        "config": {"workload": f"{prec}_lu_nopivot_plus_fp64_gmres_ir", "n": n, "nb": nb,
                   "nrhs": 1, "matrix": "diagonally dominant (off-diagonal uniform[-0.5,0.5), "
                   "diagonal = row sum of |off-diagonal|), column-major",
                   "storage": "bf16" if prec == "bf16" else "fp16",
                   "scale_tile": 128 if prec == "fp8" else None,
                   "peak_frac_fp64_equivalent_vs_mfma": round(value / mma_peak, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_GBS, 4),
                     "traffic": traffic_from_profile(
                         "lp_schur16_bf16_ir.md" if name == "bf16_ir" else "lp_schur8_fp8_ir.md",
                         LP_SRC),
                     "kernel": f"lp_schur{'16' if prec == 'bf16' else '8'}_kernel "
                               f"(trailing update)",
                     "launches": scnt, "avg_launch_ms": round(sms / max(1, scnt), 4),
                     "concurrent_with": "the look-ahead's next panel, U12 solve and operand "
                                        "packing on a second stream (three update launches per "
                                        "step; the third overlaps that work)",
                     "mfma_tflops": round(schur_flops * steps / (sms * 1e-3) / 1e12, 1)
                     if sms > 0 else None,
                     "mfma_peak_tflops": mma_peak},
        "scaled_residual": rho,
        "forward_error": {"value": fwd, "reference": "FP64 Jacobi sweeps with torch's FP64 "
                          "matrix-vector product on the resident A", "sweeps": sweeps,
                          "reference_last_step": jstep},
        "refinement": {"outer": reps[-1]["outer_iters"], "inner": reps[-1]["inner_iters"],
                       "converged": reps[-1]["converged"],
                       "t_convert_ms": round(reps[-1]["t_convert_ms"], 3),
                       "t_factor_ms": round(reps[-1]["t_factor_ms"], 3),
                       "t_refine_ms": round(reps[-1]["t_refine_ms"], 3)},
        "phases_ms_per_step": phases,
    }
    del A, X, b, x_ref
    torch.cuda.empty_cache()
    prec_id = 0 if prec == "bf16" else 2
    # about 16 s of host work for either leg
    return out, (lambda: cpu_baseline_mxp(cfg, seed, prec_id, 6144))


# ---------------------------------------------------------------- phase model
PHASE_UNITS = {
    # phase: (work of one panel step from (n, m, nb), description)
    "gemm": (lambda n, m, nb: 2.0 * (m - nb) ** 2 * nb, "2 (m-nb)^2 nb  [~ N^2 NB]"),
    "pfact": (lambda n, m, nb: float(m) * nb * nb, "m nb^2  [~ N NB^2]"),
    # the interchanges of a step reach the columns right of its panel; those
    # left of it are applied once after the factorization (step -1 below)
    "swap": (lambda n, m, nb: float(m - nb) * nb, "(m-nb) nb  [~ N NB]"),
    "trsm": (lambda n, m, nb: float(nb) * nb * (m - nb), "nb^2 (m-nb)"),
}


def fit_linear(xs, ys):
    """Least squares y = a x + c; returns (a, c, r2, rms relative residual)."""
    import numpy as np

    X = np.column_stack([xs, np.ones(len(xs))])
    coef, *_ = np.linalg.lstsq(X, ys, rcond=None)
    pred = X @ coef
    ss_res = float(((ys - pred) ** 2).sum())
    ss_tot = float(((ys - ys.mean()) ** 2).sum())
    r2 = 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
    rel = float(np.sqrt((((ys - pred) / np.maximum(ys, 1e-9)) ** 2).mean()))
    return float(coef[0]), float(coef[1]), r2, rel


def phase_series(n, nb, lookahead):
    """One factorization with per-step phase intervals: ({phase: {step: ms}},
    wall ms)."""
    import torch

    from paper_2604_09517_amd import api, inputs

    api.set_lookahead(lookahead)
    seed = inputs.config_seed(1)
    A = api.fortran_empty(n, n)
    piv = torch.empty(n, dtype=torch.int32, device="cuda")
    wall = 0.0
    for rep in range(2):          # the first run warms up
        api.fill_uniform(A, seed, inputs.STREAM_A)
        torch.cuda.synchronize()
        api.profile_reset()
        api.profile_enable(rep == 1)
        t0 = time.perf_counter()
        api.lu_factor(A, nb, piv)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        api.profile_enable(False)
    series = {}
    for ph in PHASE_UNITS:
        d = {}
        for step, ms, _ in api.profile_intervals(ph):
            d[step] = d.get(step, 0.0) + ms
        series[ph] = d
    api.profile_reset()
    api.set_lookahead(1)
    del A
    torch.cuda.empty_cache()
    return series, wall


def run_phase_model(args):
    import numpy as np

    n = 32768
    nbs = [128, 256, 384, 512]
    rows = []          # (nb, step, m, phase, ms)
    walls = {}
    for nb in nbs:
        for la in (0, 1):
            series, wall = phase_series(n, nb, la)
            walls[(nb, la)] = (wall, {p: sum(v.values()) for p, v in series.items()},
                               series["swap"].get(-1, 0.0))
            log(f"phase series n={n} nb={nb} lookahead={la}: {wall:.1f} ms")
            if la == 0:
                for ph, d in series.items():
                    for step, ms in d.items():
                        if step >= 0:   # the deferred interchanges are no panel step
                            rows.append((nb, step, n - step * nb, ph, ms))
    fits = {}
    for ph, (f, desc) in PHASE_UNITS.items():
        pts = [(f(n, m, nb), ms) for nb, step, m, p, ms in rows if p == ph and m - nb > 0]
        xs = np.array([p[0] for p in pts])
        ys = np.array([p[1] for p in pts])
        fits[ph] = fit_linear(xs, ys) + (desc, len(pts))
    # GEMM / SWAP crossover per NB: first step whose SWAP time reaches its GEMM time
    cross = {}
    ag, cg = fits["gemm"][:2]
    asw, csw = fits["swap"][:2]
    for nb in nbs:
        steps = sorted({s for b, s, m, p, ms in rows if b == nb})
        g = {s: ms for b, s, m, p, ms in rows if b == nb and p == "gemm"}
        w = {s: ms for b, s, m, p, ms in rows if b == nb and p == "swap"}
        meas = next((s for s in steps if s in g and s in w and w[s] >= g[s]), None)
        pred = next((s for s in steps if asw * (n - s * nb - nb) * nb + csw >=
                     ag * 2.0 * (n - s * nb - nb) ** 2 * nb + cg), None)
        cross[nb] = (meas, pred, len(steps))
    # serial totals per NB predicted by the fit, against the measured ones
    pred_tot = {}
    for nb in nbs:
        t = 0.0
        for k0 in range(0, n, nb):
            m = n - k0
            for ph, (f, _) in PHASE_UNITS.items():
                if ph in ("gemm", "trsm") and m - nb <= 0:
                    continue
                a, c = fits[ph][:2]
                t += a * f(n, m, nb) + c
        pred_tot[nb] = t + walls[(nb, 0)][2]   # plus the measured deferred interchanges
    lines = ["# Per-step phase model of the FP64 factorization (N = 32768)", "",
             "Command: `python bench.py --phase-model <out.md>` (HIP events around every "
             "phase of every panel step on the stream it runs on; one warm-up factorization, "
             "then one recorded factorization per NB and look-ahead depth).", "",
             "Cost model of Sec. III-A.1 per panel step, m = rows left at the step: "
             "T = a * work + c, fitted by least squares over every step of the look-ahead-0 "
             "runs at all four NB.", "",
             "| phase | work per step | a (ms per unit) | c (ms) | R^2 | rms rel. residual | steps |",
             "|---|---|---|---|---|---|---|"]
    for ph, (a, c, r2, rel, desc, cnt) in fits.items():
        lines.append(f"| {ph} | {desc} | {a:.4e} | {c:.4f} | {r2:.4f} | {rel:.3f} | {cnt} |")
    g_rate = 1.0 / fits["gemm"][0] / 1e9 if fits["gemm"][0] > 0 else 0.0
    deferred = {nb: walls[(nb, 0)][2] for nb in nbs}
    lines += ["", f"The DGEMM slope corresponds to {g_rate:.1f} TFLOP/s at the margin; the "
              "intercepts are per-step latencies (launch gaps, partial waves).  The "
              "interchanges of the columns left of each panel run once after the "
              "factorization: " + ", ".join(f"{deferred[nb]:.1f} ms at NB = {nb}" for nb in nbs)
              + " (included in the SWAP sums below).", "",
              "| NB | serial total measured (ms) | serial total from the fit (ms) | "
              "look-ahead 1 total (ms) | PFACT / SWAP / DTRSM / DGEMM sums at depth 0 (ms) | "
              "GEMM/SWAP crossover step measured / fitted (of steps) |",
              "|---|---|---|---|---|---|"]
    for nb in nbs:
        w0, s0, _ = walls[(nb, 0)]
        w1 = walls[(nb, 1)][0]
        cm, cp, ns = cross[nb]
        lines.append(f"| {nb} | {w0:.1f} | {pred_tot[nb]:.1f} | {w1:.1f} | "
                     f"{s0['pfact']:.1f} / {s0['swap']:.1f} / {s0['trsm']:.1f} / "
                     f"{s0['gemm']:.1f} | {cm} / {cp} ({ns}) |")
    best = min(nbs, key=lambda b: walls[(b, 1)][0])
    lines += ["", f"Fastest NB at look-ahead 1: {best}.", "",
              "Per-step series at NB = 256, look-ahead 0 (every 8th step):", "",
              "| step | m | PFACT | SWAP | DTRSM | DGEMM (ms) |", "|---|---|---|---|---|---|"]
    ser = {p: {s: ms for b, s, m, pp, ms in rows if b == 256 and pp == p} for p in PHASE_UNITS}
    for s in sorted(ser["pfact"])[::8]:
        lines.append(f"| {s} | {n - s * 256} | {ser['pfact'].get(s, 0):.3f} | "
                     f"{ser['swap'].get(s, 0):.3f} | {ser['trsm'].get(s, 0):.3f} | "
                     f"{ser['gemm'].get(s, 0):.3f} |")
    with open(args.phase_model, "w") as f:
        f.write("\n".join(lines) + "\n")
    log(f"wrote {args.phase_model}")
    print(json.dumps({"phase_model": {ph: {"a_ms_per_unit": v[0], "c_ms": v[1], "r2": v[2],
                                           "rel_rms": v[3]} for ph, v in fits.items()},
                      "crossover": {str(k): v for k, v in cross.items()},
                      "walls_ms": {f"{k[0]}/{k[1]}": v[0] for k, v in walls.items()}}),
          flush=True)


def copy_calibration(nbytes):
    """A plain device copy of known size (rocprofv3 counter calibration)."""
    import torch

    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                      "launches": 3}), flush=True)


def leg_record(out, cpu, steps, warmup, no_cpu):
    """A mixed-precision workload of the default run, as one sub-record."""
    rec = {"workload": out["config"]["workload"], "value": out["value"], "unit": out["unit"],
           "ms_per_step": out["ms_per_step"], "steps": steps, "warmup": warmup,
           "dtype": out["dtype"]}
    for k, v in out.items():
        if k not in rec and k != "metric":
            rec[k] = v
    rec["cpu_baseline"] = None if no_cpu else cpu()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all",
                    choices=["all", "fp64_large", "fp64_small", "bf16_ir", "fp8_ir"])
    ap.add_argument("--leg-steps", type=int, default=3,
                    help="timed steps of each mixed-precision leg of the default run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lookahead", type=int, default=1, choices=[0, 1],
                    help="look-ahead depth of the FP64 factorization")
    ap.add_argument("--nb", type=int, default=0, help="panel width of the FP64 workload")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run only a plain copy of this many bytes (counter calibration)")
    ap.add_argument("--phase-model", default="",
                    help="write the per-step phase model summary to this path")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU: this build has no multi-GPU path "
               f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})")
        print(msg, file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    from paper_2604_09517_amd import api, inputs
    api.lib()
    if args.phase_model:
        run_phase_model(args)
        return
    head = "fp64_large" if args.workload == "all" else args.workload
    cfg = inputs.WORKLOADS[head]
    if head.startswith("fp64"):
        out, cpu = run_fp64(args, cfg, args.steps, args.warmup, args.nb or None)
    else:
        out, cpu = run_mxp(args, cfg, head, args.steps, args.warmup)
    line = {
        "metric": out.pop("metric"),
        "value": out.pop("value"),
        "unit": out.pop("unit"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": out.pop("dtype"),
        "data": "synthetic (seeded counter-based generator, generated in HBM)",
        "config": out.pop("config"),
        "roofline": out.pop("roofline"),
    }
    line.update(out)
    line["cpu_baseline"] = None if args.no_cpu_baseline else cpu()
    if args.workload == "all":
        legs = []
        lsteps, lwarm = max(1, min(args.steps, args.leg_steps)), min(args.warmup, 1)
        for name in ("bf16_ir", "fp8_ir"):
            o, c = run_mxp(args, inputs.WORKLOADS[name], name, lsteps, lwarm)
            legs.append(leg_record(o, c, lsteps, lwarm, args.no_cpu_baseline))
        line["legs"] = legs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
