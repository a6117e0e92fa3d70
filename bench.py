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
step, since the factorization works in place).  Exactly `--steps` steps are
timed between two device synchronisations.

Output: one JSON line.  `roofline` covers the dominant kernel (the FP64 MFMA
trailing update for the fp64 workloads): its algorithmic flops per launch over
its average launch time, both from HIP events recorded on the kernel's stream
during the timed steps.  `cpu_baseline` times the CPU oracle on a bounded
sample of the same workload (rank 0 only).
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

METRIC = "Effective TFLOP/s (2N\u00b3/3): FP64 LU vs BF16/FP8 LU+FP64 IR at residual<16"
PEAK_TFLOPS = {"f64": 78.6, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0}
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


def run_fp64(args, cfg):
    import torch

    from paper_2604_09517_amd import api, inputs

    n, nb = cfg["n"], cfg["nb"]
    seed = inputs.config_seed(cfg["index"])
    total = args.warmup + args.steps
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

    for w in range(args.warmup):
        api.lu_factor(mats[w], nb, piv[w])
        api.lu_solve(mats[w], piv[w], rhs[w])
        torch.cuda.synchronize()
        log(f"warmup step {w} done")

    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(args.warmup, total):
        _, _, info = api.lu_factor(mats[k], nb, piv[k])
        api.lu_solve(mats[k], piv[k], rhs[k])
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    prof = api.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms:.1f} ms/step")

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
    phases = {p: round(v[0] / args.steps, 3) for p, v in prof.items() if v[2] > 0}
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
    for A in mats:
        del A
    mats.clear()
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


def run_mxp(args, cfg, name):
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
    for w in range(args.warmup):
        _, rep, _, _ = api.mxp_solve(A, b, X=X, work=work, opts=opts)
        torch.cuda.synchronize()
        log(f"warmup step {w}: {rep}")
    api.profile_reset()
    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        _, rep, _, _ = api.mxp_solve(A, b, X=X, work=work, opts=opts)
        reps.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.profile_enable(False)
    prof = api.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    rho = api.scaled_residual(A, X, b)[0]
    log(f"timed {args.steps} steps: {ms:.1f} ms/step, residual {rho:.3e}, last report {reps[-1]}")
    sms, sbytes, scnt = prof["lp_schur"]   # (milliseconds, bytes, launches)
    achieved = sbytes / (sms * 1e-3) / 1e9 if sms > 0 else 0.0
    schur_flops = sum(2.0 * (n - k0 - nb) ** 2 * nb for k0 in range(0, n - nb, nb))
    mma_peak = PEAK_TFLOPS["bf16" if prec == "bf16" else "fp8"]
    value = (2.0 / 3.0) * n ** 3 / (ms * 1e-3) / 1e12
    phases = {p: round(v[0] / args.steps, 3) for p, v in prof.items() if v[2] > 0}
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
                   "peak_frac_fp64_equivalent_vs_mfma": round(value / mma_peak, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(achieved / 8000.0, 4),
                     "traffic": traffic_from_profile(
                         "lp_schur16_bf16_ir.md" if name == "bf16_ir" else "lp_schur8_fp8_ir.md",
                         LP_SRC),
                     "kernel": f"lp_schur{'16' if prec == 'bf16' else '8'}_kernel "
                               f"(trailing update)",
                     "launches": scnt, "avg_launch_ms": round(sms / max(1, scnt), 4),
                     "mfma_tflops": round(schur_flops * args.steps / (sms * 1e-3) / 1e12, 1)
                     if sms > 0 else None,
                     "mfma_peak_tflops": mma_peak},
        "scaled_residual": rho,
        "refinement": {"outer": reps[-1]["outer_iters"], "inner": reps[-1]["inner_iters"],
                       "converged": reps[-1]["converged"],
                       "t_convert_ms": round(reps[-1]["t_convert_ms"], 3),
                       "t_factor_ms": round(reps[-1]["t_factor_ms"], 3),
                       "t_refine_ms": round(reps[-1]["t_refine_ms"], 3)},
        "phases_ms_per_step": phases,
    }
    del A, work
    torch.cuda.empty_cache()
    prec_id = 0 if prec == "bf16" else 2
    return out, (lambda: cpu_baseline_mxp(cfg, seed, prec_id))


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fp64_large",
                    choices=["fp64_large", "fp64_small", "bf16_ir", "fp8_ir"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lookahead", type=int, default=1, choices=[0, 1],
                    help="look-ahead depth of the FP64 factorization")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run only a plain copy of this many bytes (counter calibration)")
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
    cfg = inputs.WORKLOADS[args.workload]
    if args.workload.startswith("fp64"):
        out, cpu = run_fp64(args, cfg)
    else:
        out, cpu = run_mxp(args, cfg, args.workload)
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
