"""Writes tests/golden/c2_pivots.npz: the oracle's interchange sequence of the
N = 32768, NB = 256 FP64 factorization of the seeded uniform matrix (the bench
workload), with the relative gap of every pivot search.

Calls only the oracle and the seeded input generator.  Run from the repository
root:  python tests/golden/make_c2_pivots.py   (about 8 GiB of host memory and
some minutes on a few cores).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2604_09517_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_pivots.npz")


def main():
    cfg = inputs.WORKLOADS["fp64_large"]
    n, nb = cfg["n"], cfg["nb"]
    seed = inputs.config_seed(cfg["index"])
    t0 = time.time()
    A = inputs.uniform_matrix(seed, inputs.STREAM_A, n, n, threads=os.cpu_count() or 1)
    print(f"generated {n}x{n} in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    ipiv, gaps, info = oracle.getrf_gaps_inplace(A, nb)
    print(f"oracle getrf in {time.time() - t0:.1f} s on {oracle.threads()} threads, info {info}",
          flush=True)
    np.savez_compressed(OUT, n=n, nb=nb, seed=seed, ipiv=ipiv, gaps=gaps.astype(np.float32),
                        info=info)
    print(f"wrote {OUT}: min gap {gaps.min():.3e} at column {int(gaps.argmin())}")


if __name__ == "__main__":
    main()
