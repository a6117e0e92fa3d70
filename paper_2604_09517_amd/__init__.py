"""MI355X-native dense LU solver: FP64 LU with partial pivoting and the
mixed-precision LU + FP64 refinement variant, as hand-written HIP kernels for
gfx950 behind a small C ABI (include/mxlu.h).

Importing the package loads nothing; the HIP library is loaded on the first
call into `paper_2604_09517_amd.api` (and raises if it has not been built).
"""

__all__ = ["api", "inputs", "autograd"]
