// Launchers of the refinement kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "asource.h"

namespace mxlu {

constexpr int kTrsvBs = 256;   // block rows of the FP32 triangular solves

// y = A x (b == NULL) or y = b - A x; op(A) = A (trans 0) or A^T (trans 1),
// A in memory or regenerated from its seed (ASource).
// part, asum_part: nsplit * n doubles (asum_part optional: |op(A)| row sums).
// stats (optional, zeroed by the caller): [0] max|y|, [1] max row sum, [2] max|x|
// as bit patterns of non-negative doubles.
int gemv_f64(int trans, int64_t n, const ASource &src, const double *x,
             const double *b, double *y, double *part, double *asum_part, int nsplit,
             unsigned long long *stats, hipStream_t s);
// out[c] = V[:, c] . z for c < ncols; part holds ncols * nchunks doubles.
int dots_f64(int64_t n, int ncols, const double *V, int64_t ldv, const double *z, double *part,
             int nchunks, double *out, hipStream_t s);
// z += sign * V[:, :k] h   (h on the device, k <= 256)
int gemv_small_f64(int64_t n, int k, const double *V, int64_t ldv, const double *h, double sign,
                   double *z, hipStream_t s);
int scale_copy_f64(int64_t n, const double *z, double alpha, double *v, hipStream_t s);
int axpy_f64(int64_t n, const double *z, double *x, hipStream_t s);
int absmax_f64(int64_t n, const double *v, unsigned long long *out, hipStream_t s);
// State of the single-launch blocked triangular solves: xs holds n tagged
// words (zeroed once at allocation), tag the last tag used (each solve takes
// the next one), expired one device int set when a wait expires.
struct TrsvChain {
    uint64_t *xs;
    int *expired;
    uint32_t tag;
};

// d = M r (trans 0) or M^T r (trans 1) with M = U^-1 L^-1 P from the stored
// factors F; perm (optional) is the row order of P.  v32: n floats scratch;
// smax: one device word.
int lp_precond_apply(int fmt, int trans, int64_t n, const uint16_t *F, int64_t ldf,
                     const int32_t *perm, const double *r, double *d, float *v32,
                     unsigned long long *smax, TrsvChain &ch, hipStream_t s);
// d = M r with M = U^-1 L^-1 P from FP32 factors (FP32 storage; forward only).
int lp_precond_apply_f32(int64_t n, const float *F, int64_t ldf, const int32_t *perm,
                         const double *r, double *d, float *v32, unsigned long long *smax,
                         hipStream_t s);

}  // namespace mxlu
