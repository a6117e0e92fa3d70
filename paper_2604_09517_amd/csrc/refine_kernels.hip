// Kernels of the FP64 iterative refinement (Sec. III-A.2: residuals and
// corrections in FP64; Sec. II-B: refinement based on GMRES) and of its
// preconditioner M = U^-1 L^-1 P applied in FP32 to the low-precision factors.
#include <hip/hip_runtime.h>

#include "common.h"
#include "lp_common.h"
#include "refine_kernels.h"

namespace {

using namespace mxlu;

__device__ __forceinline__ void atomic_max_abs(unsigned long long *dst, double v) {
    atomicMax(dst, (unsigned long long)__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ double bits_to_double(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

// ---------------------------------------------------------------- GEMV
// partial[s][i] = sum over columns j of split s of A[i, j] x[j] (ascending
// j); with asum, the |A[i, j]| row sums of the split go to asum_part.
__global__ __launch_bounds__(256) void gemv_n_partial_kernel(int64_t n, const double *__restrict__ A,
                                                             int64_t lda,
                                                             const double *__restrict__ x,
                                                             int64_t cps, double *__restrict__ part,
                                                             double *__restrict__ asum_part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * cps;
    const int64_t j1 = (j0 + cps < n) ? j0 + cps : n;
    if (i >= n) return;
    double acc = 0.0, as = 0.0;
    int64_t j = j0;
    for (; j + 4 <= j1; j += 4) {
        const double a0 = MXLU_AT(A, i, j, lda), a1 = MXLU_AT(A, i, j + 1, lda);
        const double a2 = MXLU_AT(A, i, j + 2, lda), a3 = MXLU_AT(A, i, j + 3, lda);
        acc = fma(a0, x[j], acc);
        acc = fma(a1, x[j + 1], acc);
        acc = fma(a2, x[j + 2], acc);
        acc = fma(a3, x[j + 3], acc);
        if (asum_part) as += fabs(a0) + fabs(a1) + fabs(a2) + fabs(a3);
    }
    for (; j < j1; ++j) {
        const double a = MXLU_AT(A, i, j, lda);
        acc = fma(a, x[j], acc);
        if (asum_part) as += fabs(a);
    }
    part[(size_t)blockIdx.y * n + i] = acc;
    if (asum_part) asum_part[(size_t)blockIdx.y * n + i] = as;
}

// Transposed: part[s][i] = sum over rows j of split s of A[j, i] x[j]; one
// wave per i (column i of A is contiguous).
__global__ __launch_bounds__(256) void gemv_t_partial_kernel(int64_t n, const double *__restrict__ A,
                                                             int64_t lda,
                                                             const double *__restrict__ x,
                                                             int64_t cps, double *__restrict__ part,
                                                             double *__restrict__ asum_part) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t j0 = (int64_t)blockIdx.y * cps;
    const int64_t j1 = (j0 + cps < n) ? j0 + cps : n;
    if (i >= n) return;
    double acc = 0.0, as = 0.0;
    for (int64_t j = j0 + lane; j < j1; j += 64) {
        const double a = MXLU_AT(A, j, i, lda);
        acc = fma(a, x[j], acc);
        as += fabs(a);
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off);
        as += __shfl_xor(as, off);
    }
    if (lane == 0) {
        part[(size_t)blockIdx.y * n + i] = acc;
        if (asum_part) asum_part[(size_t)blockIdx.y * n + i] = as;
    }
}

// y[i] = (b ? b[i] - sum_s part : sum_s part); maxima of |y| and of the
// |A| row sums go to stats[0] and stats[1] (bit patterns), |x| to stats[2].
__global__ void gemv_finish_kernel(int64_t n, int nsplit, const double *__restrict__ part,
                                   const double *__restrict__ asum_part,
                                   const double *__restrict__ b, double *__restrict__ y,
                                   const double *__restrict__ xv,
                                   unsigned long long *__restrict__ stats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m_y = 0.0, m_a = 0.0, m_x = 0.0;
    if (i < n) {
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * n + i];
        const double v = b ? b[i] - s : s;
        y[i] = v;
        m_y = fabs(v);
        if (asum_part) {
            double a = 0.0;
            for (int k = 0; k < nsplit; ++k) a += asum_part[(size_t)k * n + i];
            m_a = a;
        }
        if (xv) m_x = fabs(xv[i]);
    }
    if (stats) {
        for (int off = 32; off > 0; off >>= 1) {
            m_y = fmax(m_y, __shfl_xor(m_y, off));
            m_a = fmax(m_a, __shfl_xor(m_a, off));
            m_x = fmax(m_x, __shfl_xor(m_x, off));
        }
        if ((threadIdx.x & 63) == 0) {
            atomic_max_abs(&stats[0], m_y);
            if (asum_part) atomic_max_abs(&stats[1], m_a);
            if (xv) atomic_max_abs(&stats[2], m_x);
        }
    }
}

// ---------------------------------------------------------------- BLAS-1/2
// part[c][chunk] = sum over the chunk of V[:, c] * z
__global__ __launch_bounds__(256) void dots_partial_kernel(int64_t n, const double *__restrict__ V,
                                                           int64_t ldv,
                                                           const double *__restrict__ z,
                                                           int64_t chunk, double *__restrict__ part,
                                                           int nchunks) {
    __shared__ double red[256];
    const int c = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc = fma(MXLU_AT(V, i, c, ldv), z[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)c * nchunks + blockIdx.x] = red[0];
}

__global__ void dots_reduce_kernel(int ncols, int nchunks, const double *__restrict__ part,
                                   double *__restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double s = 0.0;
    for (int k = 0; k < nchunks; ++k) s += part[(size_t)c * nchunks + k];
    out[c] = s;
}

// z[i] += sign * sum_c V[i, c] h[c]   (c ascending)
__global__ void gemv_small_kernel(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                  const double *__restrict__ h, double sign,
                                  double *__restrict__ z) {
    __shared__ double hs[256];
    if ((int)threadIdx.x < k) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = z[i];
    for (int c = 0; c < k; ++c) acc = fma(sign * MXLU_AT(V, i, c, ldv), hs[c], acc);
    z[i] = acc;
}

__global__ void scale_copy_kernel(int64_t n, const double *__restrict__ z, double alpha,
                                  double *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = z[i] * alpha;
}

__global__ void axpy_kernel(int64_t n, const double *__restrict__ z, double *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + z[i];
}

__global__ void absmax_kernel(int64_t n, const double *__restrict__ v,
                              unsigned long long *__restrict__ out) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(v[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomic_max_abs(out, m);
}

// ---------------------------------------------------------------- precond
// v32[i] = fp32( r[src(i)] / s ), s = *smax (bits) or 1 when zero;
// src(i) = perm[i] when perm is given (apply P), else i.
__global__ void precond_in_kernel(int64_t n, const double *__restrict__ r,
                                  const int32_t *__restrict__ perm,
                                  const unsigned long long *__restrict__ smax,
                                  float *__restrict__ v32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = bits_to_double(*smax);
    const double ri = r[perm ? perm[i] : i];
    v32[i] = s > 0.0 ? (float)(ri / s) : 0.0f;
}

// d[dst(i)] = s * fp64(v32[i]); dst(i) = perm[i] when given (apply P^T).
__global__ void precond_out_kernel(int64_t n, const float *__restrict__ v32,
                                   const int32_t *__restrict__ perm,
                                   const unsigned long long *__restrict__ smax,
                                   double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = bits_to_double(*smax);
    d[perm ? perm[i] : i] = s > 0.0 ? s * (double)v32[i] : 0.0;
}

// Blocked triangular solve in FP32 with the stored factor F (16-bit),
// blocks of kTrsvBs rows.  Launch `step` (one per block, in solve order)
// first applies the finished block `prev` to the rows of the blocks still to
// be solved (one workgroup per block), then workgroup 0 solves the diagonal
// block `cur` = the next one in order.  Each element accumulates its terms
// in the order of the textbook substitution (column-oriented for L and U:
// ascending k for L, descending k for U; ascending i for the transposed
// forms within a block).
//   kind 0: L (unit lower), forward;   kind 1: U (upper), backward
//   kind 2: U^T (lower), forward;      kind 3: L^T (unit upper), backward
template <int FMT, int KIND>
__global__ __launch_bounds__(256) void trsv_step_kernel(int64_t n, const uint16_t *__restrict__ F,
                                                        int64_t ldf, float *__restrict__ v,
                                                        int64_t prev, int64_t cur, int nblk,
                                                        int dir) {
    constexpr int BS = kTrsvBs;
    __shared__ float vprev[BS];
    __shared__ uint16_t Ld[BS][BS + 2];   // raw stored values (128 KB)
    const int tid = threadIdx.x;
    // block handled by this workgroup: cur + dir * blockIdx.x
    const int64_t myblk = cur + (int64_t)dir * blockIdx.x;
    const int64_t r0 = myblk * BS;
    const int rows = (int)((n - r0 < BS) ? n - r0 : BS);
    if (prev >= 0) {
        const int64_t p0 = prev * BS;
        const int pr = (int)((n - p0 < BS) ? n - p0 : BS);
        if (tid < pr) vprev[tid] = v[p0 + tid];
        __syncthreads();
        if (tid < rows) {
            const int64_t i = r0 + tid;
            float acc = v[i];
            if (KIND == 0) {          // v_i -= L[i][k] v_k, k ascending
                for (int k = 0; k < pr; ++k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)i + (size_t)(p0 + k) * ldf]), vprev[k], acc);
            } else if (KIND == 1) {   // v_i -= U[i][k] v_k, k descending
                for (int k = pr - 1; k >= 0; --k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)i + (size_t)(p0 + k) * ldf]), vprev[k], acc);
            } else if (KIND == 2) {   // v_k -= U[i][k] v_i (i in prev block), i ascending
                for (int k = 0; k < pr; ++k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)(p0 + k) + (size_t)i * ldf]), vprev[k], acc);
            } else {                  // v_k -= L[i][k] v_i, i ascending
                for (int k = 0; k < pr; ++k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)(p0 + k) + (size_t)i * ldf]), vprev[k], acc);
            }
            v[i] = acc;
        }
    }
    if (blockIdx.x != 0) return;
    // diagonal block of `cur`, staged in LDS as the effective lower/upper factor
    __syncthreads();
    for (int t = tid; t < rows * rows; t += 256) {
        const int i = t % rows, k = t / rows;
        const uint16_t f = F[(size_t)(r0 + i) + (size_t)(r0 + k) * ldf];
        if (KIND == 0 || KIND == 1) Ld[i][k] = f;
        else Ld[k][i] = f;     // transposed forms: Ld[i][k] = F[k][i]
    }
    __syncthreads();
    if (tid >= 64) return;
    // one wave: lane owns rows lane, lane+64, lane+128, lane+192
    float x[BS / 64];
#pragma unroll
    for (int q = 0; q < BS / 64; ++q) {
        const int i = tid + 64 * q;
        x[q] = (i < rows) ? v[r0 + i] : 0.0f;
    }
    constexpr bool FWD = (KIND == 0 || KIND == 2);
    constexpr bool UNIT = (KIND == 0 || KIND == 3);
#pragma unroll
    for (int q = 0; q < BS / 64; ++q) {
        for (int kk = 0; kk < 64; ++kk) {
            const int s = q * 64 + kk;
            if (s >= rows) break;
            const int k = FWD ? s : rows - 1 - s;
            const int kq = k / 64, kl = k % 64;
            // finish x_k on its owner lane, then broadcast it
            float xk = 0.0f;
#pragma unroll
            for (int qq = 0; qq < BS / 64; ++qq)
                if (qq == kq) {
                    if (!UNIT && tid == kl) x[qq] = x[qq] / lp_to_f32<FMT>(Ld[k][k]);
                    xk = __shfl(x[qq], kl);
                }
#pragma unroll
            for (int qq = 0; qq < BS / 64; ++qq) {
                const int i = tid + 64 * qq;
                if (i < rows && (FWD ? i > k : i < k))
                    x[qq] = fmaf(-lp_to_f32<FMT>(Ld[i][k]), xk, x[qq]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < BS / 64; ++q) {
        const int i = tid + 64 * q;
        if (i < rows) v[r0 + i] = x[q];
    }
}

unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

namespace mxlu {

int gemv_f64(int trans, int64_t n, const double *A, int64_t lda, const double *x,
             const double *b, double *y, double *part, double *asum_part, int nsplit,
             unsigned long long *stats, hipStream_t s) {
    if (n <= 0) return 0;
    const int64_t cps = (n + nsplit - 1) / nsplit;
    if (trans == 0)
        hipLaunchKernelGGL(gemv_n_partial_kernel, dim3(g1(n), (unsigned)nsplit), dim3(256), 0, s,
                           n, A, lda, x, cps, part, asum_part);
    else
        hipLaunchKernelGGL(gemv_t_partial_kernel, dim3((unsigned)((n + 3) / 4), (unsigned)nsplit),
                           dim3(256), 0, s, n, A, lda, x, cps, part, asum_part);
    MXLU_LAUNCH_CHECK();
    hipLaunchKernelGGL(gemv_finish_kernel, dim3(g1(n)), dim3(256), 0, s, n, nsplit, part,
                       asum_part, b, y, x, stats);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int dots_f64(int64_t n, int ncols, const double *V, int64_t ldv, const double *z, double *part,
             int nchunks, double *out, hipStream_t s) {
    if (ncols <= 0) return 0;
    const int64_t chunk = (n + nchunks - 1) / nchunks;
    hipLaunchKernelGGL(dots_partial_kernel, dim3((unsigned)nchunks, (unsigned)ncols), dim3(256), 0,
                       s, n, V, ldv, z, chunk, part, nchunks);
    MXLU_LAUNCH_CHECK();
    hipLaunchKernelGGL(dots_reduce_kernel, dim3((unsigned)((ncols + 63) / 64)), dim3(64), 0, s,
                       ncols, nchunks, part, out);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int gemv_small_f64(int64_t n, int k, const double *V, int64_t ldv, const double *h, double sign,
                   double *z, hipStream_t s) {
    if (n <= 0 || k <= 0) return 0;
    if (k > 256) {
        set_error_msg("gemv_small_f64: more than 256 columns");
        return MXLU_E_NOMEM;
    }
    hipLaunchKernelGGL(gemv_small_kernel, dim3(g1(n)), dim3(256), 0, s, n, k, V, ldv, h, sign, z);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int scale_copy_f64(int64_t n, const double *z, double alpha, double *v, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(scale_copy_kernel, dim3(g1(n)), dim3(256), 0, s, n, z, alpha, v);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int axpy_f64(int64_t n, const double *z, double *x, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(axpy_kernel, dim3(g1(n)), dim3(256), 0, s, n, z, x);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int absmax_f64(int64_t n, const double *v, unsigned long long *out, hipStream_t s) {
    if (n <= 0) return 0;
    const unsigned grid = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(absmax_kernel, dim3(grid), dim3(256), 0, s, n, v, out);
    MXLU_LAUNCH_CHECK();
    return 0;
}

template <int FMT, int KIND>
static int trsv_run(int64_t n, const uint16_t *F, int64_t ldf, float *v, hipStream_t s) {
    const int64_t nblk = (n + kTrsvBs - 1) / kTrsvBs;
    const bool fwd = (KIND == 0 || KIND == 2);
    const int dir = fwd ? 1 : -1;
    for (int64_t t = 0; t < nblk; ++t) {
        const int64_t cur = fwd ? t : nblk - 1 - t;
        const int64_t prev = (t == 0) ? -1 : cur - dir;
        const unsigned grid = (unsigned)(nblk - t);     // blocks cur, cur+dir, ...
        hipLaunchKernelGGL((trsv_step_kernel<FMT, KIND>), dim3(grid), dim3(256), 0, s, n, F, ldf, v,
                           prev, cur, (int)nblk, dir);
        MXLU_LAUNCH_CHECK();
    }
    return 0;
}

int lp_precond_apply(int fmt, int trans, int64_t n, const uint16_t *F, int64_t ldf,
                     const int32_t *perm, const double *r, double *d, float *v32,
                     unsigned long long *smax, hipStream_t s) {
    if (n <= 0) return 0;
    MXLU_HIP_TRY(hipMemsetAsync(smax, 0, sizeof(unsigned long long), s));
    MXLU_TRY(absmax_f64(n, r, smax, s));
    // forward: v = P r / s; L; U.   transposed: v = r / s; U^T; L^T; P^T v.
    hipLaunchKernelGGL(precond_in_kernel, dim3(g1(n)), dim3(256), 0, s, n, r,
                       trans ? nullptr : perm, smax, v32);
    MXLU_LAUNCH_CHECK();
    int rc;
    if (fmt == kFmtBf16) {
        rc = trans ? trsv_run<kFmtBf16, 2>(n, F, ldf, v32, s) : trsv_run<kFmtBf16, 0>(n, F, ldf, v32, s);
        if (!rc) rc = trans ? trsv_run<kFmtBf16, 3>(n, F, ldf, v32, s) : trsv_run<kFmtBf16, 1>(n, F, ldf, v32, s);
    } else {
        rc = trans ? trsv_run<kFmtFp16, 2>(n, F, ldf, v32, s) : trsv_run<kFmtFp16, 0>(n, F, ldf, v32, s);
        if (!rc) rc = trans ? trsv_run<kFmtFp16, 3>(n, F, ldf, v32, s) : trsv_run<kFmtFp16, 1>(n, F, ldf, v32, s);
    }
    if (rc) return rc;
    hipLaunchKernelGGL(precond_out_kernel, dim3(g1(n)), dim3(256), 0, s, n, v32,
                       trans ? perm : nullptr, smax, d);
    MXLU_LAUNCH_CHECK();
    return 0;
}

}  // namespace mxlu
