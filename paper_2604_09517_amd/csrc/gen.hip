// Seeded synthetic inputs in HBM, and the FP64 scaled-residual check.
//
// Generator: SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014) used as
// a counter-based hash; written here from that definition, independently of
// the host implementation it is tested against.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "asource.h"
#include "common.h"

namespace {

constexpr uint64_t kGolden = mxlu::kGenGolden;

__host__ __device__ inline uint64_t splitmix_finalise(uint64_t z) { return mxlu::gen_mix(z); }

// One thread per element of a column strip; grid.y walks column blocks.
__global__ void fill_uniform_kernel(int64_t rows, int64_t cols, double *A,
                                    int64_t lda, uint64_t key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        const uint64_t idx = (uint64_t)j * (uint64_t)rows + (uint64_t)i;
        const uint64_t h = splitmix_finalise(key + kGolden * (idx + 1ull));
        // top 32 bits times 2^-32, minus 1/2: exact in FP64
        MXLU_AT(A, i, j, lda) = (double)(h >> 32) * 0x1p-32 - 0.5;
    }
}

// Row sums of |a_ij| over j != i, one thread per row (coalesced across the
// rows of each column).  Generator values are multiples of 2^-32 of size
// <= 1/2, so the sum is exact for n < 2^21 and independent of order.
__global__ void diag_dominant_kernel(int64_t n, double *A, int64_t lda) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j)
        if (j != i) s += fabs(MXLU_AT(A, i, j, lda));
    MXLU_AT(A, i, i, lda) = s;
}

// The diagonal of the seeded diagonally dominant matrix without storing the
// matrix: diag[i] = sum over j != i of |u(j n + i)| (exact in any order, as
// above), one thread per row.
__global__ void gen_dominant_diag_kernel(int64_t n, uint64_t key, double *diag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t step = kGolden * (uint64_t)n;
    uint64_t z = key + kGolden * ((uint64_t)i + 1ull);
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j, z += step)
        if (j != i) s += fabs(mxlu::gen_value(z));
    diag[i] = s;
}

// Residual check: per row i and column c, r = b - sum_j op(A)_ij x_j and the
// row's |op(A)| sum; partial maxima are combined with atomics on the bit
// patterns of non-negative doubles (monotone as unsigned integers).
__global__ void residual_rows_kernel(int64_t n, const double *A, int64_t lda,
                                     const double *X, int64_t ldx,
                                     const double *B, int64_t ldb, int c,
                                     unsigned long long *out /*[3]: |r|, |A|row, */) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *x = X + (size_t)c * (size_t)ldx;
    double acc = B[(size_t)c * (size_t)ldb + i];
    double asum = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        const double a = MXLU_AT(A, i, j, lda);
        acc = fma(-a, x[j], acc);
        asum += fabs(a);
    }
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(fabs(acc)));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(asum));
}

// Transposed: row i of A^T is column i of A (contiguous); one wave per i.
__global__ void residual_cols_kernel(int64_t n, const double *A, int64_t lda,
                                     const double *X, int64_t ldx,
                                     const double *B, int64_t ldb, int c,
                                     unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    const double *x = X + (size_t)c * (size_t)ldx;
    double acc = 0.0, asum = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
        const double a = MXLU_AT(A, j, i, lda);
        acc = fma(a, x[j], acc);
        asum += fabs(a);
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off);
        asum += __shfl_xor(asum, off);
    }
    if (lane == 0) {
        const double r = B[(size_t)c * (size_t)ldb + i] - acc;
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(fabs(r)));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(asum));
    }
}

__global__ void absmax_kernel(int64_t n, const double *v, unsigned long long *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0;
    for (int64_t k = i; k < n; k += (int64_t)gridDim.x * blockDim.x) m = fmax(m, fabs(v[k]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

}  // namespace

namespace mxlu {
int gen_dominant_diag(int64_t n, uint64_t key, double *diag, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(gen_dominant_diag_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, n, key, diag);
    MXLU_LAUNCH_CHECK();
    return 0;
}
}  // namespace mxlu

extern "C" int mxlu_fill_uniform(int64_t rows, int64_t cols, double *A,
                                 int64_t lda, uint64_t seed, uint64_t stream_id,
                                 void *stream) {
    if (rows < 0) return -1;
    if (cols < 0) return -2;
    if (rows > 0 && cols > 0 && !A) return -3;
    if (lda < (rows > 1 ? rows : 1)) return -4;
    if (rows == 0 || cols == 0) return 0;
    if (int rc = mxlu::check_device()) return rc;
    const uint64_t key = splitmix_finalise(seed + kGolden * (stream_id + 1ull));
    dim3 grid((unsigned)((rows + 255) / 256), (unsigned)(cols < 8192 ? cols : 8192));
    hipLaunchKernelGGL(fill_uniform_kernel, grid, dim3(256), 0, (hipStream_t)stream,
                       rows, cols, A, lda, key);
    MXLU_LAUNCH_CHECK();
    return 0;
}

extern "C" int mxlu_make_diag_dominant(int64_t n, double *A, int64_t lda, void *stream) {
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n == 0) return 0;
    if (int rc = mxlu::check_device()) return rc;
    hipLaunchKernelGGL(diag_dominant_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, n, A, lda);
    MXLU_LAUNCH_CHECK();
    return 0;
}

extern "C" int mxlu_scaled_residual(int64_t n, int64_t nrhs, const double *A,
                                    int64_t lda, const double *X, int64_t ldx,
                                    const double *B, int64_t ldb, int trans,
                                    double *out, void *stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && nrhs > 0 && !X) return -5;
    if (ldx < (n > 1 ? n : 1)) return -6;
    if (n > 0 && nrhs > 0 && !B) return -7;
    if (ldb < (n > 1 ? n : 1)) return -8;
    if (trans != 0 && trans != 1) return -9;
    if (nrhs > 0 && !out) return -10;
    if (n == 0 || nrhs == 0) {
        for (int64_t c = 0; c < nrhs; ++c) out[c] = 0.0;
        return 0;
    }
    if (int rc = mxlu::check_device()) return rc;
    hipStream_t s = (hipStream_t)stream;
    mxlu::Scratch scratch(s);
    unsigned long long *d = scratch.alloc_n<unsigned long long>(4 * (size_t)nrhs);
    if (!d) return MXLU_E_NOMEM;
    MXLU_HIP_TRY(hipMemsetAsync(d, 0, 4 * sizeof(unsigned long long) * (size_t)nrhs, s));
    for (int64_t c = 0; c < nrhs; ++c) {
        unsigned long long *o = d + 4 * c;
        if (trans == 0)
            hipLaunchKernelGGL(residual_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256),
                               0, s, n, A, lda, X, ldx, B, ldb, (int)c, o);
        else
            hipLaunchKernelGGL(residual_cols_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0,
                               s, n, A, lda, X, ldx, B, ldb, (int)c, o);
        MXLU_LAUNCH_CHECK();
        hipLaunchKernelGGL(absmax_kernel, dim3(64), dim3(256), 0, s, n, X + (size_t)c * ldx, o + 2);
        hipLaunchKernelGGL(absmax_kernel, dim3(64), dim3(256), 0, s, n, B + (size_t)c * ldb, o + 3);
        MXLU_LAUNCH_CHECK();
    }
    unsigned long long h[4 * 64];
    for (int64_t c0 = 0; c0 < nrhs; c0 += 64) {
        const int64_t cnt = (nrhs - c0 < 64) ? nrhs - c0 : 64;
        MXLU_HIP_TRY(hipMemcpyAsync(h, d + 4 * c0, 4 * sizeof(unsigned long long) * cnt,
                                    hipMemcpyDeviceToHost, s));
        MXLU_HIP_TRY(hipStreamSynchronize(s));
        for (int64_t c = 0; c < cnt; ++c) {
            double v[4];
            for (int k = 0; k < 4; ++k) {
                long long bits = (long long)h[4 * c + k];
                std::memcpy(&v[k], &bits, sizeof(double));
            }
            const double eps = 0x1p-53;
            const double den = eps * (v[1] * v[2] + v[3]) * (double)n;
            out[c0 + c] = den > 0 ? v[0] / den : (v[0] > 0 ? INFINITY : 0.0);
        }
    }
    return 0;
}
