// Kernels of the FP64 iterative refinement (Sec. III-A.2: residuals and
// corrections in FP64; Sec. II-B: refinement based on GMRES) and of its
// preconditioner M = U^-1 L^-1 P applied in FP32 to the low-precision factors.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "asource.h"
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
// j); with asum, the |A[i, j]| row sums of the split go to asum_part.  The
// seeded form regenerates each A[i, j] from its counter (consecutive j of a
// row step the counter by G n), so the matrix is never read from memory; its
// terms are taken in the same order, so both forms give the same bits.
template <bool SEEDED>
__global__ __launch_bounds__(256) void gemv_n_partial_kernel(int64_t n, ASource src,
                                                             const double *__restrict__ x,
                                                             int64_t cps, double *__restrict__ part,
                                                             double *__restrict__ asum_part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.y * cps;
    const int64_t j1 = (j0 + cps < n) ? j0 + cps : n;
    if (i >= n) return;
    double acc = 0.0, as = 0.0;
    if constexpr (!SEEDED) {
        const double *__restrict__ A = src.A;
        const int64_t lda = src.lda;
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
    } else {
        // |a| sums of generator values are exact in any order (multiples of
        // 2^-32 below 2^21 in size), so the grouping above does not matter
        const uint64_t step = kGenGolden * (uint64_t)n;
        uint64_t z = src.key + kGenGolden * ((uint64_t)j0 * (uint64_t)n + (uint64_t)i + 1ull);
        for (int64_t j = j0; j < j1; ++j, z += step) {
            const double a = (src.diag && j == i) ? src.diag[i] : gen_value(z);
            acc = fma(a, x[j], acc);
            if (asum_part) as += fabs(a);
        }
    }
    part[(size_t)blockIdx.y * n + i] = acc;
    if (asum_part) asum_part[(size_t)blockIdx.y * n + i] = as;
}

// The same for a stored A with even lda and 16-byte alignment: two adjacent
// rows per thread (one 16-byte load per column covers both), each row's
// terms still in ascending j, eight columns per iteration in flight.
__global__ __launch_bounds__(256) void gemv_n_partial2_kernel(int64_t n, const double *__restrict__ A,
                                                              int64_t lda,
                                                              const double *__restrict__ x,
                                                              int64_t cps, double *__restrict__ part,
                                                              double *__restrict__ asum_part) {
    const int64_t i = 2 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
    const int64_t j0 = (int64_t)blockIdx.y * cps;
    const int64_t j1 = (j0 + cps < n) ? j0 + cps : n;
    if (i >= n) return;
    double acc0 = 0.0, acc1 = 0.0, as0 = 0.0, as1 = 0.0;
    if (i + 1 < n) {
        int64_t j = j0;
        for (; j + 8 <= j1; j += 8) {
            double2 a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                a[q] = *reinterpret_cast<const double2 *>(&A[(size_t)i + (size_t)(j + q) * lda]);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double xq = x[j + q];
                acc0 = fma(a[q].x, xq, acc0);
                acc1 = fma(a[q].y, xq, acc1);
            }
            if (asum_part) {
                // the same grouping as the one-row form: four terms, then added
#pragma unroll
                for (int h = 0; h < 8; h += 4) {
                    as0 += fabs(a[h].x) + fabs(a[h + 1].x) + fabs(a[h + 2].x) + fabs(a[h + 3].x);
                    as1 += fabs(a[h].y) + fabs(a[h + 1].y) + fabs(a[h + 2].y) + fabs(a[h + 3].y);
                }
            }
        }
        for (; j + 4 <= j1; j += 4) {
            double2 a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a[q] = *reinterpret_cast<const double2 *>(&A[(size_t)i + (size_t)(j + q) * lda]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double xq = x[j + q];
                acc0 = fma(a[q].x, xq, acc0);
                acc1 = fma(a[q].y, xq, acc1);
            }
            if (asum_part) {
                as0 += fabs(a[0].x) + fabs(a[1].x) + fabs(a[2].x) + fabs(a[3].x);
                as1 += fabs(a[0].y) + fabs(a[1].y) + fabs(a[2].y) + fabs(a[3].y);
            }
        }
        for (; j < j1; ++j) {
            const double2 a = *reinterpret_cast<const double2 *>(&A[(size_t)i + (size_t)j * lda]);
            acc0 = fma(a.x, x[j], acc0);
            acc1 = fma(a.y, x[j], acc1);
            if (asum_part) {
                as0 += fabs(a.x);
                as1 += fabs(a.y);
            }
        }
        part[(size_t)blockIdx.y * n + i + 1] = acc1;
        if (asum_part) asum_part[(size_t)blockIdx.y * n + i + 1] = as1;
    } else {   // the last row of an odd n
        int64_t j = j0;
        for (; j + 4 <= j1; j += 4) {
            const double a0 = MXLU_AT(A, i, j, lda), a1 = MXLU_AT(A, i, j + 1, lda);
            const double a2 = MXLU_AT(A, i, j + 2, lda), a3 = MXLU_AT(A, i, j + 3, lda);
            acc0 = fma(a0, x[j], acc0);
            acc0 = fma(a1, x[j + 1], acc0);
            acc0 = fma(a2, x[j + 2], acc0);
            acc0 = fma(a3, x[j + 3], acc0);
            if (asum_part) as0 += fabs(a0) + fabs(a1) + fabs(a2) + fabs(a3);
        }
        for (; j < j1; ++j) {
            const double a = MXLU_AT(A, i, j, lda);
            acc0 = fma(a, x[j], acc0);
            if (asum_part) as0 += fabs(a);
        }
    }
    part[(size_t)blockIdx.y * n + i] = acc0;
    if (asum_part) asum_part[(size_t)blockIdx.y * n + i] = as0;
}

// Transposed: part[s][i] = sum over rows j of split s of A[j, i] x[j]; one
// wave per i (column i of A is contiguous).
template <bool SEEDED>
__global__ __launch_bounds__(256) void gemv_t_partial_kernel(int64_t n, ASource src,
                                                             const double *__restrict__ x,
                                                             int64_t cps, double *__restrict__ part,
                                                             double *__restrict__ asum_part) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t j0 = (int64_t)blockIdx.y * cps;
    const int64_t j1 = (j0 + cps < n) ? j0 + cps : n;
    if (i >= n) return;
    double acc = 0.0, as = 0.0;
    if constexpr (!SEEDED) {
        for (int64_t j = j0 + lane; j < j1; j += 64) {
            const double a = MXLU_AT(src.A, j, i, src.lda);
            acc = fma(a, x[j], acc);
            as += fabs(a);
        }
    } else {
        uint64_t z = src.key + kGenGolden * ((uint64_t)i * (uint64_t)n + (uint64_t)(j0 + lane) + 1ull);
        for (int64_t j = j0 + lane; j < j1; j += 64, z += 64ull * kGenGolden) {
            const double a = (src.diag && j == i) ? src.diag[i] : gen_value(z);
            acc = fma(a, x[j], acc);
            as += fabs(a);
        }
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

// Blocked triangular solve in FP32 with the stored factor F (16-bit), blocks
// of kTrsvBs rows, in one launch.  Workgroup w owns the w-th block in solve
// order: it stages its diagonal block in LDS, then, for every earlier block
// in solve order, waits for that block's solution and applies it to its own
// rows (thread = row), then solves its diagonal block with one wave and
// publishes the solution.  Every element accumulates its terms in the order
// of the textbook substitution (column-oriented for L and U: ascending k for
// L, descending k for U; ascending i for the transposed forms).
//   kind 0: L (unit lower), forward;   kind 1: U (upper), backward
//   kind 2: U^T (lower), forward;      kind 3: L^T (unit upper), backward
// Publication: each solved value goes to xs as a 64-bit word holding the
// float's bits and, in the upper half, the launch's tag; writers and readers
// use agent-scope relaxed atomics and a reader polls each word until it
// carries the tag, so no fences are needed.  Tags are unique per launch, so
// words of earlier solves never match.  Workgroup w waits only on
// workgroups with smaller ids, which are dispatched first, so the chain
// always progresses even when not all workgroups are resident.  The polling
// is bounded: on expiry *expired is set and the solve completes with
// invalid values.
__device__ __forceinline__ uint64_t ll_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier that orders LDS only, so that global loads issued before it stay in
// flight across it (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int FMT, int KIND>
__global__ __launch_bounds__(256) void trsv_chain_kernel(int64_t n, const uint16_t *__restrict__ F,
                                                         int64_t ldf, float *__restrict__ v,
                                                         uint64_t *xs, uint32_t tag, int nblk,
                                                         int *expired) {
    constexpr int BS = kTrsvBs;
    constexpr bool FWD = (KIND == 0 || KIND == 2);
    constexpr bool UNIT = (KIND == 0 || KIND == 3);
    __shared__ uint16_t Ld[BS][BS + 2];   // raw stored values (129 KB)
    __shared__ float xprev[BS];
    // column-major kinds: 32 columns x 256 rows of an earlier block, staged
    // with 16-byte loads so that each thread can read its row
    __shared__ __attribute__((aligned(16))) uint16_t stg[32][BS];
    const int tid = threadIdx.x;
    const int w = blockIdx.x;
    const int64_t myblk = FWD ? w : nblk - 1 - w;
    const int64_t r0 = myblk * BS;
    const int rows = (int)((n - r0 < BS) ? n - r0 : BS);
    const int64_t i = r0 + tid;          // this thread's row

    // diagonal block, staged as the effective lower/upper factor
    for (int t = tid; t < rows * rows; t += 256) {
        const int ii = t % rows, k = t / rows;
        const uint16_t f = F[(size_t)(r0 + ii) + (size_t)(r0 + k) * ldf];
        if (KIND == 0 || KIND == 1) Ld[ii][k] = f;
        else Ld[k][ii] = f;     // transposed forms: Ld[i][k] = F[k][i]
    }
    float acc = (tid < rows) ? v[i] : 0.0f;
    constexpr bool COLMAJOR = (KIND == 0 || KIND == 1);
    // column-major kinds, full blocks: chunk cc (32 columns of the earlier
    // block) is loaded as 4 x 16 bytes per thread (8 rows of one column each)
    auto ld_chunk = [&](int64_t p0, int cc, uint4 (&g)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q, col = idx >> 5, rg = idx & 31;
            const uint16_t *src = &F[(size_t)(r0 + 8 * rg) + (size_t)(p0 + 32 * cc + col) * ldf];
            if (8 * rg + 8 <= rows) {
                g[q] = *reinterpret_cast<const uint4 *>(src);
            } else {   // rows past the matrix (last block): zeros
                uint16_t h[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) h[e] = (8 * rg + e < rows) ? src[e] : (uint16_t)0;
                g[q] = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                                  h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
            }
        }
    };
    auto chunk_of = [&](int c) { return (KIND == 1) ? 7 - c : c; };   // solve order
    auto apply_chunk = [&](int cc, const uint4 (&g)[4]) {
        lds_barrier();   // the previous chunk is consumed
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = tid + 256 * q, col = idx >> 5, rg = idx & 31;
            *reinterpret_cast<uint4 *>(&stg[col][8 * rg]) = g[q];
        }
    };
    auto fma_chunk = [&](int cc) {
        if (KIND == 0) {
#pragma unroll
            for (int kk = 0; kk < 32; ++kk)
                acc = fmaf(-lp_to_f32<FMT>(stg[kk][tid]), xprev[32 * cc + kk], acc);
        } else {
#pragma unroll
            for (int kk = 31; kk >= 0; --kk)
                acc = fmaf(-lp_to_f32<FMT>(stg[kk][tid]), xprev[32 * cc + kk], acc);
        }
    };
    // transposed kinds: fr holds the thread's row of the earlier block, F
    // values for k = 2j, 2j+1 packed in one word, loaded before the wait
    uint32_t fr[COLMAJOR ? 1 : BS / 2];
    // column-major kinds: gb holds the 8 chunks of the next full earlier
    // block; slot c is refilled with the following block's chunk c as soon
    // as it is staged, so a whole block of loads is in flight while the
    // current one is applied
    constexpr int NG = COLMAJOR ? 8 : 1;
    uint4 gb[NG][4];
    uint32_t cr[NG][16];
    bool have = false;   // gb holds the current earlier block
    for (int t = 0; t < w; ++t) {
        const int64_t pb = FWD ? t : nblk - 1 - t;
        const int64_t p0 = pb * BS;
        const int pr = (int)((n - p0 < BS) ? n - p0 : BS);
        const bool full = (pr == BS);   // the earlier block is full
        // the last earlier block is on the chain's critical path: its values
        // move into registers (the thread's row, two values per word) while
        // its solution is still awaited, so that only its multiply-adds follow
        // the arrival
        const bool last = COLMAJOR && full && t == w - 1;
        if (full) {
            if (COLMAJOR) {
                if (!have)
#pragma unroll
                    for (int c = 0; c < NG; ++c) ld_chunk(p0, chunk_of(c), gb[c]);
                if (last) {
#pragma unroll
                    for (int c = 0; c < NG; ++c) {
                        apply_chunk(chunk_of(c), gb[c]);
                        lds_barrier();
#pragma unroll
                        for (int q = 0; q < 16; ++q)
                            cr[c][q] = (uint32_t)stg[2 * q][tid] | ((uint32_t)stg[2 * q + 1][tid] << 16);
                    }
                }
            } else if (tid < rows) {   // F[k][i] for k in the earlier block: contiguous in k
                const uint4 *q = reinterpret_cast<const uint4 *>(&F[(size_t)p0 + (size_t)i * ldf]);
#pragma unroll
                for (int j = 0; j < BS / 8; ++j) {
                    const uint4 u = q[j];
                    fr[4 * j] = u.x;
                    fr[4 * j + 1] = u.y;
                    fr[4 * j + 2] = u.z;
                    fr[4 * j + 3] = u.w;
                }
            }
        }
        lds_barrier();   // the previous block's values are consumed
        // one thread watches the block's first word (many pollers on the same
        // lines would slow the producer's stores); then every thread reads
        // its word, which has normally arrived by then
        if (tid == 0) {
            const uint64_t *src = &xs[p0];
            uint64_t x = ll_load(src);
            long spins = 0;
            while ((uint32_t)(x >> 32) != tag) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1L << 26)) {
                    atomicExch(expired, 1);
                    break;
                }
                x = ll_load(src);
            }
        }
        lds_barrier();
        if (tid < pr) {
            const uint64_t *src = &xs[p0 + tid];
            uint64_t x = ll_load(src);
            long spins = 0;
            while ((uint32_t)(x >> 32) != tag) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1L << 26)) {
                    atomicExch(expired, 1);
                    break;
                }
                x = ll_load(src);
            }
            xprev[tid] = __uint_as_float((uint32_t)x);
        }
        lds_barrier();
        if (last) {
            // the same terms in the same order as fma_chunk over the chunks
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                const int cc = chunk_of(c);
                if (KIND == 0) {
#pragma unroll
                    for (int kk = 0; kk < 32; ++kk)
                        acc = fmaf(-lp_to_f32<FMT>((uint16_t)(cr[c][kk >> 1] >> (16 * (kk & 1)))),
                                   xprev[32 * cc + kk], acc);
                } else {
#pragma unroll
                    for (int kk = 31; kk >= 0; --kk)
                        acc = fmaf(-lp_to_f32<FMT>((uint16_t)(cr[c][kk >> 1] >> (16 * (kk & 1)))),
                                   xprev[32 * cc + kk], acc);
                }
            }
            have = false;
        } else if (full && COLMAJOR) {
            // chunks in solve order; each staged chunk's slot takes the next
            // earlier block's chunk (when that block is full)
            const int64_t pn = FWD ? t + 1 : nblk - 2 - t;
            const bool next = t + 1 < w && (n - pn * BS >= BS);
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                apply_chunk(chunk_of(c), gb[c]);
                if (next) ld_chunk(pn * BS, chunk_of(c), gb[c]);
                lds_barrier();
                fma_chunk(chunk_of(c));
            }
            have = next;
        } else if (full && tid < rows) {
            // U^T, L^T: k ascending
#pragma unroll
            for (int j = 0; j < BS / 2; ++j) {
                acc = fmaf(-lp_to_f32<FMT>((uint16_t)fr[j]), xprev[2 * j], acc);
                acc = fmaf(-lp_to_f32<FMT>((uint16_t)(fr[j] >> 16)), xprev[2 * j + 1], acc);
            }
        } else if (tid < rows) {   // a partial block (the last one of n)
            if (KIND == 0) {
                for (int k = 0; k < pr; ++k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)i + (size_t)(p0 + k) * ldf]), xprev[k], acc);
            } else if (KIND == 1) {
                for (int k = pr - 1; k >= 0; --k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)i + (size_t)(p0 + k) * ldf]), xprev[k], acc);
            } else {
                for (int k = 0; k < pr; ++k)
                    acc = fmaf(-lp_to_f32<FMT>(F[(size_t)(p0 + k) + (size_t)i * ldf]), xprev[k], acc);
            }
        }
    }
    // Diagonal block: four sub-blocks of 64 rows in solve order.  Wave sb
    // owns the rows of sub-block sb (thread = row, as above): it solves them
    // (step j finishes x_k on its owner lane, division for U, and broadcasts
    // it with readlane; the LDS value of step j + 1 is read during step j),
    // publishes them in LDS, and the waves of the sub-blocks still to be
    // solved apply them to their rows, k in solve order.  Every element still
    // takes its terms in the textbook order.
    constexpr int NSB = BS / 64;
    const int wave = tid >> 6;
    float x = acc;
    const bool mine = tid < rows;
    __syncthreads();   // xprev is reused for the solution
#pragma unroll
    for (int s = 0; s < NSB; ++s) {
        const int sb = FWD ? s : NSB - 1 - s;
        const int base = sb * 64;
        const int len = min(64, rows - base);   // rows of this sub-block (<= 0: none)
        if (wave == sb && len == 64) {
            // full sub-block: the lane's row of it in registers, steps unrolled
            const int lane = tid & 63;
            uint32_t rr[32];
#pragma unroll
            for (int p = 0; p < 32; ++p)
                rr[p] = *reinterpret_cast<const uint32_t *>(&Ld[tid][base + 2 * p]);
            // every lane applies every step (the update of a lane already
            // solved is never read again); each lane's finished value is kept
            // aside at its own step, off the dependency chain
            //
            // U (non-unit): the quotient x / d of a step comes from r = RN(1/d),
            // the reciprocal of the lane's own diagonal entry computed ahead of
            // the chain: q0 = RN(x r), q = RN(q0 + (x - q0 d) r) with both
            // corrections fused multiply-adds.  While every value stays in the
            // normal range that is the correctly rounded quotient (Markstein's
            // theorem for a reciprocal rounded to nearest; also checked against
            // the division on 4e8 operand pairs, quotients at rounding
            // midpoints and divisors with all-ones significands included, and
            // scale-invariant away from underflow and overflow).  Each lane
            // keeps the value it divided; after the 64 steps one vote checks
            // |x| >= 2^-100 (or x == 0), |q| within [2^-99, 2^99] and |d| within
            // [2^-100, 2^100], and if any lane is outside, the sub-block is
            // solved again with the division: the result is the division's bit
            // for bit either way.
            const float x_in = x;
            const float dl = lp_to_f32<FMT>(Ld[tid][tid]);
            const float rdiag = UNIT ? 1.0f : 1.0f / dl;
            float xfin = x, xo = x;
#pragma unroll
            for (int j = 0; j < 64; ++j) {
                const int kl = FWD ? j : 63 - j;
                const uint32_t w2 = rr[kl >> 1];
                const float lv = lp_to_f32<FMT>((uint16_t)((kl & 1) ? (w2 >> 16) : w2));
                // on the owner lane lv is the diagonal entry
                float own = x;
                if (!UNIT) {
                    const float q0 = x * rdiag;
                    own = fmaf(fmaf(-q0, lv, x), rdiag, q0);
                    xo = (lane == kl) ? x : xo;
                }
                const float xk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(own), kl));
                xfin = (lane == kl) ? xk : xfin;
                x = fmaf(-lv, xk, x);
            }
            x = xfin;
            if (!UNIT) {
                const float ax = fabsf(xo), aq = fabsf(xfin), ad = fabsf(dl);
                const bool in = (xo == 0.0f || (ax >= 0x1p-100f && aq >= 0x1p-99f && aq <= 0x1p99f)) &&
                                ad >= 0x1p-100f && ad <= 0x1p100f;
                if (!__all(in)) {   // wave-uniform; never taken on scaled inputs
                    x = x_in;
                    xfin = x;
                    for (int j = 0; j < 64; ++j) {
                        const int kl = FWD ? j : 63 - j;
                        const float lv = lp_to_f32<FMT>(Ld[tid][base + kl]);
                        const float own = x / lv;
                        const float xk =
                            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(own), kl));
                        xfin = (lane == kl) ? xk : xfin;
                        x = fmaf(-lv, xk, x);
                    }
                    x = xfin;
                }
            }
            xprev[tid] = x;
        } else if (wave == sb && len > 0) {
            auto kat = [&](int j) { return FWD ? base + j : base + len - 1 - j; };
            // raw values of step j + 1 are read during step j (unconditionally:
            // every thread's row is inside the LDS block; rows past the
            // matrix are never stored)
            uint16_t lc = Ld[tid][kat(0)], dc = Ld[kat(0)][kat(0)];
            for (int j = 0; j < len; ++j) {
                const int k = kat(j);
                const int k1 = kat(j + 1 < len ? j + 1 : j);
                const uint16_t ln = Ld[tid][k1], dn = Ld[k1][k1];
                const float own = UNIT ? x : x / lp_to_f32<FMT>(dc);
                const float xk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(own), k - base));
                const float upd = fmaf(-lp_to_f32<FMT>(lc), xk, x);
                const bool later = FWD ? tid > k : tid < k;
                x = (tid == k) ? xk : (later ? upd : x);
                lc = ln;
                dc = dn;
            }
            xprev[tid] = x;
        }
        __syncthreads();
        if (len > 0 && (FWD ? wave > sb : wave < sb) && mine) {
            if (FWD) {
                for (int j = 0; j < len; ++j)
                    x = fmaf(-lp_to_f32<FMT>(Ld[tid][base + j]), xprev[base + j], x);
            } else {
                for (int j = len - 1; j >= 0; --j)
                    x = fmaf(-lp_to_f32<FMT>(Ld[tid][base + j]), xprev[base + j], x);
            }
        }
    }
    if (mine) {
        v[i] = x;
        __hip_atomic_store(&xs[i], ((uint64_t)tag << 32) | __float_as_uint(x), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}

unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

// FP32-storage preconditioner: the factors are FP32 numbers, solved block by
// block (kTrsv32Bs rows) in solve order with two launches per block: one
// workgroup solves the diagonal block (its rows staged in LDS, thread = row,
// each finished value broadcast through LDS), then a grid applies the block's
// solution to the rows still to be solved (thread = row, the block's values in
// LDS, the factor streamed column by column).  Every element takes its terms in
// the order of the column-oriented substitution: ascending k for L, descending
// k for U (then the division by the diagonal), one fused multiply-add each.
constexpr int kTrsv32Bs = 128;

template <bool LOWER>
__global__ __launch_bounds__(kTrsv32Bs) void trsv_f32_diag_kernel(const float *__restrict__ F,
                                                                  int64_t ldf, int64_t b0,
                                                                  int rows, float *__restrict__ v) {
    __shared__ float Ld[kTrsv32Bs][kTrsv32Bs + 1];
    __shared__ float xk[2];
    const int t = threadIdx.x;
    for (int c = 0; c < rows; ++c)
        if (t < rows) Ld[t][c] = F[(size_t)(b0 + t) + (size_t)(b0 + c) * ldf];
    __syncthreads();
    float x = t < rows ? v[b0 + t] : 0.0f;
    // slot k & 1 is rewritten at step k + 2, after every thread has passed the
    // barrier of step k + 1 and so has read it at step k
    if constexpr (LOWER) {
        for (int k = 0; k < rows; ++k) {
            if (t == k) xk[k & 1] = x;
            __syncthreads();
            const float xv = xk[k & 1];
            if (t > k && t < rows) x = fmaf(-Ld[t][k], xv, x);
        }
    } else {
        for (int k = rows - 1; k >= 0; --k) {
            if (t == k) {
                x = x / Ld[k][k];
                xk[k & 1] = x;
            }
            __syncthreads();
            const float xv = xk[k & 1];
            if (t < k) x = fmaf(-Ld[t][k], xv, x);
        }
    }
    if (t < rows) v[b0 + t] = x;
}

// rows i >= b0 + rows (LOWER) or i < b0 (upper): v_i -= sum over the block
template <bool LOWER>
__global__ __launch_bounds__(256) void trsv_f32_apply_kernel(int64_t n, const float *__restrict__ F,
                                                             int64_t ldf, int64_t b0, int rows,
                                                             float *__restrict__ v) {
    __shared__ float xb[kTrsv32Bs];
    const int t = threadIdx.x;
    if (t < rows) xb[t] = v[b0 + t];
    __syncthreads();
    const int64_t i = (LOWER ? b0 + rows : 0) + (int64_t)blockIdx.x * 256 + t;
    if (i >= (LOWER ? n : b0)) return;
    float x = v[i];
    if constexpr (LOWER) {
#pragma unroll 16
        for (int k = 0; k < rows; ++k) x = fmaf(-F[(size_t)i + (size_t)(b0 + k) * ldf], xb[k], x);
    } else {
#pragma unroll 16
        for (int k = rows - 1; k >= 0; --k)
            x = fmaf(-F[(size_t)i + (size_t)(b0 + k) * ldf], xb[k], x);
    }
    v[i] = x;
}

}  // namespace

namespace mxlu {

int gemv_f64(int trans, int64_t n, const ASource &src, const double *x,
             const double *b, double *y, double *part, double *asum_part, int nsplit,
             unsigned long long *stats, hipStream_t s) {
    if (n <= 0) return 0;
    const int64_t cps = (n + nsplit - 1) / nsplit;
    const dim3 gn(g1(n), (unsigned)nsplit), gt((unsigned)((n + 3) / 4), (unsigned)nsplit);
    if (trans == 0 && !src.seeded() && src.lda % 2 == 0 && (uintptr_t)src.A % 16 == 0)
        hipLaunchKernelGGL(gemv_n_partial2_kernel, dim3((unsigned)((n + 511) / 512), (unsigned)nsplit),
                           dim3(256), 0, s, n, src.A, src.lda, x, cps, part, asum_part);
    else if (trans == 0 && !src.seeded())
        hipLaunchKernelGGL(gemv_n_partial_kernel<false>, gn, dim3(256), 0, s, n, src, x, cps, part,
                           asum_part);
    else if (trans == 0)
        hipLaunchKernelGGL(gemv_n_partial_kernel<true>, gn, dim3(256), 0, s, n, src, x, cps, part,
                           asum_part);
    else if (!src.seeded())
        hipLaunchKernelGGL(gemv_t_partial_kernel<false>, gt, dim3(256), 0, s, n, src, x, cps, part,
                           asum_part);
    else
        hipLaunchKernelGGL(gemv_t_partial_kernel<true>, gt, dim3(256), 0, s, n, src, x, cps, part,
                           asum_part);
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
static int trsv_run(int64_t n, const uint16_t *F, int64_t ldf, float *v, TrsvChain &ch,
                    hipStream_t s) {
    const int64_t nblk = (n + kTrsvBs - 1) / kTrsvBs;
    if (nblk > 0x7fffffff) {
        set_error_msg("trsv: too many blocks");
        return MXLU_E_NOMEM;
    }
    if (((uintptr_t)F % 16) || (ldf % 8)) {
        set_error_msg("trsv: factor storage must be 16-byte aligned with ldf % 8 == 0");
        return MXLU_E_NOMEM;
    }
    const uint32_t tag = ++ch.tag;
    hipLaunchKernelGGL((trsv_chain_kernel<FMT, KIND>), dim3((unsigned)nblk), dim3(256), 0, s, n, F,
                       ldf, v, ch.xs, tag, (int)nblk, ch.expired);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_precond_apply_f32(int64_t n, const float *F, int64_t ldf, const int32_t *perm,
                         const double *r, double *d, float *v32, unsigned long long *smax,
                         hipStream_t s) {
    if (n <= 0) return 0;
    MXLU_HIP_TRY(hipMemsetAsync(smax, 0, sizeof(unsigned long long), s));
    MXLU_TRY(absmax_f64(n, r, smax, s));
    hipLaunchKernelGGL(precond_in_kernel, dim3(g1(n)), dim3(256), 0, s, n, r, perm, smax, v32);
    MXLU_LAUNCH_CHECK();
    for (int64_t b0 = 0; b0 < n; b0 += kTrsv32Bs) {   // L, forward
        const int rows = (int)std::min<int64_t>(kTrsv32Bs, n - b0);
        hipLaunchKernelGGL(trsv_f32_diag_kernel<true>, dim3(1), dim3(kTrsv32Bs), 0, s, F, ldf, b0,
                           rows, v32);
        MXLU_LAUNCH_CHECK();
        const int64_t below = n - b0 - rows;
        if (below > 0) {
            hipLaunchKernelGGL(trsv_f32_apply_kernel<true>, dim3((unsigned)((below + 255) / 256)),
                               dim3(256), 0, s, n, F, ldf, b0, rows, v32);
            MXLU_LAUNCH_CHECK();
        }
    }
    for (int64_t b0 = (n - 1) / kTrsv32Bs * kTrsv32Bs; b0 >= 0; b0 -= kTrsv32Bs) {   // U, backward
        const int rows = (int)std::min<int64_t>(kTrsv32Bs, n - b0);
        hipLaunchKernelGGL(trsv_f32_diag_kernel<false>, dim3(1), dim3(kTrsv32Bs), 0, s, F, ldf, b0,
                           rows, v32);
        MXLU_LAUNCH_CHECK();
        if (b0 > 0) {
            hipLaunchKernelGGL(trsv_f32_apply_kernel<false>, dim3((unsigned)((b0 + 255) / 256)),
                               dim3(256), 0, s, n, F, ldf, b0, rows, v32);
            MXLU_LAUNCH_CHECK();
        }
    }
    hipLaunchKernelGGL(precond_out_kernel, dim3(g1(n)), dim3(256), 0, s, n, v32, nullptr, smax,
                       d);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_precond_apply(int fmt, int trans, int64_t n, const uint16_t *F, int64_t ldf,
                     const int32_t *perm, const double *r, double *d, float *v32,
                     unsigned long long *smax, TrsvChain &ch, hipStream_t s) {
    if (n <= 0) return 0;
    MXLU_HIP_TRY(hipMemsetAsync(smax, 0, sizeof(unsigned long long), s));
    MXLU_TRY(absmax_f64(n, r, smax, s));
    // forward: v = P r / s; L; U.   transposed: v = r / s; U^T; L^T; P^T v.
    hipLaunchKernelGGL(precond_in_kernel, dim3(g1(n)), dim3(256), 0, s, n, r,
                       trans ? nullptr : perm, smax, v32);
    MXLU_LAUNCH_CHECK();
    int rc;
    if (fmt == kFmtBf16) {
        rc = trans ? trsv_run<kFmtBf16, 2>(n, F, ldf, v32, ch, s) : trsv_run<kFmtBf16, 0>(n, F, ldf, v32, ch, s);
        if (!rc) rc = trans ? trsv_run<kFmtBf16, 3>(n, F, ldf, v32, ch, s) : trsv_run<kFmtBf16, 1>(n, F, ldf, v32, ch, s);
    } else {
        rc = trans ? trsv_run<kFmtFp16, 2>(n, F, ldf, v32, ch, s) : trsv_run<kFmtFp16, 0>(n, F, ldf, v32, ch, s);
        if (!rc) rc = trans ? trsv_run<kFmtFp16, 3>(n, F, ldf, v32, ch, s) : trsv_run<kFmtFp16, 1>(n, F, ldf, v32, ch, s);
    }
    if (rc) return rc;
    hipLaunchKernelGGL(precond_out_kernel, dim3(g1(n)), dim3(256), 0, s, n, v32,
                       trans ? perm : nullptr, smax, d);
    MXLU_LAUNCH_CHECK();
    return 0;
}

}  // namespace mxlu
