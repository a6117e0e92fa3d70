// FP64 kernels of the right-looking LU other than the panel leaves
// (panel_leaf.hip) and the trailing GEMM (gemm_f64.hip):
//   SWAP   row interchanges (composed, then applied column-strip-wise),
//   DTRSM  triangular solves with a diagonal block (row per thread),
// plus the permutation helpers of the solve (Sec. III-A.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "common.h"
#include "kernels.h"

namespace {

// Barrier that orders LDS only, so that global loads issued before it stay in
// flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// SWAP.  compose: one workgroup turns the interchange sequence
// ipiv[j0 .. j0+cnt) (rows >= j0) into a list of moves (dst row <- src row).
// The rows that can change are rows j0 .. j0+cnt-1 and the distinct pivot
// rows beyond them (taken in order of first appearance).  For each such row
// d, the row whose contents end up in d is found by applying the
// interchanges to d in reverse order (each thread follows its own rows; the
// pivot list is read from LDS by all threads in step); every row whose
// source differs is one move.  apply: each workgroup copies the moves for a
// strip of columns, staging the gathered values in LDS so that all reads of
// a column precede all of its writes.
// ---------------------------------------------------------------------------
constexpr int kMaxSwaps = 1024;

__global__ __launch_bounds__(256) void swap_compose_kernel(const int32_t *__restrict__ ipiv,
                                                           int64_t j0, int cnt, int64_t nrows,
                                                           int *__restrict__ moves) {
    __shared__ int s_piv[kMaxSwaps];
    __shared__ int s_wsum[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    // relative pivot rows; an entry outside [t, nrows - j0) (possible only in
    // a sequence left by an expired wait) is taken as no interchange, so the
    // moves never address a row outside the matrix
    for (int t = tid; t < cnt; t += 256) {
        const int64_t q = (int64_t)ipiv[j0 + t] - j0;
        s_piv[t] = (q >= t && q < nrows - j0) ? (int)q : t;
    }
    __syncthreads();
    // candidate t < cnt is row t; candidate cnt + u is the pivot row of
    // interchange u when it lies beyond the block and appears there first
    int base = 0;
    for (int t0 = 0; t0 < 2 * cnt; t0 += 256) {
        const int t = t0 + tid;
        int d = -1;
        if (t < cnt) {
            d = t;
        } else if (t < 2 * cnt) {
            const int u = t - cnt;
            const int q = s_piv[u];
            if (q >= cnt) {
                d = q;
                for (int v = 0; v < u; ++v)
                    if (s_piv[v] == q) {
                        d = -1;
                        break;
                    }
            }
        }
        int src = d;
        for (int u = cnt - 1; u >= 0; --u) {
            const int q = s_piv[u];
            src = (src == u) ? q : ((src == q) ? u : src);
        }
        const bool moved = (d >= 0) && (src != d);
        // compact in candidate order: moves = [count, dst..., src...]
        const unsigned long long mask = __ballot(moved);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) s_wsum[wv] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int k = 0; k < wv; ++k) off += s_wsum[k];
        if (moved) {
            moves[1 + off + before] = d;
            moves[1 + 2 * kMaxSwaps + off + before] = src;
        }
        const int total = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
        __syncthreads();
        base += total;
    }
    if (tid == 0) moves[0] = base;
}

constexpr int kSwapColsPerBlock = 32;
constexpr int kSwapBatch = 4;   // columns staged per round

template <typename T>
__global__ __launch_bounds__(256) void swap_apply_kernel(T *__restrict__ A, int64_t lda,
                                                         int64_t j0, const int *__restrict__ moves,
                                                         int64_t c_begin, int64_t ncols,
                                                         int64_t skip_begin, int64_t skip_len) {
    __shared__ int s_dst[2 * kMaxSwaps];
    __shared__ int s_src[2 * kMaxSwaps];
    __shared__ T s_val[kSwapBatch * 2 * kMaxSwaps / 2];   // 4 x 1024
    const int tid = threadIdx.x;
    const int nm = moves[0];
    for (int t = tid; t < nm; t += 256) {
        s_dst[t] = moves[1 + t];
        s_src[t] = moves[1 + 2 * kMaxSwaps + t];
    }
    __syncthreads();
    if (nm == 0) return;
    const int64_t q0 = (int64_t)blockIdx.x * kSwapColsPerBlock;
    const int64_t q1 = (q0 + kSwapColsPerBlock < ncols) ? q0 + kSwapColsPerBlock : ncols;
    const int per_round = (nm <= 1024) ? kSwapBatch : 2;   // s_val holds 4096 values
    const int64_t skip_rel = skip_begin - c_begin;
    for (int64_t qb = q0; qb < q1; qb += per_round) {
        const int nb = (int)((q1 - qb < per_round) ? q1 - qb : per_round);
        for (int t = tid; t < nb * nm; t += 256) {
            const int b = t / nm, mv = t - b * nm;
            const int64_t q = qb + b;
            const int64_t c = c_begin + ((q < skip_rel) ? q : q + skip_len);
            s_val[t] = MXLU_AT(A, j0 + s_src[mv], c, lda);
        }
        __syncthreads();
        for (int t = tid; t < nb * nm; t += 256) {
            const int b = t / nm, mv = t - b * nm;
            const int64_t q = qb + b;
            const int64_t c = c_begin + ((q < skip_rel) ? q : q + skip_len);
            MXLU_AT(A, j0 + s_dst[mv], c, lda) = s_val[t];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Deferred interchanges of the columns left of the panels.  No later step
// reads the L columns of a finished panel, so their row interchanges can wait
// until the factorization is done; then each element moves once.  Panel j's
// rows below it end up gathered through q_j = r_{j+1} o ... o r_{K-1}, the
// composition of the gather maps of the later steps' interchanges (r_s(i) is
// the row whose content step s moves to row i: the identity but for the
// moves of step s).  q is built from the last step backwards.
__global__ void perm_iota_kernel(int64_t n, int32_t *__restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) q[i] = (int32_t)i;
}

// r at the moved rows of one step: their sources (set) or themselves (reset)
__global__ void perm_moves_kernel(const int *__restrict__ moves, int64_t j0,
                                  int32_t *__restrict__ r, int reset) {
    const int nm = moves[0];
    for (int t = threadIdx.x; t < nm; t += 256) {
        const int d = moves[1 + t];
        r[j0 + d] = (int32_t)(j0 + (reset ? d : moves[1 + 2 * kMaxSwaps + t]));
    }
}

// q[i] <- r[q[i]] for rows [i0, n)
__global__ void perm_compose_kernel(int64_t i0, int64_t n, const int32_t *__restrict__ r,
                                    int32_t *__restrict__ q) {
    const int64_t i = i0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) q[i] = r[q[i]];
}

// T (rows x cols, leading dimension rows) <- A[q[r0 + i], c0 + c]
__global__ void gather_panel_rows_kernel(const double *__restrict__ A, int64_t lda, int64_t r0,
                                         int64_t rows, int64_t c0, const int32_t *__restrict__ q,
                                   double *__restrict__ T) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < rows) T[i + c * rows] = MXLU_AT(A, q[r0 + i], c0 + c, lda);
}

// A[r0 + i, c0 + c] <- T
__global__ void put_panel_rows_kernel(const double *__restrict__ T, int64_t rows, double *__restrict__ A,
                                int64_t lda, int64_t r0, int64_t c0) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < rows) MXLU_AT(A, r0 + i, c0 + c, lda) = T[i + c * rows];
}

// One right-hand side: y -= A x with A (M x K, K <= 256 per pass) streamed
// by 64-row x 4-group workgroups: thread (r, g) sums the terms of its row over
// the g-th quarter of the k range in ascending k; the four partial sums are
// combined in a fixed order, so the result does not depend on timing.  Four
// times the workgroups of a row-per-thread form, with each thread's loads
// independent of its arithmetic.
__global__ __launch_bounds__(256) void gemv_f64_sub_kernel(int64_t M, int64_t K,
                                                           const double *__restrict__ A,
                                                           int64_t lda,
                                                           const double *__restrict__ x,
                                                           double *__restrict__ y) {
    __shared__ double xs[256];
    __shared__ double part[4][64];
    const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + r;
    double acc = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += 256) {
        const int kc = (int)((K - k0 < 256) ? K - k0 : 256);
        __syncthreads();
        if (tid < kc) xs[tid] = x[k0 + tid];
        __syncthreads();
        const int q = (kc + 3) / 4, ka = g * q, kz = (ka + q < kc) ? ka + q : kc;
        if (i < M) {
#pragma unroll 8
            for (int k = ka; k < kz; ++k) acc = fma(MXLU_AT(A, i, k0 + k, lda), xs[k], acc);
        }
    }
    part[g][r] = acc;
    __syncthreads();
    if (g == 0 && i < M) y[i] = y[i] - ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
}

// ---------------------------------------------------------------------------
// DTRSM family, kb <= 256 rows: thread i owns row i of a strip of NC columns
// of B in registers.  Step k broadcasts the finished row k through LDS (one
// LDS barrier per k, double-buffered) and every row still to be solved takes
// one fused multiply-add with its factor entry, so each entry accumulates its
// terms in the same order as the textbook substitution.  The factor entries
// are prefetched 8 steps ahead.
// ---------------------------------------------------------------------------
template <int NC, bool LOWER, bool UNIT, bool TRANS>
__global__ __launch_bounds__(256) void trsm_kernel(int kb, int64_t ncols,
                                                   const double *__restrict__ T, int64_t ldt,
                                                   double *__restrict__ B, int64_t ldb) {
    __shared__ double xs[2][NC];
    const int i = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * NC;
    const int nc = (int)((ncols - c0 < NC) ? ncols - c0 : NC);
    double b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) b[c] = (i < kb && c < nc) ? MXLU_AT(B, i, c0 + c, ldb) : 0.0;

    // Effective factor F: column k of F is the k-th column used by the
    // substitution.  LOWER && !TRANS: L (forward).  !LOWER && !TRANS: U
    // (backward).  !LOWER && TRANS: U^T, lower (forward).  LOWER && TRANS: L^T,
    // upper (backward).
    constexpr bool FORWARD = (LOWER != TRANS);
    auto fentry = [&](int row, int k) -> double {
        // F[row][k]
        return TRANS ? MXLU_AT(T, k, row, ldt) : MXLU_AT(T, row, k, ldt);
    };
    auto needs = [&](int row, int k) -> bool { return FORWARD ? (row > k) : (row < k); };

    double lbuf[8], lnext[8];
    auto prefetch = [&](int s0, double *dst) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int s = s0 + q;
            const int k = FORWARD ? s : kb - 1 - s;
            dst[q] = (s < kb && i < kb && (needs(i, k) || (!UNIT && i == k))) ? fentry(i, k) : 0.0;
        }
    };
    prefetch(0, lbuf);
    for (int s0 = 0; s0 < kb; s0 += 8) {
        prefetch(s0 + 8, lnext);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int s = s0 + q;
            if (s >= kb) break;
            const int k = FORWARD ? s : kb - 1 - s;
            if (i == k) {
                if (!UNIT) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) b[c] = b[c] / lbuf[q];
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) xs[s & 1][c] = b[c];
            }
            lds_barrier();
            if (i < kb && needs(i, k)) {
                const double f = lbuf[q];
#pragma unroll
                for (int c = 0; c < NC; ++c) b[c] = fma(-f, xs[s & 1][c], b[c]);
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) lbuf[q] = lnext[q];
    }
    if (i < kb)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nc) MXLU_AT(B, i, c0 + c, ldb) = b[c];
}

// C(M x N) -= A(K x M)^T B(K x N), N <= 16: one wave per output row i,
// lanes stride over K (column i of A is contiguous).
template <int NMAX>
__global__ __launch_bounds__(256) void gemm_tn_skinny_kernel(int64_t M, int N, int64_t K,
                                                             const double *__restrict__ A,
                                                             int64_t lda,
                                                             const double *__restrict__ B,
                                                             int64_t ldb, double *__restrict__ C,
                                                             int64_t ldc) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= M) return;
    double acc[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) acc[c] = 0.0;
    for (int64_t k = lane; k < K; k += 64) {
        const double a = MXLU_AT(A, k, i, lda);
#pragma unroll
        for (int c = 0; c < NMAX; ++c)
            if (c < N) acc[c] = fma(a, MXLU_AT(B, k, c, ldb), acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
        double v = acc[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc[c] = v;
    }
    if (lane < N) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < NMAX; ++c)
            if (c == lane) v = acc[c];
        MXLU_AT(C, i, lane, ldc) = MXLU_AT(C, i, lane, ldc) - v;
    }
}

// ---------------------------------------------------------------------------
// Permutation of the solve: replay the n interchanges on an index array kept
// in LDS when it fits, else in global memory.
// ---------------------------------------------------------------------------
// perm: the gather map of all interchanges of ipiv applied in order (row i of
// P b is b[perm[i]]).  The interchanges are taken 256 at a time: those of a
// block move only its own rows and rows below it, so each thread follows one
// candidate row (a row of the block, or a pivot row below it where it first
// appears) back through the block's interchanges to the row its content comes
// from, and the block's moves are applied at once.  An entry outside
// [j, n) is taken as no interchange, as in swap_compose.
__global__ __launch_bounds__(256) void perm_from_ipiv_kernel(int64_t n,
                                                             const int32_t *__restrict__ ipiv,
                                                             int32_t *__restrict__ perm,
                                                             int in_lds) {
    extern __shared__ int sperm[];
    __shared__ __attribute__((aligned(16))) int s_piv[256];
    int *p = in_lds ? sperm : perm;
    const int tid = threadIdx.x;
    for (int64_t t = tid; t < n; t += 256) p[t] = (int)t;
    __syncthreads();
    for (int64_t j0 = 0; j0 < n; j0 += 256) {
        const int cnt = (int)((n - j0 < 256) ? n - j0 : 256);
        // entries past cnt are identity interchanges (no effect), so every
        // loop below runs over all 256 entries, four per broadcast LDS read
        {
            const int64_t q = tid < cnt ? (int64_t)ipiv[j0 + tid] - j0 : (int64_t)tid;
            s_piv[tid] = (q >= tid && q < n - j0) ? (int)q : tid;
        }
        __syncthreads();
        const int4 *piv4 = reinterpret_cast<const int4 *>(s_piv);
        int d0 = -1, d1 = -1;
        if (tid < cnt) {
            d0 = tid;
            const int q = s_piv[tid];
            if (q >= cnt) {   // a pivot row below the block, followed where it first appears
                bool first = true;
                for (int u4 = 0; u4 < (tid + 3) / 4; ++u4) {
                    const int4 w = piv4[u4];
                    const int u = 4 * u4;
                    first = first && !(u < tid && w.x == q) && !(u + 1 < tid && w.y == q) &&
                            !(u + 2 < tid && w.z == q) && !(u + 3 < tid && w.w == q);
                }
                if (first) d1 = q;
            }
        }
        // both candidate rows traced back through the block's interchanges,
        // last to first, side by side
        int src0 = d0 < 0 ? 0 : d0, src1 = d1 < 0 ? 0 : d1;
#pragma unroll 8
        for (int u4 = 63; u4 >= 0; --u4) {
            const int4 w = piv4[u4];
            const int u = 4 * u4;
            src0 = (src0 == u + 3) ? w.w : ((src0 == w.w) ? u + 3 : src0);
            src1 = (src1 == u + 3) ? w.w : ((src1 == w.w) ? u + 3 : src1);
            src0 = (src0 == u + 2) ? w.z : ((src0 == w.z) ? u + 2 : src0);
            src1 = (src1 == u + 2) ? w.z : ((src1 == w.z) ? u + 2 : src1);
            src0 = (src0 == u + 1) ? w.y : ((src0 == w.y) ? u + 1 : src0);
            src1 = (src1 == u + 1) ? w.y : ((src1 == w.y) ? u + 1 : src1);
            src0 = (src0 == u) ? w.x : ((src0 == w.x) ? u : src0);
            src1 = (src1 == u) ? w.x : ((src1 == w.x) ? u : src1);
        }
        int d[2] = {d0, d1}, v[2] = {0, 0};
        if (d0 >= 0) v[0] = p[j0 + src0];
        if (d1 >= 0) v[1] = p[j0 + src1];
        __syncthreads();   // every source read before any move is written
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (d[e] >= 0) p[j0 + d[e]] = v[e];
        __syncthreads();
    }
    if (in_lds)
        for (int64_t t = tid; t < n; t += 256) perm[t] = sperm[t];
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One right-hand side through a triangular diagonal block of order bb <= 256
// (one workgroup of five waves): the block is solved 64 rows at a time; wave
// 0 holds the 64 x 64 diagonal sub-block, one row per lane, in registers and
// solves it with each finished value broadcast by readlane; waves 1-4 (one
// thread per row) then apply the sub-block's values to the rows still to be
// solved, their operands (coalesced column loads) having been loaded before
// the sub-block was solved, so that they arrive meanwhile.  LOWER: unit
// lower, forward; else upper with its diagonal, backward.  y (bb values) is
// read once and written once.
constexpr int kTrsvF64Threads = 320;

template <bool LOWER>
__global__ __launch_bounds__(kTrsvF64Threads) void trsv_block_f64_kernel(
    int bb, const double *__restrict__ T, int64_t ldt, double *__restrict__ y) {
    __shared__ double ys[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int u = tid - 64;   // the applying thread's index (waves 1-4)
    if (tid < bb) ys[tid] = y[tid];
    const int nsb = (bb + 63) / 64;
    for (int k = 0; k < nsb; ++k) {
        const int c0 = 64 * (LOWER ? k : nsb - 1 - k);
        const int jn = (bb - c0 < 64) ? bb - c0 : 64;
        // rows still to solve: below the sub-block (LOWER) or above it
        const int r = LOWER ? c0 + 64 + u : u;
        const bool todo = wave > 0 && (LOWER ? (r < bb) : (r < c0));
        // t: wave 0's row of the diagonal sub-block, or an applying thread's
        // row in the sub-block's columns (both independent of the solution,
        // so loaded before waiting for it)
        const int rr = c0 + lane;
        const bool ok = rr < bb;
        const int lr = wave == 0 ? rr : r;
        const bool lok = wave == 0 ? ok : todo;
        double t[64];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            t[j] = (lok && j < jn) ? T[(size_t)lr + (size_t)(c0 + j) * ldt] : 0.0;
        __syncthreads();
        if (wave == 0) {
            const double *a = t;
            double x = ok ? ys[rr] : 0.0;
            if (LOWER) {
#pragma unroll
                for (int j = 0; j < 64; ++j) {
                    const double xj = readlane_f64(x, j);   // final
                    if (lane > j) x = fma(-a[j], xj, x);
                }
            } else {
#pragma unroll
                for (int j = 63; j >= 0; --j) {
                    if (lane == j && ok) x = x / a[j];
                    const double xj = readlane_f64(x, j);
                    if (lane < j) x = fma(-a[j], xj, x);
                }
            }
            if (ok) ys[rr] = x;
        }
        __syncthreads();
        if (todo) {
            double acc = ys[r];
#pragma unroll
            for (int j = 0; j < 64; ++j)
                if (j < jn) acc = fma(-t[j], ys[c0 + j], acc);
            ys[r] = acc;
        }
    }
    __syncthreads();
    if (tid < bb) y[tid] = ys[tid];
}

__global__ void gather_rows_kernel(int64_t n, int64_t nrhs, const int32_t *__restrict__ perm,
                                   const double *__restrict__ B, int64_t ldb,
                                   double *__restrict__ Y, int64_t ldy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t src = perm[i];
    for (int64_t c = 0; c < nrhs; ++c) MXLU_AT(Y, i, c, ldy) = MXLU_AT(B, src, c, ldb);
}

__global__ void scatter_rows_kernel(int64_t n, int64_t nrhs, const int32_t *__restrict__ perm,
                                    const double *__restrict__ Y, int64_t ldy,
                                    double *__restrict__ B, int64_t ldb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t dst = perm[i];
    for (int64_t c = 0; c < nrhs; ++c) MXLU_AT(B, dst, c, ldb) = MXLU_AT(Y, i, c, ldy);
}

}  // namespace

namespace mxlu {

static int max_dynamic_lds() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            v = 65536;
        cached = v;
    }
    return cached;
}

// Dynamic LDS left to the LDS form of the leaf (the static part holds the

int swap_compose(const int32_t *ipiv, int64_t j0, int cnt, int64_t nrows, int *moves,
                 hipStream_t s) {
    if (cnt <= 0) return 0;
    if (cnt > kMaxSwaps || !moves || nrows - j0 > INT_MAX) {
        set_error_msg("laswp: too many interchanges, rows or no move buffer");
        return MXLU_E_NOMEM;
    }
    hipLaunchKernelGGL(swap_compose_kernel, dim3(1), dim3(256), 0, s, ipiv, j0, cnt, nrows,
                       moves);
    MXLU_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int swap_apply(T *A, int64_t lda, int64_t j0, const int *moves, int64_t c_begin, int64_t ncols,
               int64_t skip_begin, int64_t skip_len, hipStream_t s) {
    if (ncols <= 0) return 0;
    const unsigned grid = (unsigned)((ncols + kSwapColsPerBlock - 1) / kSwapColsPerBlock);
    hipLaunchKernelGGL(swap_apply_kernel<T>, dim3(grid), dim3(256), 0, s, A, lda, j0, moves,
                       c_begin, ncols, skip_begin, skip_len);
    MXLU_LAUNCH_CHECK();
    return 0;
}
template int swap_apply<double>(double *, int64_t, int64_t, const int *, int64_t, int64_t,
                                int64_t, int64_t, hipStream_t);
template int swap_apply<float>(float *, int64_t, int64_t, const int *, int64_t, int64_t, int64_t,
                               int64_t, hipStream_t);
template int swap_apply<uint16_t>(uint16_t *, int64_t, int64_t, const int *, int64_t, int64_t,
                                  int64_t, int64_t, hipStream_t);

int laswp_f64(double *A, int64_t lda, int64_t nrows, const int32_t *ipiv, int64_t j0, int cnt,
              int64_t c_begin, int64_t ncols, int64_t skip_begin, int64_t skip_len,
              int *moves, hipStream_t s) {
    if (cnt <= 0 || ncols <= 0) return 0;
    MXLU_TRY(swap_compose(ipiv, j0, cnt, nrows, moves, s));
    return swap_apply<double>(A, lda, j0, moves, c_begin, ncols, skip_begin, skip_len, s);
}

int laswp_left_deferred_f64(double *A, int64_t lda, int64_t n, int64_t nb,
                            const int32_t *ipiv, int *moves, int32_t *q, int32_t *r, double *T,
                            hipStream_t s) {
    const int64_t K = (n + nb - 1) / nb;
    if (K < 2) return 0;
    const unsigned gn = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(perm_iota_kernel, dim3(gn), dim3(256), 0, s, n, q);
    MXLU_LAUNCH_CHECK();
    hipLaunchKernelGGL(perm_iota_kernel, dim3(gn), dim3(256), 0, s, n, r);
    MXLU_LAUNCH_CHECK();
    for (int64_t j = K - 2; j >= 0; --j) {
        const int64_t j1 = (j + 1) * nb, kb1 = std::min(nb, n - j1);
        // q <- r_{j+1} o q
        MXLU_TRY(swap_compose(ipiv, j1, (int)kb1, n, moves, s));
        hipLaunchKernelGGL(perm_moves_kernel, dim3(1), dim3(256), 0, s, moves, j1, r, 0);
        MXLU_LAUNCH_CHECK();
        const int64_t rows = n - j1;
        const unsigned gr = (unsigned)((rows + 255) / 256);
        hipLaunchKernelGGL(perm_compose_kernel, dim3(gr), dim3(256), 0, s, j1, n, r, q);
        MXLU_LAUNCH_CHECK();
        hipLaunchKernelGGL(perm_moves_kernel, dim3(1), dim3(256), 0, s, moves, j1, r, 1);
        MXLU_LAUNCH_CHECK();
        // panel j's columns, rows below it, gathered through q
        const int64_t c0 = j * nb, cols = nb;
        hipLaunchKernelGGL(gather_panel_rows_kernel, dim3(gr, (unsigned)cols), dim3(256), 0, s, A, lda,
                           j1, rows, c0, q, T);
        MXLU_LAUNCH_CHECK();
        hipLaunchKernelGGL(put_panel_rows_kernel, dim3(gr, (unsigned)cols), dim3(256), 0, s, T, rows, A,
                           lda, j1, c0);
        MXLU_LAUNCH_CHECK();
    }
    return 0;
}

int gemv_f64_sub(int64_t M, int64_t K, const double *A, int64_t lda, const double *x, double *y,
                 hipStream_t s) {
    if (M <= 0 || K <= 0) return 0;
    hipLaunchKernelGGL(gemv_f64_sub_kernel, dim3((unsigned)((M + 63) / 64)), dim3(256), 0, s, M, K,
                       A, lda, x, y);
    MXLU_LAUNCH_CHECK();
    return 0;
}

template <bool LOWER, bool UNIT, bool TRANS>
static int trsm_launch(int kb, int64_t ncols, const double *T, int64_t ldt, double *B,
                       int64_t ldb, hipStream_t s) {
    if (kb <= 0 || ncols <= 0) return 0;
    if (kb > 256) {
        set_error_msg("trsm: diagonal block larger than 256");
        return MXLU_E_NOMEM;
    }
    if (ncols <= 4) {
        hipLaunchKernelGGL((trsm_kernel<1, LOWER, UNIT, TRANS>), dim3((unsigned)ncols), dim3(256),
                           0, s, kb, ncols, T, ldt, B, ldb);
    } else {
        const unsigned grid = (unsigned)((ncols + 15) / 16);
        hipLaunchKernelGGL((trsm_kernel<16, LOWER, UNIT, TRANS>), dim3(grid), dim3(256), 0, s, kb,
                           ncols, T, ldt, B, ldb);
    }
    MXLU_LAUNCH_CHECK();
    return 0;
}

int trsm_llnu_f64(int kb, int64_t ncols, const double *L, int64_t ldl, double *B, int64_t ldb,
                  hipStream_t s) {
    return trsm_launch<true, true, false>(kb, ncols, L, ldl, B, ldb, s);
}
int trsm_lunn_f64(int kb, int64_t ncols, const double *U, int64_t ldu, double *B, int64_t ldb,
                  hipStream_t s) {
    return trsm_launch<false, false, false>(kb, ncols, U, ldu, B, ldb, s);
}
int trsv_block_f64(int bb, bool lower, const double *T, int64_t ldt, double *y, hipStream_t s) {
    if (bb <= 0) return 0;
    if (bb > 256) {
        set_error_msg("trsv_block_f64: block larger than 256");
        return MXLU_E_NOMEM;
    }
    if (lower)
        hipLaunchKernelGGL(trsv_block_f64_kernel<true>, dim3(1), dim3(kTrsvF64Threads), 0, s, bb,
                           T, ldt, y);
    else
        hipLaunchKernelGGL(trsv_block_f64_kernel<false>, dim3(1), dim3(kTrsvF64Threads), 0, s, bb,
                           T, ldt, y);
    MXLU_LAUNCH_CHECK();
    return 0;
}
int trsm_lutn_f64(int kb, int64_t ncols, const double *U, int64_t ldu, double *B, int64_t ldb,
                  hipStream_t s) {
    return trsm_launch<false, false, true>(kb, ncols, U, ldu, B, ldb, s);
}
int trsm_lltu_f64(int kb, int64_t ncols, const double *L, int64_t ldl, double *B, int64_t ldb,
                  hipStream_t s) {
    return trsm_launch<true, true, true>(kb, ncols, L, ldl, B, ldb, s);
}

int gemm_f64_sub_tn_skinny(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc,
                           hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (N > 16) {
        set_error_msg("gemm_tn_skinny: more than 16 columns");
        return MXLU_E_NOMEM;
    }
    const unsigned grid = (unsigned)((M + 3) / 4);
    if (N == 1)
        hipLaunchKernelGGL(gemm_tn_skinny_kernel<1>, dim3(grid), dim3(256), 0, s, M, (int)N, K, A,
                           lda, B, ldb, C, ldc);
    else
        hipLaunchKernelGGL(gemm_tn_skinny_kernel<16>, dim3(grid), dim3(256), 0, s, M, (int)N, K,
                           A, lda, B, ldb, C, ldc);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int perm_from_ipiv(int64_t n, const int32_t *ipiv, int32_t *perm, hipStream_t s) {
    if (n <= 0) return 0;
    const int budget = max_dynamic_lds() - 1024;
    const int in_lds = (int64_t)n * (int64_t)sizeof(int) <= budget;
    const size_t lds = in_lds ? (size_t)n * sizeof(int) : 0;
    static bool attr_set = false;
    if (!attr_set) {
        MXLU_HIP_TRY(hipFuncSetAttribute((const void *)perm_from_ipiv_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, budget));
        attr_set = true;
    }
    hipLaunchKernelGGL(perm_from_ipiv_kernel, dim3(1), dim3(256), lds, s, n, ipiv, perm, in_lds);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int gather_rows_f64(int64_t n, int64_t nrhs, const int32_t *perm, const double *B, int64_t ldb,
                    double *Y, int64_t ldy, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return 0;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       nrhs, perm, B, ldb, Y, ldy);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int scatter_rows_f64(int64_t n, int64_t nrhs, const int32_t *perm, const double *Y, int64_t ldy,
                     double *B, int64_t ldb, hipStream_t s) {
    if (n <= 0 || nrhs <= 0) return 0;
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       n, nrhs, perm, Y, ldy, B, ldb);
    MXLU_LAUNCH_CHECK();
    return 0;
}

}  // namespace mxlu
