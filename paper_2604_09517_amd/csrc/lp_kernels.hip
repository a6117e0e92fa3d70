// Kernels of the low-precision LU (Sec. III-A.2: factorization and trailing
// updates in reduced precision, no pivoting) other than the MFMA update.
//
// Storage F holds the matrix in bf16 or fp16 (raw 16-bit words).  Per panel
// step at column k0 (width kb, m = n - k0 rows):
//   * the m x kb panel is copied to an FP32 buffer P and factored there in
//     FP32 (inner blocks of kLpIb columns: diagonal block + row TRSM + column
//     TRSM in one kernel, then an FP32 update of the panel's remaining
//     columns).  Every element accumulates its terms in ascending k with one
//     fused multiply-add per term and the division last, i.e. exactly the
//     operation sequence of unblocked elimination of the panel in FP32;
//   * the panel is rounded back to F; the L21 part is also written
//     transposed (k contiguous), the operand layout of the MFMA update;
//   * U12 = L11^-1 A12 in FP32 with the unrounded L11 of P, rounded to F;
//   * FP8 variant: L21 and U12 are quantised per tile to e4m3fn with
//     power-of-two scales.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "asource.h"
#include "common.h"
#include "lp_common.h"
#include "lp_kernels.h"

namespace {

// Barrier that orders LDS only, so that global loads issued before it stay in
// flight across it (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

using namespace mxlu;

// ---------------------------------------------------------------- convert
template <int FMT>
__global__ void convert_kernel(int64_t rows, int64_t cols, const double *__restrict__ A,
                               int64_t lda, uint16_t *__restrict__ F, int64_t ldf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y)
        F[(size_t)i + (size_t)j * (size_t)ldf] = f64_to_lp<FMT>(MXLU_AT(A, i, j, lda));
}

// The same with four adjacent rows per thread (two 16-byte loads of A, one
// 8-byte store of F) when lda is even, A 16-byte aligned, ldf a multiple of
// four and F 8-byte aligned; each element is rounded exactly as above.
template <int FMT>
__global__ void convert4_kernel(int64_t rows, int64_t cols, const double *__restrict__ A,
                                int64_t lda, uint16_t *__restrict__ F, int64_t ldf) {
    const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        const double *a = &A[(size_t)i + (size_t)j * (size_t)lda];
        uint16_t *f = &F[(size_t)i + (size_t)j * (size_t)ldf];
        if (i + 4 <= rows) {
            const double2 a01 = *reinterpret_cast<const double2 *>(a);
            const double2 a23 = *reinterpret_cast<const double2 *>(a + 2);
            uint2 w;
            w.x = (uint32_t)f64_to_lp<FMT>(a01.x) | ((uint32_t)f64_to_lp<FMT>(a01.y) << 16);
            w.y = (uint32_t)f64_to_lp<FMT>(a23.x) | ((uint32_t)f64_to_lp<FMT>(a23.y) << 16);
            *reinterpret_cast<uint2 *>(f) = w;
        } else {
            for (int64_t r = 0; i + r < rows; ++r) f[r] = f64_to_lp<FMT>(a[r]);
        }
    }
}

// The same rounding from the seeded generator's values (the FP64 matrix is
// never stored): F[i, j] <- round(a_ij).
template <int FMT>
__global__ void convert_seeded_kernel(int64_t n, ASource src, uint16_t *__restrict__ F,
                                      int64_t ldf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        F[(size_t)i + (size_t)j * (size_t)ldf] = f64_to_lp<FMT>(src.at(i, j));
}

// FP32 storage: F = fp32(A), IEEE round to nearest even (the cast), from A in
// memory or regenerated from its seed.
__global__ void convert_f32_kernel(int64_t n, ASource src, float *__restrict__ F, int64_t ldf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        F[(size_t)i + (size_t)j * (size_t)ldf] = (float)src.at(i, j);
}

template <int FMT>
__global__ void lp_to_f32_kernel(int64_t rows, int64_t cols, const uint16_t *__restrict__ F,
                                 int64_t ldf, float *__restrict__ P, int64_t ldp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y)
        P[(size_t)i + (size_t)j * (size_t)ldp] = lp_to_f32<FMT>(F[(size_t)i + (size_t)j * (size_t)ldf]);
}

template <int FMT>
__global__ void f32_to_lp_kernel(int64_t rows, int64_t cols, const float *__restrict__ P,
                                 int64_t ldp, uint16_t *__restrict__ F, int64_t ldf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y)
        F[(size_t)i + (size_t)j * (size_t)ldf] = f32_to_lp<FMT>(P[(size_t)i + (size_t)j * (size_t)ldp]);
}

// The same two copies with four adjacent rows per thread (8-byte 16-bit and
// 16-byte FP32 accesses) when both leading dimensions are multiples of four
// and the pointers aligned; each element is converted as above.
template <int FMT>
__global__ void lp_to_f32_4_kernel(int64_t rows, int64_t cols, const uint16_t *__restrict__ F,
                                   int64_t ldf, float *__restrict__ P, int64_t ldp) {
    const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        const uint16_t *f = &F[(size_t)i + (size_t)j * (size_t)ldf];
        float *p = &P[(size_t)i + (size_t)j * (size_t)ldp];
        if (i + 4 <= rows) {
            const uint2 w = *reinterpret_cast<const uint2 *>(f);
            *reinterpret_cast<float4 *>(p) = make_float4(
                lp_to_f32<FMT>((uint16_t)(w.x & 0xffffu)), lp_to_f32<FMT>((uint16_t)(w.x >> 16)),
                lp_to_f32<FMT>((uint16_t)(w.y & 0xffffu)), lp_to_f32<FMT>((uint16_t)(w.y >> 16)));
        } else {
            for (int64_t r = 0; i + r < rows; ++r) p[r] = lp_to_f32<FMT>(f[r]);
        }
    }
}

template <int FMT>
__global__ void f32_to_lp_4_kernel(int64_t rows, int64_t cols, const float *__restrict__ P,
                                   int64_t ldp, uint16_t *__restrict__ F, int64_t ldf) {
    const int64_t i = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= rows) return;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        const float *p = &P[(size_t)i + (size_t)j * (size_t)ldp];
        uint16_t *f = &F[(size_t)i + (size_t)j * (size_t)ldf];
        if (i + 4 <= rows) {
            const float4 v = *reinterpret_cast<const float4 *>(p);
            uint2 w;
            w.x = (uint32_t)f32_to_lp<FMT>(v.x) | ((uint32_t)f32_to_lp<FMT>(v.y) << 16);
            w.y = (uint32_t)f32_to_lp<FMT>(v.z) | ((uint32_t)f32_to_lp<FMT>(v.w) << 16);
            *reinterpret_cast<uint2 *>(f) = w;
        } else {
            for (int64_t r = 0; i + r < rows; ++r) f[r] = f32_to_lp<FMT>(p[r]);
        }
    }
}

// ---------------------------------------------------------------- panel leaf
// Inner block [c, c+ib) of the FP32 panel P (m x kb, leading dimension ldp).
// In every workgroup, wave 0 factors the ib x ib diagonal block in its
// registers (no pivoting) and leaves it in LDS;
// workgroups [0, nrow) then finish rows c+ib.. of the block columns (row
// TRSM with U of the diagonal block), workgroups [nrow, nrow+ncol) finish
// rows c..c+ib of the panel columns right of the block (unit-lower TRSM).
// The factored diagonal block goes back to P once, from the last workgroup
// to have read it (counted in *count, zero on entry and left zero): a
// workgroup that wrote it earlier would change values that a workgroup
// scheduled later still has to read.
// FULL: ib == kLpIb, the loops carry no width predicates (every loop is
// unrolled at compile time, so the rows stay in registers).
template <bool FULL>
__global__ __launch_bounds__(256) void lp_leaf_nopiv_kernel(int m, int kb, int c, int ib_arg,
                                                            float *__restrict__ P, int64_t ldp,
                                                            int nrow, int *__restrict__ info,
                                                            int *__restrict__ count,
                                                            int64_t col_base) {
    __shared__ float D[kLpIb][kLpIb + 1];
    __shared__ int last;
    const int ib = FULL ? kLpIb : ib_arg;
    const int tid = threadIdx.x;
    if (tid < 64) {
        // wave 0 factors the diagonal block in registers: lane i holds row i;
        // at step j the pivot row's values come from lane j by readlane (the
        // lanes of one wave run in lockstep, so no barrier is needed), and
        // every element takes its terms in the order of the column loop
        float x[kLpIb];
#pragma unroll
        for (int k = 0; k < kLpIb; ++k)
            x[k] = (tid < ib && k < ib) ? P[(size_t)(c + tid) + (size_t)(c + k) * ldp] : 0.0f;
#pragma unroll
        for (int j = 0; j < kLpIb; ++j) {
            if (j < ib) {
                const float piv = __builtin_bit_cast(
                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x[j]), j));
                // an exactly zero pivot leaves its column unscaled (it is reported)
                if (tid > j && tid < ib && piv != 0.0f) x[j] = x[j] / piv;
#pragma unroll
                for (int col = j + 1; col < kLpIb; ++col) {
                    const float u = __builtin_bit_cast(
                        float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x[col]), j));
                    if (tid > j && tid < ib && col < ib) x[col] = fmaf(-x[j], u, x[col]);
                }
            }
        }
        if (tid < ib)
#pragma unroll
            for (int k = 0; k < kLpIb; ++k) D[tid][k] = x[k];
    }
    __syncthreads();
    // D is built from every value of the block this workgroup loaded, so its
    // reads have completed once the barrier is passed; atomics on one word
    // are ordered, so the workgroup that counts last writes after every read
    if (tid == 0) {
        last = atomicAdd(count, 1) == (int)gridDim.x - 1;
        if (last) atomicExch(count, 0);   // ready for the next leaf on this stream
    }
    __syncthreads();
    if (last) {
        for (int t = tid; t < ib * ib; t += 256) {
            const int i = t % ib, j = t / ib;
            P[(size_t)(c + i) + (size_t)(c + j) * ldp] = D[i][j];
        }
        if (tid == 0 && info) {
            for (int j = 0; j < ib; ++j)
                if (D[j][j] == 0.0f) {
                    atomicCAS(info, 0, (int)(col_base + c + j + 1));
                    break;
                }
        }
    }
    if ((int)blockIdx.x < nrow) {
        const int r = c + ib + blockIdx.x * 256 + tid;
        if (r >= m) return;
        float x[kLpIb];
#pragma unroll
        for (int k = 0; k < kLpIb; ++k)
            x[k] = (k < ib) ? P[(size_t)r + (size_t)(c + k) * ldp] : 0.0f;
#pragma unroll
        for (int k = 0; k < kLpIb; ++k) {
            if (k < ib) {
                const float dkk = D[k][k];
                if (dkk != 0.0f) x[k] = x[k] / dkk;
#pragma unroll
                for (int col = k + 1; col < kLpIb; ++col)
                    if (col < ib) x[col] = fmaf(-x[k], D[k][col], x[col]);
            }
        }
#pragma unroll
        for (int k = 0; k < kLpIb; ++k)
            if (k < ib) P[(size_t)r + (size_t)(c + k) * ldp] = x[k];
    } else {
        const int q = c + ib + ((int)blockIdx.x - nrow) * 256 + tid;
        if (q >= kb) return;
        float y[kLpIb];
#pragma unroll
        for (int k = 0; k < kLpIb; ++k)
            y[k] = (k < ib) ? P[(size_t)(c + k) + (size_t)q * ldp] : 0.0f;
#pragma unroll
        for (int k = 0; k < kLpIb; ++k) {
            if (k < ib) {
#pragma unroll
                for (int i = k + 1; i < kLpIb; ++i)
                    if (i < ib) y[i] = fmaf(-D[i][k], y[k], y[i]);
            }
        }
#pragma unroll
        for (int k = 0; k < kLpIb; ++k)
            if (k < ib) P[(size_t)(c + k) + (size_t)q * ldp] = y[k];
    }
}

// ---------------------------------------------------------------- FP32 GEMM
// C (M x N) -= A (M x K) B (K x N), FP32, one fused multiply-add per term in
// ascending k starting from C (the elimination order).  64 x 64 tiles,
// 256 threads, 4 x 4 outputs per thread, K staged in chunks of 16.
__global__ __launch_bounds__(256) void gemm_f32_sub_kernel(int64_t M, int64_t N, int64_t K,
                                                           const float *__restrict__ A,
                                                           int64_t lda,
                                                           const float *__restrict__ B,
                                                           int64_t ldb, float *__restrict__ C,
                                                           int64_t ldc, int tiles_m) {
    __shared__ float As[16][64 + 1];
    __shared__ float Bs[16][64 + 1];
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t row0 = (int64_t)tm * 64, col0 = (int64_t)tn * 64;
    const int tid = threadIdx.x;
    const int tr = tid & 15, tc = tid >> 4;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t r = row0 + tr + 16 * a, cc = col0 + tc + 16 * b;
            acc[a][b] = (r < M && cc < N) ? C[(size_t)r + (size_t)cc * ldc] : 0.0f;
        }
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        for (int t = tid; t < 16 * 64; t += 256) {
            const int i = t % 64, k = t / 64;
            const int64_t r = row0 + i, kk = k0 + k;
            As[k][i] = (r < M && kk < K) ? A[(size_t)r + (size_t)kk * lda] : 0.0f;
        }
        for (int t = tid; t < 16 * 64; t += 256) {
            const int k = t % 16, j = t / 16;
            const int64_t cc = col0 + j, kk = k0 + k;
            Bs[k][j] = (cc < N && kk < K) ? B[(size_t)kk + (size_t)cc * ldb] : 0.0f;
        }
        __syncthreads();
        const int kc = (int)((K - k0 < 16) ? K - k0 : 16);
        for (int k = 0; k < kc; ++k) {
            float av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[k][tr + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[k][tc + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(-av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t r = row0 + tr + 16 * a, cc = col0 + tc + 16 * b;
            if (r < M && cc < N) C[(size_t)r + (size_t)cc * ldc] = acc[a][b];
        }
}

// Large-tile form for the panel's big updates: 128 x 128 tiles, 256 threads,
// 8 x 8 outputs per thread (rows 4 ty + {0..3} and 64 + 4 ty + {0..3},
// columns 4 tx + {0..3} and 64 + 4 tx + {0..3}), K in chunks of 16 staged
// through two LDS buffers; the next chunk's global loads are in flight in
// registers while the current one is used.  The same order of terms as the
// small-tile form: one fused multiply-add per term in ascending k from C.
constexpr int kG32Tile = 128, kG32Kc = 16, kG32Ld = kG32Tile + 4;

__global__ __launch_bounds__(256) void gemm_f32_sub_big_kernel(int64_t M, int64_t N, int64_t K,
                                                               const float *__restrict__ A,
                                                               int64_t lda,
                                                               const float *__restrict__ B,
                                                               int64_t ldb, float *__restrict__ C,
                                                               int64_t ldc, int tiles_m) {
    __shared__ __attribute__((aligned(16))) float As[2][kG32Kc][kG32Ld];
    __shared__ __attribute__((aligned(16))) float Bs[2][kG32Kc][kG32Ld];
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t row0 = (int64_t)tm * kG32Tile, col0 = (int64_t)tn * kG32Tile;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    // global load roles: A rows (tid % 128), k = tid / 128 + 2 q; B k = tid % 16,
    // columns tid / 16 + 16 q (q < 8)
    const int ar = tid & 127, ak = tid >> 7;
    const int bk = tid & 15, bc = tid >> 4;
    float ra[8], rb[8];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t r = row0 + ar, kk = k0 + ak + 2 * q;
            ra[q] = (r < M && kk < K) ? A[(size_t)r + (size_t)kk * lda] : 0.0f;
            const int64_t cc = col0 + bc + 16 * q, kb = k0 + bk;
            rb[q] = (cc < N && kb < K) ? B[(size_t)kb + (size_t)cc * ldb] : 0.0f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            As[buf][ak + 2 * q][ar] = ra[q];
            Bs[buf][bk][bc + 16 * q] = rb[q];
        }
    };
    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t r = row0 + (i < 4 ? 4 * ty + i : 64 + 4 * ty + i - 4);
            const int64_t cc = col0 + (j < 4 ? 4 * tx + j : 64 + 4 * tx + j - 4);
            acc[i][j] = (r < M && cc < N) ? C[(size_t)r + (size_t)cc * ldc] : 0.0f;
        }
    const int nk = (int)((K + kG32Kc - 1) / kG32Kc);
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((int64_t)(kt + 1) * kG32Kc);
        const int kc = (int)((K - (int64_t)kt * kG32Kc < kG32Kc) ? K - (int64_t)kt * kG32Kc : kG32Kc);
        for (int k = 0; k < kc; ++k) {
            const float4 a0 = *reinterpret_cast<const float4 *>(&As[buf][k][4 * ty]);
            const float4 a1 = *reinterpret_cast<const float4 *>(&As[buf][k][64 + 4 * ty]);
            const float4 b0 = *reinterpret_cast<const float4 *>(&Bs[buf][k][4 * tx]);
            const float4 b1 = *reinterpret_cast<const float4 *>(&Bs[buf][k][64 + 4 * tx]);
            const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(-av[i], bv[j], acc[i][j]);
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t r = row0 + (i < 4 ? 4 * ty + i : 64 + 4 * ty + i - 4);
            const int64_t cc = col0 + (j < 4 ? 4 * tx + j : 64 + 4 * tx + j - 4);
            if (r < M && cc < N) C[(size_t)r + (size_t)cc * ldc] = acc[i][j];
        }
}

// Matrix-core form: 128 x 128 tiles, 256 threads, each wave a 64 x 64
// quarter as 4 x 4 blocks of v_mfma_f32_16x16x4f32, K staged through LDS in
// chunks of 16 like the large-tile form.  The instruction computes each
// output as four fused multiply-adds in ascending k (measured bit for bit
// against fmaf on millions of random operands), and the blocks walk k in
// ascending groups of four from C with A negated, so every element takes the
// same terms in the same order as the other forms.  K % 4 == 0: no padded
// term ever enters a sum.
// Lane l of a block supplies A[row l % 16][k l / 16] and B[k l / 16][col
// l % 16] and holds rows 4 (l / 16) + r of column l % 16 of the result.
constexpr int kM32Ld = kG32Tile + 16;   // A and B rows of four k map to disjoint banks

typedef float v4f32 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gemm_f32_mfma_kernel(int64_t M, int64_t N, int64_t K,
                                                            const float *__restrict__ A,
                                                            int64_t lda,
                                                            const float *__restrict__ B,
                                                            int64_t ldb, float *__restrict__ C,
                                                            int64_t ldc, int tiles_m) {
    __shared__ __attribute__((aligned(16))) float As[2][kG32Kc][kM32Ld];
    __shared__ __attribute__((aligned(16))) float Bs[2][kG32Kc][kM32Ld];
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t row0 = (int64_t)tm * kG32Tile, col0 = (int64_t)tn * kG32Tile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;
    const int li = lane & 15, lg = lane >> 4;
    // global load roles as in the large-tile form
    const int ar = tid & 127, ak = tid >> 7;
    const int bk = tid & 15, bc = tid >> 4;
    float ra[8], rb[8];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t r = row0 + ar, kk = k0 + ak + 2 * q;
            ra[q] = (r < M && kk < K) ? A[(size_t)r + (size_t)kk * lda] : 0.0f;
            const int64_t cc = col0 + bc + 16 * q, kb = k0 + bk;
            rb[q] = (cc < N && kb < K) ? B[(size_t)kb + (size_t)cc * ldb] : 0.0f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            As[buf][ak + 2 * q][ar] = ra[q];
            Bs[buf][bk][bc + 16 * q] = rb[q];
        }
    };
    v4f32 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wr + 16 * bi + 4 * lg + r;
                const int64_t col = col0 + wc + 16 * bj + li;
                acc[bi][bj][r] = (row < M && col < N) ? C[(size_t)row + (size_t)col * ldc] : 0.0f;
            }
    const int nk = (int)((K + kG32Kc - 1) / kG32Kc);
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((int64_t)(kt + 1) * kG32Kc);
        const int64_t left = K - (int64_t)kt * kG32Kc;
        const int groups = left < kG32Kc ? (int)(left / 4) : kG32Kc / 4;
        for (int g = 0; g < groups; ++g) {
            const int k = 4 * g + lg;
            float a[4], b[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) a[bi] = -As[buf][k][wr + 16 * bi + li];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) b[bj] = Bs[buf][k][wc + 16 * bj + li];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + wr + 16 * bi + 4 * lg + r;
                const int64_t col = col0 + wc + 16 * bj + li;
                if (row < M && col < N) C[(size_t)row + (size_t)col * ldc] = acc[bi][bj][r];
            }
}

// ---------------------------------------------------------------- FP32 TRSM
// B (kb x ncols) <- L^-1 B, L unit lower kb x kb (kb <= 256), thread per row,
// NC columns per workgroup, one LDS barrier per step; each thread reads its
// row of L 32 columns at a time into registers, the next 32 in flight.  More
// columns per workgroup spread each barrier over more multiply-adds.
template <int NC>
__global__ __launch_bounds__(256) void trsm_f32_llnu_kernel(int kb, int64_t ncols,
                                                            const float *__restrict__ L,
                                                            int64_t ldl, float *__restrict__ B,
                                                            int64_t ldb) {
    __shared__ float xs[2][NC];
    const int i = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * NC;
    const int nc = (int)((ncols - c0 < NC) ? ncols - c0 : NC);
    float b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        b[c] = (i < kb && c < nc) ? B[(size_t)i + (size_t)(c0 + c) * ldb] : 0.0f;
    // the thread's row of L in chunks of 32 columns, the next chunk in flight
    // while the current one is used
    float lc[32], ln[32];
    auto load_chunk = [&](int k0, float (&l)[32]) {
#pragma unroll
        for (int kk = 0; kk < 32; ++kk) {
            const int k = k0 + kk;
            l[kk] = (i < kb && k < kb && i > k) ? L[(size_t)i + (size_t)k * ldl] : 0.0f;
        }
    };
    load_chunk(0, lc);
    for (int k0 = 0; k0 < kb; k0 += 32) {
        if (k0 + 32 < kb) load_chunk(k0 + 32, ln);
#pragma unroll
        for (int kk = 0; kk < 32; ++kk) {
            const int k = k0 + kk;
            if (k < kb) {
                if (i == k)
#pragma unroll
                    for (int c = 0; c < NC; ++c) xs[k & 1][c] = b[c];
                lds_barrier();
                if (i > k && i < kb)
#pragma unroll
                    for (int c = 0; c < NC; ++c) b[c] = fmaf(-lc[kk], xs[k & 1][c], b[c]);
            }
        }
#pragma unroll
        for (int kk = 0; kk < 32; ++kk) lc[kk] = ln[kk];
    }
    if (i < kb)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nc) B[(size_t)i + (size_t)(c0 + c) * ldb] = b[c];
}

// ---------------------------------------------------------------- store
// F[i, c] <- round(P[i, c]) for the m x kb panel; for rows i >= kb also the
// chunk-packed copy of L21 (line i - kb, value c, Mp lines) when LT is given.
// 64 x 64 tiles through LDS so that both writes are coalesced.
template <int FMT>
__global__ __launch_bounds__(256) void panel_store_kernel(int64_t m, int kb,
                                                          const float *__restrict__ P,
                                                          int64_t ldp, uint16_t *__restrict__ F,
                                                          int64_t ldf, uint16_t *__restrict__ LT,
                                                          int64_t Mp, int tiles_m) {
    __shared__ uint16_t T[64][64 + 2];
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int64_t r0 = (int64_t)tm * 64;
    const int c0 = tn * 64;
    const int tid = threadIdx.x;
    for (int t = tid; t < 64 * 64; t += 256) {
        const int i = t % 64, j = t / 64;
        const int64_t r = r0 + i;
        const int c = c0 + j;
        uint16_t h = 0;
        if (r < m && c < kb) {
            h = f32_to_lp<FMT>(P[(size_t)r + (size_t)c * ldp]);
            F[(size_t)r + (size_t)c * ldf] = h;
        }
        T[i][j] = h;
    }
    if (!LT) return;
    __syncthreads();
    for (int t = tid; t < 64 * 64; t += 256) {
        const int j = t % 64, i = t / 64;
        const int64_t r = r0 + i;
        const int c = c0 + j;
        if (r >= kb && r < m && c < kb)
            LT[((size_t)(c / kLpKc) * Mp + (size_t)(r - kb)) * kLpKc + (c % kLpKc)] = T[i][j];
    }
}

// U12 (kb x nt, column-major in F) -> chunk-packed Up: one thread per 8
// values (16 bytes) of a column.
__global__ __launch_bounds__(256) void pack_u12_kernel(int64_t nt, int kb,
                                                       const uint16_t *__restrict__ U12,
                                                       int64_t ldf, uint16_t *__restrict__ Up,
                                                       int64_t Np) {
    const int per = kb / 8;
    const int64_t total = nt * per;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t j = t / per;
        const int k = (int)(t - j * per) * 8;
        const uint4 v = *reinterpret_cast<const uint4 *>(U12 + (size_t)k + (size_t)j * ldf);
        *reinterpret_cast<uint4 *>(Up + ((size_t)(k / kLpKc) * Np + (size_t)j) * kLpKc +
                                   (k % kLpKc)) = v;
    }
}

// ---------------------------------------------------------------- FP8
// L21 (rows [0, mt) of the stored panel below the diagonal block, kb columns)
// -> LTq (kb x mt bytes, k contiguous) with one power-of-two scale per tile of
// `tile` rows.  One workgroup per row tile: amax pass, then quantise through
// LDS in chunks of 64 columns.
template <int FMT>
__global__ __launch_bounds__(256) void quant_l21_kernel(int64_t mt, int kb, int tile,
                                                        const uint16_t *__restrict__ L21,
                                                        int64_t ldf, uint8_t *__restrict__ LTq,
                                                        int64_t Mp, float *__restrict__ sL) {
    __shared__ float red[256];
    __shared__ __attribute__((aligned(16))) uint8_t T[64][256 + 8];
    const int64_t r0 = (int64_t)blockIdx.x * tile;
    const int rows = (int)((mt - r0 < tile) ? mt - r0 : tile);
    const int tid = threadIdx.x;
    // 16-byte form: rows in groups of 8 (one 16-byte load each), all 256
    // threads busy (groups x columns in parallel), four bytes per store of
    // the packed copy; the general form otherwise.  Both round every element
    // the same way, and the maximum does not depend on the order.
    const bool wide = rows % 8 == 0 && ldf % 8 == 0 &&
                      ((uintptr_t)(L21 + r0) & 15) == 0;
    const int rows8 = rows / 8;
    const int cpar = wide ? 256 / rows8 : 0;
    const int g8 = wide ? tid % rows8 : 0, cl = wide ? tid / rows8 : 0;
    float amax = 0.0f;
    if (wide) {
        if (cl < cpar)
            for (int c = cl; c < kb; c += cpar) {
                const uint4 v = *reinterpret_cast<const uint4 *>(
                    L21 + (size_t)(r0 + 8 * g8) + (size_t)c * ldf);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    amax = fmaxf(amax, fabsf(lp_to_f32<FMT>((uint16_t)(w[q] & 0xffffu))));
                    amax = fmaxf(amax, fabsf(lp_to_f32<FMT>((uint16_t)(w[q] >> 16))));
                }
            }
    } else {
        for (int c = 0; c < kb; ++c)
            for (int i = tid; i < rows; i += 256)
                amax = fmaxf(amax, fabsf(lp_to_f32<FMT>(L21[(size_t)(r0 + i) + (size_t)c * ldf])));
    }
    red[tid] = amax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    const float sc = fp8_tile_scale(red[0]);
    if (tid == 0) sL[blockIdx.x] = sc;
    const float inv = 1.0f / sc;   // exact: power of two
    for (int c0 = 0; c0 < kb; c0 += 64) {
        const int cw = (kb - c0 < 64) ? kb - c0 : 64;
        __syncthreads();
        if (wide) {
            for (int j = cl; j < cw; j += cpar) {
                if (cl >= cpar) break;
                const uint4 v = *reinterpret_cast<const uint4 *>(
                    L21 + (size_t)(r0 + 8 * g8) + (size_t)(c0 + j) * ldf);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
                uint32_t lo = 0, hi = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t b0 = f32_to_e4m3(lp_to_f32<FMT>((uint16_t)(w[q] & 0xffffu)) * inv);
                    const uint32_t b1 = f32_to_e4m3(lp_to_f32<FMT>((uint16_t)(w[q] >> 16)) * inv);
                    const uint32_t pair = b0 | (b1 << 8);
                    if (q < 2) lo |= pair << (16 * q);
                    else hi |= pair << (16 * (q - 2));
                }
                *reinterpret_cast<uint2 *>(&T[j][8 * g8]) = make_uint2(lo, hi);
            }
        } else {
            for (int t = tid; t < cw * rows; t += 256) {
                const int i = t % rows, j = t / rows;
                T[j][i] = f32_to_e4m3(lp_to_f32<FMT>(L21[(size_t)(r0 + i) + (size_t)(c0 + j) * ldf]) * inv);
            }
        }
        __syncthreads();
        if (wide && cw % 4 == 0) {
            const int cw4 = cw / 4;
            for (int t = tid; t < cw4 * rows; t += 256) {
                const int jq = t % cw4, i = t / cw4;
                const int k = c0 + 4 * jq;
                const uint32_t w = (uint32_t)T[4 * jq][i] | ((uint32_t)T[4 * jq + 1][i] << 8) |
                                   ((uint32_t)T[4 * jq + 2][i] << 16) |
                                   ((uint32_t)T[4 * jq + 3][i] << 24);
                *reinterpret_cast<uint32_t *>(
                    &LTq[((size_t)(k / kLp8Kc) * Mp + (size_t)(r0 + i)) * kLp8Kc + (k % kLp8Kc)]) = w;
            }
        } else {
            for (int t = tid; t < cw * rows; t += 256) {
                const int j = t % cw, i = t / cw;
                const int k = c0 + j;
                LTq[((size_t)(k / kLp8Kc) * Mp + (size_t)(r0 + i)) * kLp8Kc + (k % kLp8Kc)] = T[j][i];
            }
        }
    }
}

// U12 (kb x nt, stored) -> Uq (kb x nt bytes, leading dimension kb), one
// scale per tile of `tile` columns.
template <int FMT>
__global__ __launch_bounds__(256) void quant_u12_kernel(int64_t nt, int kb, int tile,
                                                        const uint16_t *__restrict__ U12,
                                                        int64_t ldf, uint8_t *__restrict__ Uq,
                                                        int64_t Np, float *__restrict__ sU) {
    __shared__ float red[256];
    const int64_t q0 = (int64_t)blockIdx.x * tile;
    const int cols = (int)((nt - q0 < tile) ? nt - q0 : tile);
    const int tid = threadIdx.x;
    // 16-byte form (eight consecutive k per load, eight bytes per store) when
    // the columns are 16-byte aligned; each element is quantised as in the
    // general form, and the maximum does not depend on the order
    const bool wide = kb % 8 == 0 && ldf % 8 == 0 && ((uintptr_t)U12 & 15) == 0;
    const int kb8 = kb / 8;
    float amax = 0.0f;
    if (wide) {
        for (int t = tid; t < cols * kb8; t += 256) {
            const int j = t / kb8, k = 8 * (t % kb8);
            const uint4 v =
                *reinterpret_cast<const uint4 *>(U12 + (size_t)k + (size_t)(q0 + j) * ldf);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                amax = fmaxf(amax, fabsf(lp_to_f32<FMT>((uint16_t)(w[q] & 0xffffu))));
                amax = fmaxf(amax, fabsf(lp_to_f32<FMT>((uint16_t)(w[q] >> 16))));
            }
        }
    } else {
        for (int j = 0; j < cols; ++j)
            for (int k = tid; k < kb; k += 256)
                amax = fmaxf(amax, fabsf(lp_to_f32<FMT>(U12[(size_t)k + (size_t)(q0 + j) * ldf])));
    }
    red[tid] = amax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    const float sc = fp8_tile_scale(red[0]);
    if (tid == 0) sU[blockIdx.x] = sc;
    const float inv = 1.0f / sc;
    if (wide) {
        for (int t = tid; t < cols * kb8; t += 256) {
            const int j = t / kb8, k = 8 * (t % kb8);
            const uint4 v =
                *reinterpret_cast<const uint4 *>(U12 + (size_t)k + (size_t)(q0 + j) * ldf);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t b0 = f32_to_e4m3(lp_to_f32<FMT>((uint16_t)(w[q] & 0xffffu)) * inv);
                const uint32_t b1 = f32_to_e4m3(lp_to_f32<FMT>((uint16_t)(w[q] >> 16)) * inv);
                const uint32_t pair = b0 | (b1 << 8);
                if (q < 2) lo |= pair << (16 * q);
                else hi |= pair << (16 * (q - 2));
            }
            *reinterpret_cast<uint2 *>(
                &Uq[((size_t)(k / kLp8Kc) * Np + (size_t)(q0 + j)) * kLp8Kc + (k % kLp8Kc)]) =
                make_uint2(lo, hi);
        }
    } else {
        for (int j = 0; j < cols; ++j)
            for (int k = tid; k < kb; k += 256)
                Uq[((size_t)(k / kLp8Kc) * Np + (size_t)(q0 + j)) * kLp8Kc + (k % kLp8Kc)] =
                    f32_to_e4m3(lp_to_f32<FMT>(U12[(size_t)k + (size_t)(q0 + j) * ldf]) * inv);
    }
}

// MX form: L21 row i, block b of 32 consecutive k -> 32 e4m3 bytes at their
// place in the chunk-packed layout and the E8M0 byte sLx[b Mp + i] (scale
// 2^(byte - 127)).  One thread per row, coalesced across rows per column.
template <int FMT>
__global__ __launch_bounds__(256) void quant_l21_mx_kernel(int64_t mt, int kb,
                                                           const uint16_t *__restrict__ L21,
                                                           int64_t ldf, uint8_t *__restrict__ LTq,
                                                           int64_t Mp, uint8_t *__restrict__ sLx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= mt) return;
    for (int b = 0; b < kb / 32; ++b) {
        float v[32];
        float amax = 0.0f;
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            v[k] = lp_to_f32<FMT>(L21[(size_t)i + (size_t)(32 * b + k) * ldf]);
            amax = fmaxf(amax, fabsf(v[k]));
        }
        const int e = mx_block_exp(amax);
        const float inv = ldexpf(1.0f, -e);   // exact: a power of two
        uint32_t w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            w[q] = (uint32_t)f32_to_e4m3(v[4 * q] * inv) |
                   ((uint32_t)f32_to_e4m3(v[4 * q + 1] * inv) << 8) |
                   ((uint32_t)f32_to_e4m3(v[4 * q + 2] * inv) << 16) |
                   ((uint32_t)f32_to_e4m3(v[4 * q + 3] * inv) << 24);
        const int k0 = 32 * b;
        uint4 *dst = reinterpret_cast<uint4 *>(
            LTq + ((size_t)(k0 / kLp8Kc) * Mp + (size_t)i) * kLp8Kc + (k0 % kLp8Kc));
        dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
        dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
        sLx[(size_t)b * Mp + i] = (uint8_t)(e + 127);
    }
}

// MX form: U12 column j, block b of 32 consecutive k (contiguous in the
// column) -> 32 e4m3 bytes and the E8M0 byte sUx[b Np + j].
template <int FMT>
__global__ __launch_bounds__(256) void quant_u12_mx_kernel(int64_t nt, int kb,
                                                           const uint16_t *__restrict__ U12,
                                                           int64_t ldf, uint8_t *__restrict__ Uq,
                                                           int64_t Np, uint8_t *__restrict__ sUx) {
    const int nb = kb / 32;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nt * nb) return;
    const int64_t j = t % nt;
    const int b = (int)(t / nt);
    const uint16_t *src = U12 + (size_t)(32 * b) + (size_t)j * ldf;
    float v[32];
    float amax = 0.0f;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        v[k] = lp_to_f32<FMT>(src[k]);
        amax = fmaxf(amax, fabsf(v[k]));
    }
    const int e = mx_block_exp(amax);
    const float inv = ldexpf(1.0f, -e);
    uint32_t w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        w[q] = (uint32_t)f32_to_e4m3(v[4 * q] * inv) | ((uint32_t)f32_to_e4m3(v[4 * q + 1] * inv) << 8) |
               ((uint32_t)f32_to_e4m3(v[4 * q + 2] * inv) << 16) |
               ((uint32_t)f32_to_e4m3(v[4 * q + 3] * inv) << 24);
    const int k0 = 32 * b;
    uint4 *dst = reinterpret_cast<uint4 *>(
        Uq + ((size_t)(k0 / kLp8Kc) * Np + (size_t)j) * kLp8Kc + (k0 % kLp8Kc));
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    sUx[(size_t)b * Np + j] = (uint8_t)(e + 127);
}

dim3 grid2(int64_t rows, int64_t cols) {
    return dim3((unsigned)((rows + 255) / 256), (unsigned)(cols < 4096 ? (cols > 0 ? cols : 1) : 4096));
}

}  // namespace

namespace mxlu {

int lp_convert(int fmt, int64_t rows, int64_t cols, const double *A, int64_t lda, uint16_t *F,
               int64_t ldf, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    if (lda % 2 == 0 && (uintptr_t)A % 16 == 0 && ldf % 4 == 0 && (uintptr_t)F % 8 == 0) {
        const dim3 g((unsigned)((rows + 1023) / 1024), grid2(rows, cols).y);
        if (fmt == kFmtBf16)
            hipLaunchKernelGGL(convert4_kernel<kFmtBf16>, g, dim3(256), 0, s, rows, cols, A, lda, F,
                               ldf);
        else
            hipLaunchKernelGGL(convert4_kernel<kFmtFp16>, g, dim3(256), 0, s, rows, cols, A, lda, F,
                               ldf);
    } else if (fmt == kFmtBf16) {
        hipLaunchKernelGGL(convert_kernel<kFmtBf16>, grid2(rows, cols), dim3(256), 0, s, rows, cols,
                           A, lda, F, ldf);
    } else {
        hipLaunchKernelGGL(convert_kernel<kFmtFp16>, grid2(rows, cols), dim3(256), 0, s, rows, cols,
                           A, lda, F, ldf);
    }
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_convert_src(int fmt, int64_t n, const ASource &src, uint16_t *F, int64_t ldf,
                   hipStream_t s) {
    if (!src.seeded()) return lp_convert(fmt, n, n, src.A, src.lda, F, ldf, s);
    if (n <= 0) return 0;
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(convert_seeded_kernel<kFmtBf16>, grid2(n, n), dim3(256), 0, s, n, src, F,
                           ldf);
    else
        hipLaunchKernelGGL(convert_seeded_kernel<kFmtFp16>, grid2(n, n), dim3(256), 0, s, n, src, F,
                           ldf);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_convert_src_f32(int64_t n, const ASource &src, float *F, int64_t ldf, hipStream_t s) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(convert_f32_kernel, grid2(n, n), dim3(256), 0, s, n, src, F, ldf);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_load_f32(int fmt, int64_t rows, int64_t cols, const uint16_t *F, int64_t ldf, float *P,
                int64_t ldp, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    if (ldf % 4 == 0 && ldp % 4 == 0 && (uintptr_t)F % 8 == 0 && (uintptr_t)P % 16 == 0) {
        const dim3 g((unsigned)((rows + 1023) / 1024), grid2(rows, cols).y);
        if (fmt == kFmtBf16)
            hipLaunchKernelGGL(lp_to_f32_4_kernel<kFmtBf16>, g, dim3(256), 0, s, rows, cols, F, ldf,
                               P, ldp);
        else
            hipLaunchKernelGGL(lp_to_f32_4_kernel<kFmtFp16>, g, dim3(256), 0, s, rows, cols, F, ldf,
                               P, ldp);
    } else if (fmt == kFmtBf16) {
        hipLaunchKernelGGL(lp_to_f32_kernel<kFmtBf16>, grid2(rows, cols), dim3(256), 0, s, rows,
                           cols, F, ldf, P, ldp);
    } else {
        hipLaunchKernelGGL(lp_to_f32_kernel<kFmtFp16>, grid2(rows, cols), dim3(256), 0, s, rows,
                           cols, F, ldf, P, ldp);
    }
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_store_f32(int fmt, int64_t rows, int64_t cols, const float *P, int64_t ldp, uint16_t *F,
                 int64_t ldf, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    if (ldf % 4 == 0 && ldp % 4 == 0 && (uintptr_t)F % 8 == 0 && (uintptr_t)P % 16 == 0) {
        const dim3 g((unsigned)((rows + 1023) / 1024), grid2(rows, cols).y);
        if (fmt == kFmtBf16)
            hipLaunchKernelGGL(f32_to_lp_4_kernel<kFmtBf16>, g, dim3(256), 0, s, rows, cols, P, ldp,
                               F, ldf);
        else
            hipLaunchKernelGGL(f32_to_lp_4_kernel<kFmtFp16>, g, dim3(256), 0, s, rows, cols, P, ldp,
                               F, ldf);
    } else if (fmt == kFmtBf16) {
        hipLaunchKernelGGL(f32_to_lp_kernel<kFmtBf16>, grid2(rows, cols), dim3(256), 0, s, rows,
                           cols, P, ldp, F, ldf);
    } else {
        hipLaunchKernelGGL(f32_to_lp_kernel<kFmtFp16>, grid2(rows, cols), dim3(256), 0, s, rows,
                           cols, P, ldp, F, ldf);
    }
    MXLU_LAUNCH_CHECK();
    return 0;
}

int gemm_f32_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                 int64_t ldb, float *C, int64_t ldc, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    {   // large-tile forms when they still give every CU a few tiles
        const int64_t tm = (M + kG32Tile - 1) / kG32Tile, tn = (N + kG32Tile - 1) / kG32Tile;
        if (K >= 32 && M >= 96 && N >= 96 && tm * tn >= 512 && tm * tn <= 0x7fffffff) {
            if (K % 4 == 0)
                hipLaunchKernelGGL(gemm_f32_mfma_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0,
                                   s, M, N, K, A, lda, B, ldb, C, ldc, (int)tm);
            else
                hipLaunchKernelGGL(gemm_f32_sub_big_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0,
                                   s, M, N, K, A, lda, B, ldb, C, ldc, (int)tm);
            MXLU_LAUNCH_CHECK();
            return 0;
        }
    }
    const int64_t tm = (M + 63) / 64, tn = (N + 63) / 64;
    if (tm * tn > 0x7fffffff) {
        set_error_msg("gemm_f32_sub: grid too large");
        return MXLU_E_NOMEM;
    }
    hipLaunchKernelGGL(gemm_f32_sub_kernel, dim3((unsigned)(tm * tn)), dim3(256), 0, s, M, N, K,
                       A, lda, B, ldb, C, ldc, (int)tm);
    MXLU_LAUNCH_CHECK();
    return 0;
}

// Columns [c0, c0 + w) of the panel (rows c0 .. m-1 still to be finished),
// factored recursively: left half, its U12 (unit-lower TRSM), the update of
// the right half (one GEMM with K = the left width), right half; leaves of
// kLpIb columns.  Every element still takes its terms in ascending k, one
// fused multiply-add each, so the result equals the column-by-column order.
static int panel_nopiv_rec(int64_t m, int64_t c0, int64_t w, float *P, int64_t ldp, int *info,
                           int *count, int64_t col_base, hipStream_t s) {
    if (w <= kLpIb) {
        const int64_t rows_below = m - c0 - w;
        const int nrow = (int)((rows_below + 255) / 256);
        const dim3 grid((unsigned)(nrow > 0 ? nrow : 1));
        if (w == kLpIb)
            hipLaunchKernelGGL(lp_leaf_nopiv_kernel<true>, grid, dim3(256), 0, s, (int)m,
                               (int)(c0 + w), (int)c0, (int)w, P, ldp, nrow, info, count,
                               col_base);
        else
            hipLaunchKernelGGL(lp_leaf_nopiv_kernel<false>, grid, dim3(256), 0, s, (int)m,
                               (int)(c0 + w), (int)c0, (int)w, P, ldp, nrow, info, count,
                               col_base);
        MXLU_LAUNCH_CHECK();
        return 0;
    }
    const int64_t w1 = std::max<int64_t>(kLpIb, (w / 2) / kLpIb * kLpIb);
    MXLU_TRY(panel_nopiv_rec(m, c0, w1, P, ldp, info, count, col_base, s));
    float *L11 = P + (size_t)c0 + (size_t)c0 * ldp;
    float *U12 = P + (size_t)c0 + (size_t)(c0 + w1) * ldp;
    MXLU_TRY(trsm_f32_llnu(w1, w - w1, L11, ldp, U12, ldp, s));
    if (m - c0 - w1 > 0)
        MXLU_TRY(gemm_f32_sub(m - c0 - w1, w - w1, w1, P + (size_t)(c0 + w1) + (size_t)c0 * ldp, ldp,
                              U12, ldp, P + (size_t)(c0 + w1) + (size_t)(c0 + w1) * ldp, ldp, s));
    return panel_nopiv_rec(m, c0 + w1, w - w1, P, ldp, info, count, col_base, s);
}

int lp_panel_factor_nopiv(int64_t m, int kb, float *P, int64_t ldp, int *info, int *count,
                          int64_t col_base, hipStream_t s) {
    if (m <= 0 || kb <= 0) return 0;
    return panel_nopiv_rec(m, 0, kb, P, ldp, info, count, col_base, s);
}

int trsm_f32_llnu(int64_t kb, int64_t ncols, const float *L, int64_t ldl, float *B, int64_t ldb,
                  hipStream_t s) {
    for (int64_t b0 = 0; b0 < kb; b0 += 256) {
        const int bb = (int)((kb - b0 < 256) ? kb - b0 : 256);
        const float *Lb = L + (size_t)b0 + (size_t)b0 * ldl;
        // wide blocks (the U12 TRSM of every step): 32 columns per workgroup,
        // which halves the workgroups re-reading the 256 x 256 diagonal block
        // (measured: 319 against 336 ms per FP8 solve at N = 131072; 64
        // columns, 357 ms); narrow ones (inside the panel): 16
        if (ncols >= 8192)
            hipLaunchKernelGGL(trsm_f32_llnu_kernel<32>, dim3((unsigned)((ncols + 31) / 32)),
                               dim3(256), 0, s, bb, ncols, Lb, ldl, B + b0, ldb);
        else
            hipLaunchKernelGGL(trsm_f32_llnu_kernel<16>, dim3((unsigned)((ncols + 15) / 16)),
                               dim3(256), 0, s, bb, ncols, Lb, ldl, B + b0, ldb);
        MXLU_LAUNCH_CHECK();
        if (b0 + bb < kb) {
            int rc = gemm_f32_sub(kb - b0 - bb, ncols, bb, L + (size_t)(b0 + bb) + (size_t)b0 * ldl,
                                  ldl, B + b0, ldb, B + b0 + bb, ldb, s);
            if (rc) return rc;
        }
    }
    return 0;
}

int lp_panel_store(int fmt, int64_t m, int kb, const float *P, int64_t ldp, uint16_t *F,
                   int64_t ldf, uint16_t *LTp, int64_t Mp, hipStream_t s) {
    if (m <= 0 || kb <= 0) return 0;
    if (LTp && (kb % kLpKc || Mp < m - kb)) {
        set_error_msg("lp_panel_store: packed L21 needs kb % 32 == 0 and Mp >= m - kb");
        return MXLU_E_NOMEM;
    }
    const int64_t tm = (m + 63) / 64, tn = (kb + 63) / 64;
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(panel_store_kernel<kFmtBf16>, dim3((unsigned)(tm * tn)), dim3(256), 0,
                           s, m, kb, P, ldp, F, ldf, LTp, Mp, (int)tm);
    else
        hipLaunchKernelGGL(panel_store_kernel<kFmtFp16>, dim3((unsigned)(tm * tn)), dim3(256), 0,
                           s, m, kb, P, ldp, F, ldf, LTp, Mp, (int)tm);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_pack_u12(int64_t nt, int kb, const uint16_t *U12, int64_t ldf, uint16_t *Up, int64_t Np,
                hipStream_t s) {
    if (nt <= 0 || kb <= 0) return 0;
    if (kb % kLpKc || ldf % 8 || Np < nt || ((uintptr_t)U12 | (uintptr_t)Up) % 16) {
        set_error_msg("lp_pack_u12: kb % 32, ldf % 8, Np >= nt and 16-byte alignment required");
        return MXLU_E_NOMEM;
    }
    const int64_t total = nt * (kb / 8);
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(pack_u12_kernel, dim3(grid), dim3(256), 0, s, nt, kb, U12, ldf, Up, Np);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_quant_l21(int fmt, int64_t mt, int kb, int tile, const uint16_t *L21, int64_t ldf,
                 uint8_t *LTq, int64_t Mp, float *sL, hipStream_t s) {
    if (mt <= 0 || kb <= 0) return 0;
    if (tile > 256 || kb % kLp8Kc || Mp < mt) {
        set_error_msg("lp_quant_l21: scale tile > 256, kb % 128 or Mp < rows");
        return MXLU_E_NOMEM;
    }
    const unsigned grid = (unsigned)((mt + tile - 1) / tile);
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(quant_l21_kernel<kFmtBf16>, dim3(grid), dim3(256), 0, s, mt, kb, tile,
                           L21, ldf, LTq, Mp, sL);
    else
        hipLaunchKernelGGL(quant_l21_kernel<kFmtFp16>, dim3(grid), dim3(256), 0, s, mt, kb, tile,
                           L21, ldf, LTq, Mp, sL);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_quant_l21_mx(int fmt, int64_t mt, int kb, const uint16_t *L21, int64_t ldf, uint8_t *LTq,
                    int64_t Mp, uint8_t *sLx, hipStream_t s) {
    if (mt <= 0 || kb <= 0) return 0;
    if (kb % kLp8Kc || Mp < mt || Mp % kLp8Kc || (uintptr_t)LTq % 16) {
        set_error_msg("lp_quant_l21_mx: kb % 128, Mp >= rows, Mp % 128 and alignment required");
        return MXLU_E_NOMEM;
    }
    const unsigned grid = (unsigned)((mt + 255) / 256);
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(quant_l21_mx_kernel<kFmtBf16>, dim3(grid), dim3(256), 0, s, mt, kb, L21,
                           ldf, LTq, Mp, sLx);
    else
        hipLaunchKernelGGL(quant_l21_mx_kernel<kFmtFp16>, dim3(grid), dim3(256), 0, s, mt, kb, L21,
                           ldf, LTq, Mp, sLx);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_quant_u12_mx(int fmt, int64_t nt, int kb, const uint16_t *U12, int64_t ldf, uint8_t *Uq,
                    int64_t Np, uint8_t *sUx, hipStream_t s) {
    if (nt <= 0 || kb <= 0) return 0;
    if (kb % kLp8Kc || Np < nt || (uintptr_t)Uq % 16) {
        set_error_msg("lp_quant_u12_mx: kb % 128, Np >= columns and alignment required");
        return MXLU_E_NOMEM;
    }
    const int64_t total = nt * (kb / 32);
    const unsigned grid = (unsigned)((total + 255) / 256);
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(quant_u12_mx_kernel<kFmtBf16>, dim3(grid), dim3(256), 0, s, nt, kb, U12,
                           ldf, Uq, Np, sUx);
    else
        hipLaunchKernelGGL(quant_u12_mx_kernel<kFmtFp16>, dim3(grid), dim3(256), 0, s, nt, kb, U12,
                           ldf, Uq, Np, sUx);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_quant_u12(int fmt, int64_t nt, int kb, int tile, const uint16_t *U12, int64_t ldf,
                 uint8_t *Uq, int64_t Np, float *sU, hipStream_t s) {
    if (nt <= 0 || kb <= 0) return 0;
    if (kb % kLp8Kc || Np < nt) {
        set_error_msg("lp_quant_u12: kb % 128 or Np < columns");
        return MXLU_E_NOMEM;
    }
    const unsigned grid = (unsigned)((nt + tile - 1) / tile);
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(quant_u12_kernel<kFmtBf16>, dim3(grid), dim3(256), 0, s, nt, kb, tile,
                           U12, ldf, Uq, Np, sU);
    else
        hipLaunchKernelGGL(quant_u12_kernel<kFmtFp16>, dim3(grid), dim3(256), 0, s, nt, kb, tile,
                           U12, ldf, Uq, Np, sU);
    MXLU_LAUNCH_CHECK();
    return 0;
}

}  // namespace mxlu
