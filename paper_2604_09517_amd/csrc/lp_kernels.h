// Launchers of the low-precision LU kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "asource.h"

namespace mxlu {

// inner block (leaf) width of the FP32 panel factorization: 64 columns take
// one recursion level (its leaf, TRSM and GEMM launches) off every panel
// against 32 (measured: 405 -> 397 ms per BF16 factorization at N = 65536)
constexpr int kLpIb = 64;

// F (rows x cols, 16-bit) <- round-to-nearest-even of A (FP64).
int lp_convert(int fmt, int64_t rows, int64_t cols, const double *A, int64_t lda, uint16_t *F,
               int64_t ldf, hipStream_t s);
// The same for the n x n matrix of `src` (in memory, or regenerated from its
// seed); gen_dominant_diag fills the diagonal of the seeded dominant matrix.
int lp_convert_src(int fmt, int64_t n, const ASource &src, uint16_t *F, int64_t ldf,
                   hipStream_t s);
// F = fp32(A) for FP32 factor storage (A in memory or seeded)
int lp_convert_src_f32(int64_t n, const ASource &src, float *F, int64_t ldf, hipStream_t s);
int gen_dominant_diag(int64_t n, uint64_t key, double *diag, hipStream_t s);
// P (FP32) <- F (16-bit), exact; F <- round(P).
int lp_load_f32(int fmt, int64_t rows, int64_t cols, const uint16_t *F, int64_t ldf, float *P,
                int64_t ldp, hipStream_t s);
int lp_store_f32(int fmt, int64_t rows, int64_t cols, const float *P, int64_t ldp, uint16_t *F,
                 int64_t ldf, hipStream_t s);
// C -= A B in FP32 with the elimination order of terms.
int gemm_f32_sub(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                 int64_t ldb, float *C, int64_t ldc, hipStream_t s);
// No-pivot FP32 factorization of the m x kb panel P in place; the first
// exactly-zero pivot (col_base + column, 1-based) goes to *info if still 0.
// count: a device int, zero on entry and left zero, used by the leaves (one
// panel at a time per count).
int lp_panel_factor_nopiv(int64_t m, int kb, float *P, int64_t ldp, int *info, int *count,
                          int64_t col_base, hipStream_t s);
// B (kb x ncols) <- L^-1 B, L unit lower (FP32), any kb.
int trsm_f32_llnu(int64_t kb, int64_t ncols, const float *L, int64_t ldl, float *B, int64_t ldb,
                  hipStream_t s);
// Chunk-packed operand of the 16-bit trailing update.  Line r (a row of L21
// or a column of U12), value k, sits at ((k / kLpKc) * Rp + r) * kLpKc +
// k % kLpKc, where Rp is the line count rounded up to the tile (kLpTileM rows
// of L21, kLpTileN columns of U12): one K chunk of one tile is one contiguous
// block, which the update copies to LDS with 16-byte direct loads.
constexpr int kLpKc = 32;
constexpr int kLpTileM = 256, kLpTileN = 128;
inline int64_t lp_round_up(int64_t r, int64_t t) { return (r + t - 1) / t * t; }

// F panel <- round(P); LTp <- the L21 rows (rows kb .. m-1 of the panel),
// chunk-packed with Mp lines (optional).
int lp_panel_store(int fmt, int64_t m, int kb, const float *P, int64_t ldp, uint16_t *F,
                   int64_t ldf, uint16_t *LTp, int64_t Mp, hipStream_t s);
// Up <- U12 (kb x nt block of F, column-major, kb % 8 == 0), chunk-packed
// with Np lines.
int lp_pack_u12(int64_t nt, int kb, const uint16_t *U12, int64_t ldf, uint16_t *Up, int64_t Np,
                hipStream_t s);
// FP8 operands of the trailing update with power-of-two tile scales, chunk-
// packed like the 16-bit ones with chunks of kLp8Kc values (one byte each)
// and lines rounded up to kLp8Tile: line r, value k at
// ((k / kLp8Kc) * Rp + r) * kLp8Kc + k % kLp8Kc.
constexpr int kLp8Kc = 128;
constexpr int kLp8Tile = 128;
int lp_quant_l21(int fmt, int64_t mt, int kb, int tile, const uint16_t *L21, int64_t ldf,
                 uint8_t *LTq, int64_t Mp, float *sL, hipStream_t s);
int lp_quant_u12(int fmt, int64_t nt, int kb, int tile, const uint16_t *U12, int64_t ldf,
                 uint8_t *Uq, int64_t Np, float *sU, hipStream_t s);

// MX form: e4m3 operands in the same chunk-packed layout with one E8M0 scale
// byte per line and block of 32 k: sLx[b Mp + r], sUx[b Np + c] (scale
// 2^(byte - 127)); kb % 128 == 0.
int lp_quant_l21_mx(int fmt, int64_t mt, int kb, const uint16_t *L21, int64_t ldf, uint8_t *LTq,
                    int64_t Mp, uint8_t *sLx, hipStream_t s);
int lp_quant_u12_mx(int fmt, int64_t nt, int kb, const uint16_t *U12, int64_t ldf, uint8_t *Uq,
                    int64_t Np, uint8_t *sUx, hipStream_t s);

// Trailing update on the matrix cores, of the M x N block C whose rows are
// lines i0 .. i0 + M - 1 of the packed L operand and whose columns are lines
// j0 .. j0 + N - 1 of the packed U operand (and of their scales; i0 and j0
// multiples of the tile sizes, and for FP8 of the scale tile, so that the
// tiles are those of the whole update):
//   16-bit: C <- round(fp32(C) - L U) with L (M x K) and U (K x N) chunk-packed
//           (Mp, Np lines), K % kLpKc == 0, C 8-byte aligned with ldc % 4 == 0,
//           i0 % 256 == 0, j0 % 128 == 0
//   FP8:    C <- round(fp32(C) - (Lq Uq) sL sU), e4m3fn operands chunk-packed
//           (Mp, Np lines), K % kLp8Kc == 0, tile % 4 == 0, i0 and j0
//           multiples of 128 and of the tile
int lp_schur_update(int fmt, int64_t M, int64_t N, int K, const uint16_t *Lp, int64_t Mp,
                    int64_t i0, const uint16_t *Up, int64_t Np, int64_t j0, uint16_t *C,
                    int64_t ldc, hipStream_t s);
int lp_schur_update_fp8(int fmt, int64_t M, int64_t N, int K, const uint8_t *Lq, int64_t Mp,
                        const float *sL, int64_t i0, const uint8_t *Uq, int64_t Np,
                        const float *sU, int64_t j0, int tile, uint16_t *C, int64_t ldc,
                        hipStream_t s);
//   MX:     C <- round(fp32(C) - sum_k (Lq sLx)(Uq sUx)), the E8M0 block scales
//           applied by the matrix cores; i0 and j0 multiples of 128
int lp_schur_update_mx(int fmt, int64_t M, int64_t N, int K, const uint8_t *Lq, int64_t Mp,
                       const uint8_t *sLx, int64_t i0, const uint8_t *Uq, int64_t Np,
                       const uint8_t *sUx, int64_t j0, uint16_t *C, int64_t ldc, hipStream_t s);

}  // namespace mxlu
