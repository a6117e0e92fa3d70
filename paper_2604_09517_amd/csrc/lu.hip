// Host driver of the FP64 path: lu_factor and lu_solve (Sec. III-A.1).
//
// lu_factor runs the right-looking blocked algorithm: for each panel of width
// nb, PFACT (recursive panel factorization whose leaves are the
// multi-workgroup pivoting kernel and whose inner nodes are TRSM + MFMA GEMM
// updates inside the panel), SWAP of the panel's interchanges on the columns
// left and right of it, DTRSM for the block row U12, and the MFMA DGEMM
// trailing update A22 -= L21 U12.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace {

using namespace mxlu;

struct FactorCtx {
    int64_t n, lda;
    double *A;
    int32_t *ipiv;
    PanelExchange ex;
    int *moves;
    hipStream_t s;
};

#define TRY(x)                 \
    do {                       \
        int rc_ = (x);         \
        if (rc_) return rc_;   \
    } while (0)

// Recursive factorization of the panel columns [c, c + w) (absolute), rows
// [c, n).  The panel spans columns [k0, k0 + kb); interchanges found inside
// it are applied to its other columns as soon as they are known.
int panel_rec(const FactorCtx &f, int64_t k0, int64_t kb, int64_t c, int64_t w) {
    const int64_t n = f.n, lda = f.lda;
    double *A = f.A;
    if (w <= kLeafW) {
        TRY(panel_leaf_f64(n - c, (int)w, A, lda, c, f.ipiv, f.ex, f.s));
        // the leaf's interchanges on the panel's other columns
        TRY(laswp_f64(A, lda, f.ipiv, c, (int)w, k0, kb - w, c, w, f.moves, f.s));
        return 0;
    }
    int64_t n1 = w / 2;
    n1 = std::max<int64_t>(kLeafW, (n1 / kLeafW) * kLeafW);
    const int64_t n2 = w - n1;
    TRY(panel_rec(f, k0, kb, c, n1));
    // A12 <- L11^-1 A12 ; A22 <- A22 - A21 A12   (inside the panel)
    double *L11 = &MXLU_AT(A, c, c, lda);
    double *A12 = &MXLU_AT(A, c, c + n1, lda);
    for (int64_t b0 = 0; b0 < n1; b0 += 256) {
        const int64_t bb = std::min<int64_t>(256, n1 - b0);
        TRY(trsm_llnu_f64((int)bb, n2, &MXLU_AT(L11, b0, b0, lda), lda, &MXLU_AT(A12, b0, 0, lda),
                          lda, f.s));
        if (b0 + bb < n1)
            TRY(gemm_f64_sub(n1 - b0 - bb, n2, bb, &MXLU_AT(L11, b0 + bb, b0, lda), lda,
                             &MXLU_AT(A12, b0, 0, lda), lda, &MXLU_AT(A12, b0 + bb, 0, lda), lda,
                             f.s));
    }
    TRY(gemm_f64_sub(n - c - n1, n2, n1, &MXLU_AT(A, c + n1, c, lda), lda, A12, lda,
                     &MXLU_AT(A, c + n1, c + n1, lda), lda, f.s));
    TRY(panel_rec(f, k0, kb, c + n1, n2));
    return 0;
}

// Blocked U12 = L11^-1 A12 for any kb (diagonal blocks of 256 + GEMM).
int trsm_block_row(double *A, int64_t lda, int64_t k0, int64_t kb, int64_t ncols,
                   int64_t col0, hipStream_t s) {
    for (int64_t b0 = 0; b0 < kb; b0 += 256) {
        const int64_t bb = std::min<int64_t>(256, kb - b0);
        TRY(trsm_llnu_f64((int)bb, ncols, &MXLU_AT(A, k0 + b0, k0 + b0, lda), lda,
                          &MXLU_AT(A, k0 + b0, col0, lda), lda, s));
        if (b0 + bb < kb)
            TRY(gemm_f64_sub(kb - b0 - bb, ncols, bb, &MXLU_AT(A, k0 + b0 + bb, k0 + b0, lda),
                             lda, &MXLU_AT(A, k0 + b0, col0, lda), lda,
                             &MXLU_AT(A, k0 + b0 + bb, col0, lda), lda, s));
    }
    return 0;
}

int factor_impl(int64_t n, int64_t nb, double *A, int64_t lda, int32_t *ipiv, hipStream_t s,
                int *info_out) {
    Scratch scratch(s);
    FactorCtx f;
    f.n = n;
    f.lda = lda;
    f.A = A;
    f.ipiv = ipiv;
    f.s = s;
    f.ex.cand = scratch.alloc_n<double>((size_t)2 * kMaxGroups * (kLeafW + 2));
    f.ex.rowj = scratch.alloc_n<double>((size_t)2 * kLeafW);
    f.ex.counters = scratch.alloc_n<int>((size_t)n);
    f.ex.flags = scratch.alloc_n<int>(4);
    f.moves = scratch.alloc_n<int>(kSwapMovesInts);
    if (!f.ex.cand || !f.ex.rowj || !f.ex.counters || !f.ex.flags || !f.moves)
        return MXLU_E_NOMEM;
    MXLU_HIP_TRY(hipMemsetAsync(f.ex.counters, 0, sizeof(int) * (size_t)n, s));
    MXLU_HIP_TRY(hipMemsetAsync(f.ex.flags, 0, sizeof(int) * 4, s));

    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        const int64_t kb = std::min(nb, n - k0);
        // PFACT
        TRY(panel_rec(f, k0, kb, k0, kb));
        // SWAP on the columns left and right of the panel
        TRY(laswp_f64(A, lda, ipiv, k0, (int)kb, 0, n - kb, k0, kb, f.moves, s));
        const int64_t c1 = k0 + kb;
        if (c1 < n) {
            // DTRSM: U12 = L11^-1 A12
            TRY(trsm_block_row(A, lda, k0, kb, n - c1, c1, s));
            // DGEMM: A22 -= L21 U12
            TRY(gemm_f64_sub(n - c1, n - c1, kb, &MXLU_AT(A, c1, k0, lda), lda,
                             &MXLU_AT(A, k0, c1, lda), lda, &MXLU_AT(A, c1, c1, lda), lda, s));
        }
    }
    int flags[4] = {0, 0, 0, 0};
    MXLU_HIP_TRY(hipMemcpyAsync(flags, f.ex.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    MXLU_HIP_TRY(hipStreamSynchronize(s));
    if (flags[1]) {
        set_error_msg("lu_factor: panel grid barrier wait expired");
        return MXLU_E_TIMEOUT;
    }
    *info_out = flags[0];
    return 0;
}

}  // namespace

extern "C" int lu_factor(int64_t n, int64_t nb, double *A, int64_t lda, int32_t *ipiv,
                         void *stream) {
    if (n < 0) return -1;
    if (nb < 1) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && !ipiv) return -5;
    if (n > 0x7fffffff) return -1;
    if (nb > 1024) return -2;
    if (n == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    int info = 0;
    int rc = factor_impl(n, nb, A, lda, ipiv, (hipStream_t)stream, &info);
    if (rc) return rc;
    return info;
}

extern "C" int lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                        const int32_t *ipiv, double *B, int64_t ldb, int trans, void *stream) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && !LU) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && !ipiv) return -5;
    if (n > 0 && nrhs > 0 && !B) return -6;
    if (ldb < std::max<int64_t>(1, n)) return -7;
    if (trans != 0 && trans != 1) return -8;
    if (n > 0x7fffffff) return -1;
    if (n == 0 || nrhs == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    Scratch scratch(s);
    int32_t *perm = scratch.alloc_n<int32_t>((size_t)n);
    if (!perm) return MXLU_E_NOMEM;
    TRY(perm_from_ipiv(n, ipiv, perm, s));

    // Work on strips of at most 16 right-hand sides.
    const int64_t bs = 256;
    double *Y = scratch.alloc_n<double>((size_t)n * (size_t)std::min<int64_t>(16, nrhs));
    if (!Y) return MXLU_E_NOMEM;
    const int64_t ldy = n;
    for (int64_t r0 = 0; r0 < nrhs; r0 += 16) {
        const int64_t nr = std::min<int64_t>(16, nrhs - r0);
        double *Bc = B + (size_t)r0 * (size_t)ldb;
        if (trans == 0) {
            TRY(gather_rows_f64(n, nr, perm, Bc, ldb, Y, ldy, s));
            // L y = P b: diagonal blocks forward, updates below
            for (int64_t b0 = 0; b0 < n; b0 += bs) {
                const int64_t bb = std::min(bs, n - b0);
                TRY(trsm_llnu_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
                if (b0 + bb < n)
                    TRY(gemm_f64_sub(n - b0 - bb, nr, bb, &MXLU_AT(LU, b0 + bb, b0, lda), lda,
                                     Y + b0, ldy, Y + b0 + bb, ldy, s));
            }
            // U x = y: diagonal blocks backward, updates above
            const int64_t nblk = (n + bs - 1) / bs;
            for (int64_t bi = nblk - 1; bi >= 0; --bi) {
                const int64_t b0 = bi * bs, bb = std::min(bs, n - b0);
                TRY(trsm_lunn_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
                if (b0 > 0)
                    TRY(gemm_f64_sub(b0, nr, bb, &MXLU_AT(LU, 0, b0, lda), lda, Y + b0, ldy, Y,
                                     ldy, s));
            }
            // copy back
            MXLU_HIP_TRY(hipMemcpy2DAsync(Bc, sizeof(double) * ldb, Y, sizeof(double) * ldy,
                                          sizeof(double) * n, nr, hipMemcpyDeviceToDevice, s));
        } else {
            MXLU_HIP_TRY(hipMemcpy2DAsync(Y, sizeof(double) * ldy, Bc, sizeof(double) * ldb,
                                          sizeof(double) * n, nr, hipMemcpyDeviceToDevice, s));
            // U^T y = b: forward; block b0 first takes the contributions of
            // the solved rows above it
            for (int64_t b0 = 0; b0 < n; b0 += bs) {
                const int64_t bb = std::min(bs, n - b0);
                if (b0 > 0)
                    TRY(gemm_f64_sub_tn_skinny(bb, nr, b0, &MXLU_AT(LU, 0, b0, lda), lda, Y, ldy,
                                               Y + b0, ldy, s));
                TRY(trsm_lutn_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
            }
            // L^T z = y: backward; block first takes the rows below it
            const int64_t nblk = (n + bs - 1) / bs;
            for (int64_t bi = nblk - 1; bi >= 0; --bi) {
                const int64_t b0 = bi * bs, bb = std::min(bs, n - b0);
                if (b0 + bb < n)
                    TRY(gemm_f64_sub_tn_skinny(bb, nr, n - b0 - bb, &MXLU_AT(LU, b0 + bb, b0, lda),
                                               lda, Y + b0 + bb, ldy, Y + b0, ldy, s));
                TRY(trsm_lltu_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
            }
            TRY(scatter_rows_f64(n, nr, perm, Y, ldy, Bc, ldb, s));
        }
    }
    return 0;
}

extern "C" int mxlu_schur_update_f64(int64_t M, int64_t N, int64_t K, const double *A,
                                     int64_t lda, const double *B, int64_t ldb, double *C,
                                     int64_t ldc, void *stream) {
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (M > 0 && K > 0 && !A) return -4;
    if (lda < std::max<int64_t>(1, M)) return -5;
    if (K > 0 && N > 0 && !B) return -6;
    if (ldb < std::max<int64_t>(1, K)) return -7;
    if (M > 0 && N > 0 && !C) return -8;
    if (ldc < std::max<int64_t>(1, M)) return -9;
    if (M == 0 || N == 0 || K == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    return gemm_f64_sub(M, N, K, A, lda, B, ldb, C, ldc, (hipStream_t)stream);
}
