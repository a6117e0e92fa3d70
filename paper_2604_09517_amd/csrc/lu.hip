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
#include "lp_kernels.h"
#include "profile.h"

namespace {

using namespace mxlu;

// Element-type specific TRSM / GEMM used by the panel recursion.
template <typename T> struct PanelOps;
template <> struct PanelOps<double> {
    // B (kb x ncols) <- L^-1 B, L unit lower, any kb (diagonal blocks of 256)
    static int trsm(int64_t kb, int64_t ncols, const double *L, int64_t ldl, double *B,
                    int64_t ldb, hipStream_t s) {
        for (int64_t b0 = 0; b0 < kb; b0 += 256) {
            const int64_t bb = std::min<int64_t>(256, kb - b0);
            MXLU_TRY(trsm_llnu_f64((int)bb, ncols, &MXLU_AT(L, b0, b0, ldl), ldl, B + b0, ldb, s));
            if (b0 + bb < kb)
                MXLU_TRY(gemm_f64_sub(kb - b0 - bb, ncols, bb, &MXLU_AT(L, b0 + bb, b0, ldl), ldl,
                                 B + b0, ldb, B + b0 + bb, ldb, s));
        }
        return 0;
    }
    static int gemm(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t s) {
        return gemm_f64_sub(M, N, K, A, lda, B, ldb, C, ldc, s);
    }
};
template <> struct PanelOps<float> {
    static int trsm(int64_t kb, int64_t ncols, const float *L, int64_t ldl, float *B,
                    int64_t ldb, hipStream_t s) {
        return trsm_f32_llnu(kb, ncols, L, ldl, B, ldb, s);
    }
    static int gemm(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const float *B,
                    int64_t ldb, float *C, int64_t ldc, hipStream_t s) {
        return gemm_f32_sub(M, N, K, A, lda, B, ldb, C, ldc, s);
    }
};

template <typename T>
struct PanelCtx {
    T *P;            // panel top-left element
    int64_t ldp, m, kb, ibase;
    int32_t *ipiv;   // indexed in the caller's numbering (ibase + local)
    PanelExchange ex;
    int *moves;
    hipStream_t s;
};

// Recursive factorization of the panel columns [c, c + w) (panel-local),
// rows [c, m).  Interchanges found in a leaf are applied at once to the
// panel's other columns; the halves are joined by a TRSM and a GEMM update,
// so every element still takes its terms in ascending k (the order of
// unblocked elimination).
template <typename T>
int panel_rec(const PanelCtx<T> &f, int64_t c, int64_t w) {
    T *P = f.P;
    const int64_t ldp = f.ldp;
    if (w <= kLeafW) {
        MXLU_TRY(panel_leaf<T>(f.m - c, (int)w, P + (size_t)c + (size_t)c * ldp, ldp, f.ibase + c,
                          f.ipiv, f.ex, f.s));
        if (f.kb > w) {
            MXLU_TRY(swap_compose(f.ipiv, f.ibase + c, (int)w, f.moves, f.s));
            MXLU_TRY(swap_apply<T>(P, ldp, c, f.moves, 0, f.kb - w, c, w, f.s));
        }
        return 0;
    }
    int64_t n1 = w / 2;
    n1 = std::max<int64_t>(kLeafW, (n1 / kLeafW) * kLeafW);
    const int64_t n2 = w - n1;
    MXLU_TRY(panel_rec(f, c, n1));
    T *A12 = P + (size_t)c + (size_t)(c + n1) * ldp;
    MXLU_TRY(PanelOps<T>::trsm(n1, n2, P + (size_t)c + (size_t)c * ldp, ldp, A12, ldp, f.s));
    MXLU_TRY(PanelOps<T>::gemm(f.m - c - n1, n2, n1, P + (size_t)(c + n1) + (size_t)c * ldp, ldp, A12,
                          ldp, P + (size_t)(c + n1) + (size_t)(c + n1) * ldp, ldp, f.s));
    MXLU_TRY(panel_rec(f, c + n1, n2));
    return 0;
}

}  // namespace

namespace mxlu {
// GEPP of the m x kb panel P (element (0, 0) is row/column ibase of the
// caller's matrix); ipiv[ibase ..] receives caller-numbered rows.
template <typename T>
int panel_factor(T *P, int64_t ldp, int64_t m, int64_t kb, int64_t ibase, int32_t *ipiv,
                 const PanelExchange &ex, int *moves, hipStream_t s) {
    PanelCtx<T> f{P, ldp, m, kb, ibase, ipiv, ex, moves, s};
    return panel_rec(f, 0, kb);
}
template int panel_factor<double>(double *, int64_t, int64_t, int64_t, int64_t, int32_t *,
                                  const PanelExchange &, int *, hipStream_t);
template int panel_factor<float>(float *, int64_t, int64_t, int64_t, int64_t, int32_t *,
                                 const PanelExchange &, int *, hipStream_t);

int alloc_panel_exchange(Scratch &scratch, int64_t n, PanelExchange *ex, hipStream_t s) {
    const size_t slot_words = (size_t)2 * kMaxGroups * (2 * kLeafW + 4);
    const size_t rowj_words = (size_t)2 * 2 * kLeafW;
    ex->slots = scratch.alloc_n<uint64_t>(slot_words);
    ex->rowj = scratch.alloc_n<uint64_t>(rowj_words);
    ex->flags = scratch.alloc_n<int>(4);
    (void)n;
    if (!ex->slots || !ex->rowj || !ex->flags) return MXLU_E_NOMEM;
    // sequence number 0 is never current: zeroed words never match
    MXLU_HIP_TRY(hipMemsetAsync(ex->slots, 0, sizeof(uint64_t) * slot_words, s));
    MXLU_HIP_TRY(hipMemsetAsync(ex->rowj, 0, sizeof(uint64_t) * rowj_words, s));
    MXLU_HIP_TRY(hipMemsetAsync(ex->flags, 0, sizeof(int) * 4, s));
    return 0;
}
}  // namespace mxlu

namespace {

int factor_impl(int64_t n, int64_t nb, double *A, int64_t lda, int32_t *ipiv, hipStream_t s,
                int *info_out) {
    Scratch scratch(s);
    PanelExchange ex;
    MXLU_TRY(alloc_panel_exchange(scratch, n, &ex, s));
    int *moves = scratch.alloc_n<int>(kSwapMovesInts);
    if (!moves) return MXLU_E_NOMEM;
    // packed -U12^T for the trailing update (nb rows of up to n values)
    const int64_t ldbn = (n + 1) / 2 * 2;
    double *Bn = scratch.alloc_n<double>((size_t)nb * (size_t)ldbn);
    if (!Bn) return MXLU_E_NOMEM;

    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        const int64_t kb = std::min(nb, n - k0);
        const int64_t m = n - k0, c1 = k0 + kb;
        {   // PFACT
            PhaseScope ph(kPhasePfact, s, (double)m * kb * 8.0);
            MXLU_TRY(panel_factor<double>(&MXLU_AT(A, k0, k0, lda), lda, m, kb, k0, ipiv, ex, moves,
                                     s));
        }
        {   // SWAP on the columns left and right of the panel
            PhaseScope ph(kPhaseSwap, s, 32.0 * kb * (double)(n - kb));
            MXLU_TRY(laswp_f64(A, lda, ipiv, k0, (int)kb, 0, n - kb, k0, kb, moves, s));
        }
        if (c1 < n) {
            const int64_t nt = n - c1;
            double *L21 = &MXLU_AT(A, c1, k0, lda), *U12 = &MXLU_AT(A, k0, c1, lda);
            const bool ring = gemm_f64_ring_ok(nt, nt, kb, L21, lda);
            {   // DTRSM: U12 = L11^-1 A12 (then, for the ring kernel, -U12^T packed)
                PhaseScope ph(kPhaseTrsm, s, (double)kb * (kb - 1) * (double)nt);
                MXLU_TRY(PanelOps<double>::trsm(kb, nt, &MXLU_AT(A, k0, k0, lda), lda, U12, lda, s));
                if (ring) MXLU_TRY(pack_neg_transpose_f64(kb, nt, U12, lda, Bn, ldbn, s));
            }
            {   // DGEMM: A22 -= L21 U12
                PhaseScope ph(kPhaseGemm, s, 2.0 * (double)nt * (double)nt * (double)kb);
                if (ring)
                    MXLU_TRY(gemm_f64_ring(nt, nt, kb, L21, lda, Bn, ldbn, &MXLU_AT(A, c1, c1, lda),
                                           lda, s));
                else
                    MXLU_TRY(gemm_f64_sub(nt, nt, kb, L21, lda, U12, lda, &MXLU_AT(A, c1, c1, lda),
                                          lda, s, true));
            }
        }
    }
    int flags[4] = {0, 0, 0, 0};
    MXLU_HIP_TRY(hipMemcpyAsync(flags, ex.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
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
    PhaseScope ph(kPhaseSolve, s, 8.0 * (double)n * (double)n);
    int32_t *perm = scratch.alloc_n<int32_t>((size_t)n);
    if (!perm) return MXLU_E_NOMEM;
    MXLU_TRY(perm_from_ipiv(n, ipiv, perm, s));

    // Work on strips of at most 16 right-hand sides.
    const int64_t bs = 256;
    double *Y = scratch.alloc_n<double>((size_t)n * (size_t)std::min<int64_t>(16, nrhs));
    if (!Y) return MXLU_E_NOMEM;
    const int64_t ldy = n;
    for (int64_t r0 = 0; r0 < nrhs; r0 += 16) {
        const int64_t nr = std::min<int64_t>(16, nrhs - r0);
        double *Bc = B + (size_t)r0 * (size_t)ldb;
        if (trans == 0) {
            MXLU_TRY(gather_rows_f64(n, nr, perm, Bc, ldb, Y, ldy, s));
            // L y = P b: diagonal blocks forward, updates below
            for (int64_t b0 = 0; b0 < n; b0 += bs) {
                const int64_t bb = std::min(bs, n - b0);
                MXLU_TRY(trsm_llnu_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
                if (b0 + bb < n)
                    MXLU_TRY(gemm_f64_sub(n - b0 - bb, nr, bb, &MXLU_AT(LU, b0 + bb, b0, lda), lda,
                                     Y + b0, ldy, Y + b0 + bb, ldy, s));
            }
            // U x = y: diagonal blocks backward, updates above
            const int64_t nblk = (n + bs - 1) / bs;
            for (int64_t bi = nblk - 1; bi >= 0; --bi) {
                const int64_t b0 = bi * bs, bb = std::min(bs, n - b0);
                MXLU_TRY(trsm_lunn_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
                if (b0 > 0)
                    MXLU_TRY(gemm_f64_sub(b0, nr, bb, &MXLU_AT(LU, 0, b0, lda), lda, Y + b0, ldy, Y,
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
                    MXLU_TRY(gemm_f64_sub_tn_skinny(bb, nr, b0, &MXLU_AT(LU, 0, b0, lda), lda, Y, ldy,
                                               Y + b0, ldy, s));
                MXLU_TRY(trsm_lutn_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
            }
            // L^T z = y: backward; block first takes the rows below it
            const int64_t nblk = (n + bs - 1) / bs;
            for (int64_t bi = nblk - 1; bi >= 0; --bi) {
                const int64_t b0 = bi * bs, bb = std::min(bs, n - b0);
                if (b0 + bb < n)
                    MXLU_TRY(gemm_f64_sub_tn_skinny(bb, nr, n - b0 - bb, &MXLU_AT(LU, b0 + bb, b0, lda),
                                               lda, Y + b0 + bb, ldy, Y + b0, ldy, s));
                MXLU_TRY(trsm_lltu_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy, s));
            }
            MXLU_TRY(scatter_rows_f64(n, nr, perm, Y, ldy, Bc, ldb, s));
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
    return gemm_f64_sub(M, N, K, A, lda, B, ldb, C, ldc, (hipStream_t)stream, true);
}

extern "C" int mxlu_outer_update_f64(int64_t M, int64_t N, int64_t K, const double *A,
                                     int64_t lda, const double *B, int64_t ldb, double *C,
                                     int64_t ldc, int accumulate, void *stream) {
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (M > 0 && K > 0 && !A) return -4;
    if (lda < std::max<int64_t>(1, M)) return -5;
    if (N > 0 && K > 0 && !B) return -6;
    if (ldb < std::max<int64_t>(1, N)) return -7;
    if (M > 0 && N > 0 && !C) return -8;
    if (ldc < std::max<int64_t>(1, M)) return -9;
    if (accumulate != 0 && accumulate != 1) return -10;
    if (M == 0 || N == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    return gemm_f64_nt_sub(M, N, K, A, lda, B, ldb, C, ldc, accumulate != 0, (hipStream_t)stream);
}
