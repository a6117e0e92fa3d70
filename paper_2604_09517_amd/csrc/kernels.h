// Host-side launchers of the library's kernels (internal interface).
// Every launcher enqueues on stream `s` and returns 0 or an MXLU_E_* code.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>

namespace mxlu {

// C(M x N) -= A(M x K) * B(K x N), FP64, column-major.
// `trailing` marks the DGEMM phase of the factorization (its own kernel
// instance, so that profiles separate it from the updates inside the panel).
int gemm_f64_sub(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double *C, int64_t ldc, hipStream_t s,
                 bool trailing = false);
// C(M x N) = (accumulate ? C : 0) - A(M x K) * B(N x K)^T.
// The trailing update A22 -= L21 U12 of the factorization with the
// register-direct kernel: full 128 x 128 tiles, K % 16 == 0, lda even and A
// 16-byte aligned (gemm_f64_update_ok; C must also be 16-byte aligned with
// ldc even); B comes as Bn = -U12^T, row-major with leading dimension
// ldbn >= N (even, 16-byte aligned), written by pack_neg_transpose_f64.
bool gemm_f64_update_ok(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda);
int pack_neg_transpose_f64(int64_t K, int64_t N, const double *B, int64_t ldb, double *Bn,
                           int64_t ldbn, hipStream_t s);
int gemm_f64_update(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                    const double *Bn, int64_t ldbn, double *C, int64_t ldc, hipStream_t s);
int gemm_f64_nt_sub(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc, bool accumulate,
                    hipStream_t s);

// Exchange area of the multi-workgroup panel kernel (64-bit words, each a
// 32-bit payload tagged with a 32-bit column sequence number).
struct PanelExchange {
    uint64_t *slots;  // [2][kMaxGroups][4] candidates, then [2][kMaxGroups][kLeafW * 2] rows
    uint64_t *rowj;   // [2][kLeafW * 2] the current pivot row's old contents
    int *flags;       // [0]: first zero pivot (1-based), [1]: wait expired
    int group_cap;    // CUs a leaf may occupy (0: all); the LDS form puts one workgroup on each
};
constexpr int kLeafW = 32;        // columns factored by one leaf kernel
constexpr int kMaxGroups = 256;   // workgroups of one leaf kernel (<= CUs)

// Factor the m x w (w <= kLeafW) leaf whose top-left element is P (leading
// dimension ldp) with partial pivoting.  r0 is the leaf's first row/column
// index within the caller's numbering: ipiv[r0 .. r0+w) receives r0 + the
// pivot row within the leaf; the column numbers r0 + j + 1 are the values of
// the workgroups' sequence flags, so they must grow from leaf to leaf.
// Workgroups the leaf kernel launches for an m-row leaf with group cap `cap`
// (they must all be resident at once), or -1 when no geometry fits.
template <typename T> int panel_leaf_groups(int64_t m, int cap);

// Inputs of the leaf planner: the CUs the leaf may use (cap > 0: that many,
// else all `cus`), workgroups of the register form per CU (0: form not
// available), dynamic LDS per workgroup of the LDS form, element size.
struct LeafDevice {
    int cap, cus, occ_reg1, occ_reg2, elem_bytes;
    int64_t lds_budget;
};
enum { kLeafNone = 0, kLeafReg1 = 1, kLeafReg2 = 2, kLeafLds = 3 };
// Form (kLeaf*) and geometry (rows per group R, groups G) of an m-row leaf;
// host arithmetic only.
int leaf_plan(int64_t m, const LeafDevice &d, int64_t *R, int64_t *G);
// The current device's facts for the FP64 leaf with group cap `cap`.
int leaf_device_f64(int cap, LeafDevice *d);

template <typename T>
int panel_leaf(int64_t m, int w, T *P, int64_t ldp, int64_t r0, int32_t *ipiv,
               const PanelExchange &ex, hipStream_t s);

// Interchanges ipiv[j0 .. j0+cnt) (rows >= j0, cnt <= 1024, of a matrix with
// nrows rows) composed into a list of row moves, then applied to the columns
// c_begin + q (q < ncols, skipping [skip_begin, skip_begin + skip_len)) of a
// matrix of T.  An interchange row outside [j0 + t, nrows) counts as none.
int swap_compose(const int32_t *ipiv, int64_t j0, int cnt, int64_t nrows, int *moves,
                 hipStream_t s);
// The interchanges of every step applied to the columns left of its panel,
// deferred to after the factorization (each element moves once).  q, r: n
// ints of scratch; T: (n - nb) x nb doubles of scratch.
// y -= A x (one right-hand side; A is M x K, column-major), deterministic.
int gemv_f64_sub(int64_t M, int64_t K, const double *A, int64_t lda, const double *x, double *y,
                 hipStream_t s);
int laswp_left_deferred_f64(double *A, int64_t lda, int64_t n, int64_t nb,
                            const int32_t *ipiv, int *moves, int32_t *q, int32_t *r, double *T,
                            hipStream_t s);
template <typename T>
int swap_apply(T *A, int64_t lda, int64_t j0, const int *moves, int64_t c_begin, int64_t ncols,
               int64_t skip_begin, int64_t skip_len, hipStream_t s);

// Apply the interchanges ipiv[j0 .. j0+cnt) (absolute rows, cnt <= 1024) to
// the columns c_begin + q (q < ncols, skipping [skip_begin, skip_begin +
// skip_len)).  `moves` is a device buffer of kSwapMovesInts ints.
constexpr int kSwapMovesInts = 1 + 4 * 1024;
int laswp_f64(double *A, int64_t lda, int64_t nrows, const int32_t *ipiv, int64_t j0, int cnt,
              int64_t c_begin, int64_t ncols, int64_t skip_begin, int64_t skip_len,
              int *moves, hipStream_t s);

// B(kb x ncols) = L^-1 B with L unit lower (kb x kb), kb <= 256.
int trsm_llnu_f64(int kb, int64_t ncols, const double *L, int64_t ldl, double *B,
                  int64_t ldb, hipStream_t s);
// B(kb x ncols) = U^-1 B with U upper, non-unit (kb <= 256).
// One right-hand side y (bb <= 256 values) through the diagonal block T:
// lower = unit lower forward, else upper (non-unit) backward.
int trsv_block_f64(int bb, bool lower, const double *T, int64_t ldt, double *y, hipStream_t s);
int trsm_lunn_f64(int kb, int64_t ncols, const double *U, int64_t ldu, double *B,
                  int64_t ldb, hipStream_t s);
// B(kb x ncols) = U^-T B (U upper non-unit) and B = L^-T B (L unit lower).
int trsm_lutn_f64(int kb, int64_t ncols, const double *U, int64_t ldu, double *B,
                  int64_t ldb, hipStream_t s);
int trsm_lltu_f64(int kb, int64_t ncols, const double *L, int64_t ldl, double *B,
                  int64_t ldb, hipStream_t s);

class Scratch;
extern std::atomic<int> g_expire_waits;
// Zeroed exchange area of the panel kernels for a matrix of order n.
int alloc_panel_exchange(Scratch &scratch, int64_t n, PanelExchange *ex, hipStream_t s);
// GEPP of the m x kb panel P (recursive; leaves are panel_leaf<T>); element
// (0, 0) is row/column ibase of the caller's matrix, ipiv[ibase ..] receives
// caller-numbered rows; the interchanges are applied inside the panel only.
// moves: kSwapMovesInts device ints.
template <typename T>
int panel_factor(T *P, int64_t ldp, int64_t m, int64_t kb, int64_t ibase, int32_t *ipiv,
                 const PanelExchange &ex, int *moves, hipStream_t s);

// C(M x N) -= A(K x M)^T * B(K x N), N <= 16 (transposed solves' updates).
int gemm_f64_sub_tn_skinny(int64_t M, int64_t N, int64_t K, const double *A, int64_t lda,
                           const double *B, int64_t ldb, double *C, int64_t ldc,
                           hipStream_t s);

// perm[i] = original row at position i after the interchanges ipiv[0..n).
int perm_from_ipiv(int64_t n, const int32_t *ipiv, int32_t *perm, hipStream_t s);
// Y(i, c) = B(perm[i], c)  (gather)   /   B(perm[i], c) = Y(i, c)  (scatter)
int gather_rows_f64(int64_t n, int64_t nrhs, const int32_t *perm, const double *B,
                    int64_t ldb, double *Y, int64_t ldy, hipStream_t s);
int scatter_rows_f64(int64_t n, int64_t nrhs, const int32_t *perm, const double *Y,
                     int64_t ldy, double *B, int64_t ldb, hipStream_t s);

// Streams of the mixed-precision factorization's look-ahead: `panel` factors
// the next panel while the rest of the trailing update runs on the caller's
// stream.  False at look-ahead depth 0 or when the streams are missing; on
// true the caller holds the process-wide look-ahead lock in *lk until its
// factorization has completed (the streams are shared by every call).
struct AheadStreams {
    hipStream_t panel = nullptr;
};
bool lp_ahead_streams(AheadStreams *out, std::unique_lock<std::mutex> *lk);

}  // namespace mxlu
