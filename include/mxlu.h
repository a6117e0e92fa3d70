/*
 * mxlu.h -- C ABI of the MI355X (gfx950) dense LU solver.
 *
 * The operations are those of the paper's benchmarks (Sec. III-A.1: solve
 * A x = b, A an N x N FP64 matrix: factor P A = L U with row interchanges
 * chosen by the largest magnitude in each column, then solve with the two
 * triangular factors; the factorization is the right-looking blocked
 * algorithm of panel width NB with the phases PFACT, SWAP, DTRSM, DGEMM;
 * Sec. III-A.2: the mixed-precision variant, low-precision factorization and
 * trailing updates without pivoting, accuracy restored by FP64 iterative
 * refinement; Sec. II-B: refinement based on GMRES).
 *
 * Conventions for every entry point
 *   - Matrices are column-major with a leading dimension >= max(1, rows).
 *   - All array arguments are DEVICE pointers (memory of the current HIP
 *     device), owned by the caller.  The library never frees caller memory;
 *     internal scratch is allocated stream-ordered on `stream` and released
 *     before the call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it.
 *   - Return value: 0 on success; -k when the k-th argument is invalid
 *     (checked on the host before anything is enqueued); > 0 from a
 *     factorization when a pivot is exactly zero (see lu_factor); <= -1000 for
 *     runtime failures (MXLU_E_*), with details in mxlu_last_error().
 *   - Pivots: LAPACK interchange sequence, int32, 0-based: at step j row j was
 *     swapped with row ipiv[j] >= j.  P = P_{n-1} ... P_0 and P A = L U.
 */
#ifndef MXLU_H
#define MXLU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MXLU_OK = 0,
    MXLU_E_NODEV = -1001,    /* no HIP device visible */
    MXLU_E_HIP = -1002,      /* a HIP runtime call failed */
    MXLU_E_NOMEM = -1003,    /* a size overflows or an allocation failed */
    MXLU_E_NOTCONV = -1004,  /* refinement did not reach the threshold */
    MXLU_E_TIMEOUT = -1005,  /* a kernel's bounded wait expired (results invalid) */
    MXLU_E_WORKSPACE = -1006 /* caller workspace too small */
};

/*
 * lu_factor -- blocked right-looking LU with partial pivoting (Sec. III-A.1).
 *   n      order of A (>= 0)
 *   nb     panel width NB (1 <= nb <= 1024)
 *   A      n x n FP64, leading dimension lda; overwritten by L (unit lower,
 *          multipliers below the diagonal) and U (upper), as LAPACK getrf
 *   ipiv   n int32 (device): the interchange sequence
 * Pivot choice: the first row of largest magnitude (ties go to the smaller
 * row index).  An exactly zero pivot column is left unscaled and the call
 * returns its 1-based index (the first one); the factorization still
 * completes.  Synchronises `stream` once at the end (to read that status).
 */
int lu_factor(int64_t n, int64_t nb, double *A, int64_t lda, int32_t *ipiv,
              void *stream);

/*
 * mxlu_set_lookahead -- look-ahead depth of lu_factor (Sec. III-A.1 names
 * look-ahead as the way to take the panel off the critical path; Sec. IV-B's
 * configuration table runs HPL with depth 1).  Process-wide, default 1.
 *   depth 0: each step runs PFACT, SWAP, DTRSM and DGEMM in order on the
 *            caller's stream.
 *   depth 1: the update of the next panel's columns runs first; that panel
 *            is then factored on a stream masked to a quarter of the CUs
 *            while the rest of the update runs on a stream masked to the
 *            other CUs; both join the caller's stream before the next SWAP.
 *            Used when n and nb are multiples of 128, lda is even, A is
 *            16-byte aligned and n > nb; otherwise lu_factor runs depth 0.
 * The same depth applies to the low-precision factorization of mxp_solve
 * without pivoting: at depth 1 the update of the next panel's columns runs
 * first, then that panel is factored on a side stream of the library while
 * the rest of the update runs on the caller's stream (used when nb is a
 * multiple of 128 and, for FP8 with tile scales, of scale_tile).
 * The factors and ipiv are the same at both depths (each element takes the
 * same operations in the same order).  Returns 0, or -1 for a depth other
 * than 0 or 1.
 */
int mxlu_set_lookahead(int depth);

/*
 * mxlu_release -- destroys what the library keeps between calls: the two
 * CU-masked streams of the look-ahead and the side stream of the
 * mixed-precision look-ahead (per device), and the pooled timing events.  They are created again on demand.  Call it only while no library
 * work is in flight; it also runs at process exit (registered when the
 * streams are first created, so before the HIP runtime's own teardown).
 * Returns 0.
 *
 * Residency.  The panel kernels' workgroups exchange pivot candidates while
 * running, so all of them must be resident at once: the planner sizes them
 * to the CUs they may use (all CUs on the caller's stream; a quarter of the
 * CUs, capped at 7/8 of those, on the look-ahead's panel stream).  Kernels of
 * other processes or other streams that hold those CUs can delay the panel;
 * its waits are bounded, and when one expires lu_factor returns
 * MXLU_E_TIMEOUT (the factors are then invalid, but every access stays
 * inside A and ipiv).  Look-ahead factorizations of one process are
 * serialised (they share the library's streams).
 */
int mxlu_release(void);

/*
 * mxlu_debug_expire_waits -- test hook, process-wide (0 = off, the default):
 * when on, every panel factorization starts as if one of its bounded waits
 * had already expired, so each wait gives up at its first check and every
 * kernel runs to completion; the call then returns MXLU_E_TIMEOUT.  Lets
 * tests exercise that path without delaying any kernel.  Returns 0, or -1
 * for a value other than 0 or 1.
 */
int mxlu_debug_expire_waits(int on);

/*
 * mxlu_debug_poison_scratch -- test hook, process-wide (-1 = off, the
 * default): when 0..255, every scratch buffer the library allocates for a
 * call is first filled with that byte on the call's stream, so that tests can
 * show that no result depends on what the memory held before (the results
 * with 0x00 and with 0xFF, a NaN pattern, must be the same bit for bit).
 * Returns 0, or -1 for a value outside [-1, 255].
 */
int mxlu_debug_poison_scratch(int byte);

/*
 * lu_solve -- triangular solves with the factors of lu_factor (Sec. III-A.1).
 *   trans = 0: solves A X = B  (apply P, L y = P b, U x = y)
 *   trans = 1: solves A^T X = B (U^T y = b, L^T z = y, x = P^T z)
 *   B      n x nrhs FP64, leading dimension ldb; overwritten by X
 * Fully asynchronous on `stream`.
 */
int lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
             const int32_t *ipiv, double *B, int64_t ldb, int trans,
             void *stream);

/*
 * lu_solve_noalloc -- lu_solve for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the same solves, bit for bit, with no hipMalloc,
 * hipFree or other allocating call.  Its scratch (the row permutation and a
 * strip of up to 16 right-hand sides) lives in a library-owned device array
 * of 8.25 MiB per device (held until the process ends), whose device address
 * is looked up on the first call on each device.  Limit: n <= 65536 (larger
 * n returns MXLU_E_WORKSPACE, nothing enqueued).  Every call on a device
 * shares that device's array: calls that overlap on one device (on different
 * streams or threads) race and must be serialised by the caller.  Arguments,
 * other return values and stream behaviour as lu_solve.
 */
int lu_solve_noalloc(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                     const int32_t *ipiv, double *B, int64_t ldb, int trans,
                     void *stream);

/*
 * mxlu_panel_factor_f64 -- the PFACT phase on its own (Sec. III-A.1: the
 * panel factorization with partial pivoting): GEPP of the m x nb panel P
 * (FP64, column-major, leading dimension ldp, m >= nb, nb <= 1024) in place,
 * with the pivot rules of lu_factor.  ipiv (nb int32, device) receives the
 * interchange sequence, 0-based rows of the panel; every interchange is
 * applied to the whole panel row.  Returns 0, the 1-based first exactly-zero
 * pivot column, -k for an invalid argument, or MXLU_E_*.  Synchronises
 * `stream` once at the end.
 */
int mxlu_panel_factor_f64(int64_t m, int64_t nb, double *P, int64_t ldp, int32_t *ipiv,
                          void *stream);

/*
 * mxlu_schur_update_f64 -- the DGEMM phase on its own (Sec. III-A.1: update
 * of the trailing submatrix): C (M x N) <- C - A (M x K) * B (K x N), FP64,
 * column-major, on the FP64 matrix cores.  Asynchronous on `stream`.
 */
int mxlu_schur_update_f64(int64_t M, int64_t N, int64_t K, const double *A,
                          int64_t lda, const double *B, int64_t ldb, double *C,
                          int64_t ldc, void *stream);

/*
 * mxlu_outer_update_f64 -- C (M x N) <- (accumulate ? C : 0) - A (M x K) B^T,
 * B given as N x K (FP64 matrix cores).  Used for the gradient of a solve
 * with respect to the matrix, dA = -Lambda X^T.  Asynchronous on `stream`.
 */
int mxlu_outer_update_f64(int64_t M, int64_t N, int64_t K, const double *A,
                          int64_t lda, const double *B, int64_t ldb, double *C,
                          int64_t ldc, int accumulate, void *stream);

/* Precision of the mixed-precision factorization. */
enum {
    MXLU_PREC_BF16 = 0,  /* bf16 storage, BF16 MFMA trailing update, FP32 accumulation */
    MXLU_PREC_FP16 = 1,  /* fp16 storage, FP16 MFMA trailing update, FP32 accumulation */
    MXLU_PREC_FP8 = 2,   /* fp16 storage, e4m3fn operands with per-tile power-of-two
                            FP32 scales in the trailing update, FP32 accumulation */
    MXLU_PREC_FP8_MX = 3, /* fp16 storage, e4m3fn operands with one E8M0 (power-of-two)
                            scale per row of L21 / column of U12 and block of 32 k,
                            applied by the matrix cores (OCP MX block scaling);
                            FP32 accumulation; scale_tile unused */
    MXLU_PREC_FP32 = 4    /* fp32 storage (4 bytes per factor value), FP32 panel, TRSM and
                            trailing update (vector fused multiply-adds, k ascending);
                            forward solves only (trans must be 0) */
};
enum { MXLU_IR_CLASSICAL = 0, MXLU_IR_GMRES = 1 };

typedef struct {
    int32_t prec;            /* MXLU_PREC_* */
    int32_t pivot;           /* 0: no pivoting (Sec. III-A.2); 1: partial pivoting on FP32 values */
    int64_t nb;              /* panel width */
    int32_t refine;          /* MXLU_IR_CLASSICAL or MXLU_IR_GMRES */
    int32_t restart;         /* GMRES cycle length m */
    int32_t max_outer;       /* refinement steps */
    int32_t max_inner_total; /* GMRES Arnoldi steps over all cycles */
    double inner_tol;        /* GMRES: stop a cycle when the estimate <= inner_tol * beta */
    double resid_threshold;  /* stop when the HPL scaled residual < this (16) */
    int32_t scale_tile;      /* FP8: rows (cols) per scale tile of L21 (U12); a multiple of 4, <= 256 */
    int32_t reuse_factors;   /* 1: the factors in `work` come from an earlier call
                                with the same A, n, opts: skip conversion and LU */
    int32_t trans;           /* 0: solve A X = B; 1: solve A^T X = B */
    int32_t x_init;          /* 0: x0 = M b; 1: X holds the initial guess */
    int32_t factor_steps;    /* > 0: stop the factorization after this many panel
                                steps, leaving the trailing block updated but
                                unfactored (a partial LU whose trailing block is
                                the Schur complement); 0: factor completely */
} mxp_opts;

typedef struct {
    int32_t converged;       /* 1 when every column reached resid_threshold */
    int32_t outer_iters;     /* refinement steps, summed over the columns */
    int32_t inner_iters;     /* GMRES Arnoldi steps, summed over the columns */
    int32_t info;            /* > 0: first exactly-zero pivot column (1-based) */
    double scaled_residual;  /* largest final HPL scaled residual over the columns */
    double t_convert_ms, t_factor_ms, t_refine_ms;  /* event-timed phases */
} mxp_report;

/* Fill *opts with the defaults: BF16, no pivoting, nb 512, GMRES, restart 30,
 * max_outer 20, max_inner_total 300, inner_tol 1e-6, threshold 16, tile 128,
 * complete factorization. */
void mxp_default_opts(mxp_opts *opts);

/* Bytes of caller workspace mxp_solve needs for order n with the FP64 matrix
 * at leading dimension lda (>= n), or 0 when an argument is invalid or the
 * size overflows.  The workspace starts with the low-precision factors: an n x n
 * column-major array of 16-bit words (bf16 for MXLU_PREC_BF16, fp16 for the
 * FP16 and FP8 precisions) or of FP32 values (MXLU_PREC_FP32) with leading
 * dimension mxp_factor_ld(n), holding L (unit lower, below the diagonal) and U
 * (upper), as lu_factor does in FP64. */
size_t mxp_workspace_bytes(int64_t n, int64_t lda, const mxp_opts *opts);
int64_t mxp_factor_ld(int64_t n);

/*
 * mxp_convert -- the down-conversion step alone (Sec. III-A.2: the matrix is
 * stored in reduced precision): F (rows x cols, 16-bit words, leading
 * dimension ldf) <- A (FP64) rounded to nearest, ties to even, directly from
 * FP64.  prec: MXLU_PREC_BF16 -> bf16, MXLU_PREC_FP16 / FP8 / FP8_MX -> fp16
 * (MXLU_PREC_FP32 is not a 16-bit format: -1).  Asynchronous.
 */
int mxp_convert(int32_t prec, int64_t rows, int64_t cols, const double *A, int64_t lda,
                uint16_t *F, int64_t ldf, void *stream);

/*
 * mxp_solve -- mixed-precision solve (Sec. III-A.2, Sec. II-B).
 *   A      n x n FP64 (unmodified; used for the FP64 residuals)
 *   B      n x nrhs FP64 right-hand sides (unmodified)
 *   X      n x nrhs FP64 solution (in: initial guess when opts->x_init = 1)
 *   work   caller workspace of >= mxp_workspace_bytes(n, opts) bytes; holds
 *          the low-precision factors on return (reusable, see reuse_factors)
 *   ipiv   n int32 when opts->pivot = 1 (written unless reuse_factors), else NULL
 *   report filled on return (host struct), may be NULL
 * Steps: convert A to the storage precision (round to nearest even from
 * FP64); blocked LU in low precision; x0 = M b with M = U^-1 L^-1 P applied in
 * FP32; then refinement with FP64 residuals r = b - A x until the HPL scaled
 * residual ||r||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n), eps = 2^-53,
 * drops below opts->resid_threshold: classical (x += M r) or GMRES-IR.
 * Returns MXLU_E_NOTCONV when a column does not converge (X holds the last
 * iterate, report is filled).  Synchronises `stream` once per refinement step.
 */
int mxp_solve(int64_t n, int64_t nrhs, const double *A, int64_t lda,
              const double *B, int64_t ldb, double *X, int64_t ldx,
              void *work, size_t work_bytes, int32_t *ipiv,
              const mxp_opts *opts, mxp_report *report, void *stream);

/*
 * mxp_solve_seeded -- mxp_solve for the seeded synthetic matrix, regenerated
 * wherever it is needed instead of being stored (Sec. II-B names scalable
 * generation of the input matrix among what HPL-MxP asks for): the
 * conversion to the storage precision and every FP64 residual r = b - op(A) x
 * compute a_ij from its counter, so no n x n FP64 array exists (at
 * n = 131072 that is 128 GiB of HBM not needed).  The matrix is the one
 * mxlu_fill_uniform(n, n, ., seed, stream_id) writes, and with dominant = 1
 * the one mxlu_make_diag_dominant then makes (its diagonal, the sums of the
 * rows' absolute off-diagonal values, is computed first by one pass over the
 * regenerated entries into n doubles of internal scratch).  Arguments from
 * nrhs on, results and the order of every floating-point operation are those
 * of mxp_solve on that matrix (the two give the same bits); work_bytes as
 * mxp_workspace_bytes(n, n, opts).  Returns as mxp_solve (-k for the k-th
 * argument of this signature).
 */
int mxp_solve_seeded(int64_t n, uint64_t seed, uint64_t stream_id, int dominant, int64_t nrhs,
                     const double *B, int64_t ldb, double *X, int64_t ldx, void *work,
                     size_t work_bytes, int32_t *ipiv, const mxp_opts *opts, mxp_report *report,
                     void *stream);

/*
 * Seeded synthetic inputs (not part of the method).  Element (i, j) of a
 * rows x cols matrix is u(j*rows + i) with the counter-based generator
 *   mix(z) = SplitMix64 finaliser, key = mix(seed + G (stream_id + 1)),
 *   u(idx) = (mix(key + G (idx + 1)) >> 32) * 2^-32 - 0.5,  G = 0x9E3779B97F4A7C15.
 * mxlu_make_diag_dominant replaces each diagonal entry of A by the sum of
 * the absolute values of the other entries of its row (exact in FP64 for
 * generator values).
 */
int mxlu_fill_uniform(int64_t rows, int64_t cols, double *A, int64_t lda,
                      uint64_t seed, uint64_t stream_id, void *stream);
int mxlu_make_diag_dominant(int64_t n, double *A, int64_t lda, void *stream);

/*
 * mxlu_scaled_residual -- verification in FP64 on the device (not timed):
 * for each column c of X, R(:,c) = B(:,c) - op(A) X(:,c) and
 * out[c] = ||R(:,c)||_inf / (eps (||op(A)||_inf ||X(:,c)||_inf + ||B(:,c)||_inf) n)
 * with eps = 2^-53; op(A) = A (trans 0) or A^T (trans 1).  out is a HOST
 * array of nrhs doubles; synchronises `stream`.
 */
int mxlu_scaled_residual(int64_t n, int64_t nrhs, const double *A, int64_t lda,
                         const double *X, int64_t ldx, const double *B,
                         int64_t ldb, int trans, double *out, void *stream);

/*
 * Instrumentation (not part of the method): per-phase GPU time measured with
 * HIP events on the caller's stream.  Phases: 0 PFACT, 1 SWAP, 2 DTRSM,
 * 3 DGEMM trailing update, 4 solve, 5 conversion, 6 low-precision LU,
 * 7 refinement, 8 low-precision trailing update.  mxlu_profile_read
 * synchronises on the recorded events and returns, per phase, the summed
 * milliseconds, the summed nominal work (flops for DGEMM: 2 M N K per launch;
 * bytes for phase 8: 4 M N + operand bytes) and the number of intervals;
 * arrays are HOST arrays of `nphase` entries (any may be NULL).
 */
int mxlu_profile_enable(int on);
int mxlu_profile_reset(void);
int mxlu_profile_read(double *ms, double *work, int64_t *count, int nphase);
/*
 * mxlu_profile_intervals -- the individual intervals of one phase since the
 * last reset, in recording order: step[k] is the panel step the interval
 * belongs to (k0 / nb of the factorization; -1 outside a factorization),
 * ms[k] its GPU time, work[k] its nominal work.  Fills at most `cap` entries
 * of the HOST arrays (any may be NULL) and returns the number of intervals,
 * or < 0 on error.  Synchronises on the recorded events.
 */
int64_t mxlu_profile_intervals(int phase, int64_t *step, double *ms, double *work, int64_t cap);

/*
 * Planning helpers: host arithmetic only (no device access), the rules the
 * library applies with the current device's facts; exposed for tests.
 *   mxlu_plan_panel_cus: CUs given to the look-ahead's panel stream on a
 *     device with `cus` CUs: cus / 4 when that is a multiple of 32 (an equal
 *     number in every shader engine of an 8-XCD, 4-engine-per-XCD part),
 *     else 0 (no look-ahead).
 *   mxlu_plan_panel_leaf: form of the panel leaf for m rows when at most
 *     `cap` CUs may hold it (0: all `cus`), with occ_reg1 / occ_reg2
 *     workgroups per CU for the register forms (0: not available),
 *     lds_budget bytes of dynamic LDS for the LDS form and elements of
 *     elem_bytes (4 or 8; the register forms are FP64 only).  Returns
 *     1 or 2 (register form, rows per thread), 3 (LDS form), 0 (no form
 *     fits: the call would fail with MXLU_E_NOMEM), -1 (bad argument);
 *     *rows_per_group and *groups receive the geometry.
 *   mxlu_plan_lookahead: CUs of the panel stream when lu_factor(n, nb) runs
 *     look-ahead depth 1 on such a device (given 16-byte aligned A and even
 *     lda), else 0.
 */
int mxlu_plan_panel_cus(int cus);
int mxlu_plan_panel_leaf(int64_t m, int cap, int cus, int occ_reg1, int occ_reg2,
                         int64_t lds_budget, int elem_bytes, int64_t *rows_per_group,
                         int64_t *groups);
int mxlu_plan_lookahead(int64_t n, int64_t nb, int cus, int occ_reg1, int occ_reg2,
                        int64_t lds_budget);

/* Static description of a status code. */
const char *mxlu_status_string(int status);
/* Detail of the last runtime failure on the calling thread ("" if none). */
const char *mxlu_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MXLU_H */
