/*
 * mxlu_oracle.c -- CPU reference ("oracle") for the dense LU solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the bench's CPU-baseline leg
 * do.  It shares no code with the HIP library.
 *
 * Plain, slow, obviously correct C in FP64 (FP32 where the mixed-precision
 * method fixes FP32 arithmetic).  No BLAS.  Every multiply-add is an explicit
 * fma()/fmaf() so that the rounding is a stated property of the code, and the
 * file is compiled with -ffp-contract=off so the compiler adds no others.
 *
 * What is computed (Sec. III-A.1 of the paper: Gaussian elimination with
 * row partial pivoting, then the two triangular solves with the factors; the
 * phases PFACT, SWAP, DTRSM, DGEMM of the right-looking blocked algorithm;
 * Sec. III-A.2 for the
 * mixed-precision variant: low-precision factorization and trailing updates,
 * no pivoting, FP64 residuals and corrections):
 *
 *   oracle_getrf      blocked right-looking GEPP, panel width nb
 *   oracle_getrf_gaps the same, with the relative gap of every pivot search
 *   oracle_getrs      solve with the factors, A x = b or A^T x = b
 *   oracle_round      round an FP64 value to bf16 / fp16 / e4m3fn (RNE)
 *   oracle_lp_getrf   low-precision blocked LU (storage in bf16 or fp16,
 *                     all steps, or the first max_steps: oracle_lp_getrf_steps,
 *                     FP32 panel/TRSM, BF16/FP16 or FP8-with-tile-scales
 *                     trailing update), with or without partial pivoting
 *   oracle_lp_precond apply M = U^-1 L^-1 P (or its transpose) in FP32
 *
 * Conventions (LAPACK getrf/getrs): column-major, leading dimension lda,
 * ipiv is the interchange sequence, 0-based: row j was swapped with row
 * ipiv[j] >= j at step j.  Return value of a factorization: 0, or the 1-based
 * index of the first column whose pivot is exactly zero.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------ */
/* FP64 blocked GEPP                                                         */
/* ------------------------------------------------------------------------ */

/* Swap rows r1 and r2 of A over columns [c0, c1). */
static void swap_rows(double *A, int64_t lda, int64_t r1, int64_t r2,
                      int64_t c0, int64_t c1)
{
    if (r1 == r2) return;
    for (int64_t c = c0; c < c1; ++c) {
        double t = A[IDX(r1, c, lda)];
        A[IDX(r1, c, lda)] = A[IDX(r2, c, lda)];
        A[IDX(r2, c, lda)] = t;
    }
}

/*
 * PFACT: unblocked GEPP of the panel A[k0:n, k0:k0+kb] (getf2).  For each
 * column j: pivot = first row i >= j maximising |A[i,j]| (ties -> smaller i);
 * swap rows j and pivot inside the panel; divide the column below the
 * diagonal by the pivot; rank-1 update of the panel columns to the right.
 * An exactly zero pivot column is left unscaled and recorded in *info.
 */
static void panel_getf2(int64_t n, int64_t k0, int64_t kb, double *A,
                        int64_t lda, int32_t *ipiv, int *info, double *gaps)
{
    for (int64_t j = k0; j < k0 + kb; ++j) {
        int64_t p = j;
        double best = fabs(A[IDX(j, j, lda)]);
        for (int64_t i = j + 1; i < n; ++i) {
            double v = fabs(A[IDX(i, j, lda)]);
            if (v > best) { best = v; p = i; }
        }
        if (gaps) {   /* relative gap to the runner-up candidate */
            double second = -1.0;
            for (int64_t i = j; i < n; ++i) {
                double v = fabs(A[IDX(i, j, lda)]);
                if (i != p && v > second) second = v;
            }
            gaps[j] = (second < 0.0) ? 1.0
                    : (best > 0.0 ? (best - second) / best : 0.0);
        }
        ipiv[j] = (int32_t)p;
        if (A[IDX(p, j, lda)] != 0.0) {
            swap_rows(A, lda, j, p, k0, k0 + kb);
            double piv = A[IDX(j, j, lda)];
            for (int64_t i = j + 1; i < n; ++i)
                A[IDX(i, j, lda)] = A[IDX(i, j, lda)] / piv;
        } else if (*info == 0) {
            *info = (int)(j + 1);
        }
        /* rank-1 update of columns j+1 .. k0+kb-1 of the panel */
        #pragma omp parallel for schedule(static) if ((n - j) * (k0 + kb - j) > 65536)
        for (int64_t c = j + 1; c < k0 + kb; ++c) {
            double u = A[IDX(j, c, lda)];
            for (int64_t i = j + 1; i < n; ++i)
                A[IDX(i, c, lda)] = fma(-A[IDX(i, j, lda)], u, A[IDX(i, c, lda)]);
        }
    }
}

/*
 * One step of the right-looking blocked algorithm at column k0 with panel
 * width kb: PFACT, SWAP on the columns outside the panel, DTRSM for the block
 * row U12 = L11^-1 A12 (forward substitution, unit lower), and the trailing
 * DGEMM A22 -= L21 U12 with the k index summed in ascending order.
 * gaps (optional) receives the pivot searches' relative gaps (panel_getf2).
 */
static void getrf_step(int64_t n, int64_t k0, int64_t kb, double *A,
                       int64_t lda, int32_t *ipiv, int *info, double *gaps)
{
    panel_getf2(n, k0, kb, A, lda, ipiv, info, gaps);

    /* SWAP: apply this panel's interchanges, in order, to the other columns */
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        if (c >= k0 && c < k0 + kb) continue;
        for (int64_t j = k0; j < k0 + kb; ++j) {
            int64_t p = ipiv[j];
            if (p != j) {
                double t = A[IDX(j, c, lda)];
                A[IDX(j, c, lda)] = A[IDX(p, c, lda)];
                A[IDX(p, c, lda)] = t;
            }
        }
    }

    int64_t c1 = k0 + kb;
    /* DTRSM: U12 = L11^-1 A12, column by column */
    #pragma omp parallel for schedule(static)
    for (int64_t c = c1; c < n; ++c) {
        for (int64_t k = k0; k < c1; ++k) {
            double x = A[IDX(k, c, lda)];
            for (int64_t i = k + 1; i < c1; ++i)
                A[IDX(i, c, lda)] = fma(-A[IDX(i, k, lda)], x, A[IDX(i, c, lda)]);
        }
    }

    /* DGEMM: A22 -= L21 * U12 */
    #pragma omp parallel for schedule(static)
    for (int64_t c = c1; c < n; ++c) {
        for (int64_t k = k0; k < c1; ++k) {
            double u = A[IDX(k, c, lda)];
            for (int64_t i = c1; i < n; ++i)
                A[IDX(i, c, lda)] = fma(-A[IDX(i, k, lda)], u, A[IDX(i, c, lda)]);
        }
    }
}

/*
 * Blocked GEPP of the n x n matrix A (overwritten by L\U).  Runs the first
 * `max_steps` panel steps only when max_steps >= 0 (used to time a bounded
 * sample of a large factorization); max_steps < 0 runs them all.
 */
static int getrf_blocked(int64_t n, int64_t nb, double *A, int64_t lda,
                         int32_t *ipiv, int64_t max_steps, double *gaps)
{
    if (n < 0 || nb < 1 || lda < (n > 1 ? n : 1)) return -1;
    int info = 0;
    int64_t step = 0;
    for (int64_t k0 = 0; k0 < n; k0 += nb, ++step) {
        if (max_steps >= 0 && step >= max_steps) break;
        int64_t kb = (n - k0 < nb) ? (n - k0) : nb;
        getrf_step(n, k0, kb, A, lda, ipiv, &info, gaps);
    }
    return info;
}

int oracle_getrf_steps(int64_t n, int64_t nb, double *A, int64_t lda,
                       int32_t *ipiv, int64_t max_steps)
{
    return getrf_blocked(n, nb, A, lda, ipiv, max_steps, NULL);
}

/*
 * The same factorization, also reporting for every column j the relative gap
 * between the two largest candidate magnitudes of its pivot search,
 * gaps[j] = (|a_pj| - max_{i >= j, i != p} |a_ij|) / |a_pj| (1 for a single
 * candidate, 0 for a zero column).  A tiny gap marks a column where another
 * rounding order may legally pick the other row; the pivot comparison uses it
 * at sizes where re-running the oracle per mismatch is too slow.
 */
int oracle_getrf_gaps(int64_t n, int64_t nb, double *A, int64_t lda,
                      int32_t *ipiv, double *gaps)
{
    if (!gaps) return -6;
    return getrf_blocked(n, nb, A, lda, ipiv, -1, gaps);
}

/* Threads the OpenMP loops of this file use. */
int oracle_threads(void) { return omp_get_max_threads(); }

int oracle_getrf(int64_t n, int64_t nb, double *A, int64_t lda, int32_t *ipiv)
{
    return oracle_getrf_steps(n, nb, A, lda, ipiv, -1);
}

/*
 * PFACT of the leading panel alone: unblocked GEPP of an m x kb panel (the
 * first step of the blocked algorithm only reads these columns, so its pivots
 * and L\U panel are those of the full factorization's first step).
 */
int oracle_panel_getf2(int64_t m, int64_t kb, double *A, int64_t lda, int32_t *ipiv)
{
    if (m < 0 || kb < 0 || kb > m || lda < (m > 1 ? m : 1)) return -1;
    int info = 0;
    panel_getf2(m, 0, kb, A, lda, ipiv, &info, NULL);
    return info;
}

/*
 * Solve with the factors of oracle_getrf.  trans = 0: A X = B, i.e. apply the
 * interchanges to B in order, forward substitution with unit-lower L, back
 * substitution with U (true division).  trans = 1: A^T X = B, i.e. U^T y = b
 * (forward), L^T z = y (backward), then the interchanges in reverse order.
 * B (n x nrhs, leading dimension ldb) is overwritten with X.
 */
int oracle_getrs(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                 const int32_t *ipiv, double *B, int64_t ldb, int trans)
{
    if (n < 0 || nrhs < 0 || lda < (n > 1 ? n : 1) || ldb < (n > 1 ? n : 1))
        return -1;
    if (trans != 0 && trans != 1) return -8;
    #pragma omp parallel for schedule(static) if (nrhs > 1)
    for (int64_t r = 0; r < nrhs; ++r) {
        double *b = B + (size_t)r * (size_t)ldb;
        if (trans == 0) {
            for (int64_t j = 0; j < n; ++j) {
                int64_t p = ipiv[j];
                if (p != j) { double t = b[j]; b[j] = b[p]; b[p] = t; }
            }
            for (int64_t k = 0; k < n; ++k) {          /* L y = P b */
                double x = b[k];
                for (int64_t i = k + 1; i < n; ++i)
                    b[i] = fma(-LU[IDX(i, k, lda)], x, b[i]);
            }
            for (int64_t k = n - 1; k >= 0; --k) {     /* U x = y */
                b[k] = b[k] / LU[IDX(k, k, lda)];
                double x = b[k];
                for (int64_t i = 0; i < k; ++i)
                    b[i] = fma(-LU[IDX(i, k, lda)], x, b[i]);
            }
        } else {
            for (int64_t k = 0; k < n; ++k) {          /* U^T y = b */
                double acc = b[k];
                for (int64_t i = 0; i < k; ++i)
                    acc = fma(-LU[IDX(i, k, lda)], b[i], acc);
                b[k] = acc / LU[IDX(k, k, lda)];
            }
            for (int64_t k = n - 1; k >= 0; --k) {     /* L^T z = y */
                double acc = b[k];
                for (int64_t i = k + 1; i < n; ++i)
                    acc = fma(-LU[IDX(i, k, lda)], b[i], acc);
                b[k] = acc;
            }
            for (int64_t j = n - 1; j >= 0; --j) {     /* x = P^T z */
                int64_t p = ipiv[j];
                if (p != j) { double t = b[j]; b[j] = b[p]; b[p] = t; }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Low-precision formats, written from their definitions                     */
/* ------------------------------------------------------------------------ */
/*
 * A binary floating-point format with p significand bits (implicit bit
 * included) and minimum normal exponent emin holds, for |x| in
 * [2^E, 2^(E+1)) with E >= emin, the multiples of 2^(E-p+1); below 2^emin
 * (subnormals) the multiples of 2^(emin-p+1).  Round to nearest, ties to even,
 * directly from the FP64 value (no intermediate FP32 rounding):
 *
 *   bf16    p = 8,  emin = -126, largest finite (2 - 2^-7) 2^127, then inf
 *   fp16    p = 11, emin = -14,  largest finite 65504, then inf
 *   e4m3fn  p = 4,  emin = -6,   largest finite 448, no inf (OCP FP8 spec):
 *           conversions saturate to +-448.
 */
enum { ORACLE_BF16 = 0, ORACLE_FP16 = 1, ORACLE_E4M3 = 2, ORACLE_FP32 = 3 };

double oracle_round(double x, int fmt)
{
    int p, emin;
    double maxfin;
    int saturate;
    switch (fmt) {
    case ORACLE_BF16: p = 8;  emin = -126; maxfin = ldexp(2.0 - ldexp(1.0, -7), 127); saturate = 0; break;
    case ORACLE_FP16: p = 11; emin = -14;  maxfin = 65504.0; saturate = 0; break;
    case ORACLE_E4M3: p = 4;  emin = -6;   maxfin = 448.0;   saturate = 1; break;
    case ORACLE_FP32: p = 24; emin = -126; maxfin = ldexp(2.0 - ldexp(1.0, -23), 127); saturate = 0; break;
    default: return NAN;
    }
    if (x != x || x == 0.0) return x;
    if (isinf(x)) return saturate ? copysign(maxfin, x) : x;
    int e2;
    (void)frexp(x, &e2);            /* |x| = f 2^e2, f in [0.5, 1) */
    int E = e2 - 1;                 /* |x| in [2^E, 2^(E+1)) */
    if (E < emin) E = emin;
    double q = ldexp(1.0, E - (p - 1));      /* spacing of the format there */
    double y = nearbyint(x / q) * q;         /* default mode: ties to even */
    if (fabs(y) > maxfin) {
        if (saturate) return copysign(maxfin, x);
        return copysign(INFINITY, x);
    }
    return y;
}

void oracle_round_array(int64_t count, const double *in, double *out, int fmt)
{
    for (int64_t t = 0; t < count; ++t) out[t] = oracle_round(in[t], fmt);
}

/*
 * Power-of-two scale for a tile with largest magnitude amax: the smallest
 * s = 2^k with amax / s <= 448 (the e4m3fn maximum); s = 1 for an all-zero
 * tile.  A power of two keeps the scaling and the unscaling exact.
 */
double oracle_fp8_scale(double amax)
{
    if (!(amax > 0.0)) return 1.0;
    int e2;
    double f = frexp(amax / 448.0, &e2);     /* amax/448 = f 2^e2, f in [0.5,1) */
    /* ceil(log2(amax/448)) is e2 when f > 0.5, e2-1 when amax/448 is a power of 2 */
    int k = (f == 0.5) ? e2 - 1 : e2;
    return ldexp(1.0, k);
}

/*
 * E8M0 block scale of the MX form: the smallest power of two 2^e with
 * amax / 2^e <= 448 (as oracle_fp8_scale), e limited to the E8M0 exponent
 * range [-127, 127]; 1 for an all-zero block.
 */
double oracle_mx_scale(double amax)
{
    if (!(amax > 0.0)) return 1.0;
    int e2;
    double f = frexp(amax / 448.0, &e2);
    int k = (f == 0.5) ? e2 - 1 : e2;
    if (k < -127) k = -127;
    if (k > 127) k = 127;
    return ldexp(1.0, k);
}

/* ------------------------------------------------------------------------ */
/* Low-precision LU (the mixed-precision variant)                            */
/* ------------------------------------------------------------------------ */
/*
 * Storage S holds, as FP64 numbers, values representable in the storage
 * format (bf16 for prec 0, fp16 for prec 1, 2 and 3, FP32 for prec 4).  prec 2 keeps fp16 storage
 * but performs the trailing update with e4m3fn operands and FP32 tile scales.
 *
 * Step at column k0 with width kb (m = n - k0 rows):
 *   PFACT (FP32): the m x kb panel read from S into FP32 and factored by
 *     getf2 in FP32 (fmaf updates, true division); with pivot = 1 the pivot
 *     search compares the FP32 values; the panel is stored back rounded.
 *   SWAP (pivot = 1): interchanges applied to the stored other columns.
 *   TRSM (FP32): U12 = L11^-1 A12 with the unrounded FP32 L11 of the panel,
 *     forward substitution in ascending order, stored rounded.
 *   Update: A22 <- round_s( fp32(A22) - L21 U12 ), operands as stored.
 *     prec 0/1: accumulation in FP32 from fp32(A22), k ascending (fmaf).
 *     prec 2:   L21 quantised per tile of `tile` rows x kb, U12 per tile of
 *               kb x `tile` columns, to e4m3fn with power-of-two scales;
 *               acc = sum_k Lq Uq in FP32 (k ascending, from 0);
 *               A22 <- round_fp16( fp32(A22) - (acc * sL) * sU ).
 *     prec 4:   FP32 storage (IEEE binary32): every rounding to storage is
 *               a rounding to FP32, the update as for prec 0/1.
 *     prec 3:   MX form: each row of L21 and column of U12 quantised in
 *               blocks of 32 k with one E8M0 scale per block;
 *               acc = sum_k (Lq sL)(Uq sU) in FP32 (k ascending, from 0);
 *               A22 <- round_fp16( fp32(A22) - acc ).
 */
static float to_f32(double v) { return (float)v; }   /* exact for stored values */

int oracle_lp_getrf_steps(int64_t n, int64_t nb, int prec, int pivot, int64_t tile,
                          double *S, int64_t lds, int32_t *ipiv, int64_t max_steps)
{
    if (n < 0 || nb < 1 || lds < (n > 1 ? n : 1)) return -1;
    if (prec < 0 || prec > 4 || tile < 1) return -3;
    int sfmt = (prec == 0) ? ORACLE_BF16 : (prec == 4) ? ORACLE_FP32 : ORACLE_FP16;
    int info = 0;

    /* storage conversion of the input */
    for (int64_t c = 0; c < n; ++c)
        for (int64_t i = 0; i < n; ++i)
            S[IDX(i, c, lds)] = oracle_round(S[IDX(i, c, lds)], sfmt);

    float *P = (float *)malloc(sizeof(float) * (size_t)n * (size_t)nb);
    float *Lq = NULL, *Uq = NULL;
    double *sL = NULL, *sU = NULL;
    const int fp8 = (prec == 2 || prec == 3);
    if (fp8) {
        /* prec 2: one scale per tile; prec 3: one per (line, block of 32 k) */
        size_t ns = (prec == 2) ? (size_t)(n / tile + 1)
                                : (size_t)n * (size_t)((nb + 31) / 32);
        Lq = (float *)malloc(sizeof(float) * (size_t)n * (size_t)nb);
        Uq = (float *)malloc(sizeof(float) * (size_t)n * (size_t)nb);
        sL = (double *)malloc(sizeof(double) * ns);
        sU = (double *)malloc(sizeof(double) * ns);
    }
    if (!P || (fp8 && (!Lq || !Uq || !sL || !sU))) {
        free(P); free(Lq); free(Uq); free(sL); free(sU);
        return -1000;
    }

    int64_t step = 0;
    for (int64_t k0 = 0; k0 < n; k0 += nb, ++step) {
        if (max_steps >= 0 && step >= max_steps) break;
        int64_t kb = (n - k0 < nb) ? (n - k0) : nb;
        int64_t m = n - k0;
        /* PFACT in FP32; P is the m x kb panel, leading dimension m */
        for (int64_t c = 0; c < kb; ++c)
            for (int64_t i = 0; i < m; ++i)
                P[IDX(i, c, m)] = to_f32(S[IDX(k0 + i, k0 + c, lds)]);
        for (int64_t j = 0; j < kb; ++j) {
            int64_t p = j;
            if (pivot) {
                float best = fabsf(P[IDX(j, j, m)]);
                for (int64_t i = j + 1; i < m; ++i) {
                    float v = fabsf(P[IDX(i, j, m)]);
                    if (v > best) { best = v; p = i; }
                }
                ipiv[k0 + j] = (int32_t)(k0 + p);
            } else if (ipiv) {
                ipiv[k0 + j] = (int32_t)(k0 + j);
            }
            if (P[IDX(p, j, m)] != 0.0f) {
                if (p != j)
                    for (int64_t c = 0; c < kb; ++c) {
                        float t = P[IDX(j, c, m)];
                        P[IDX(j, c, m)] = P[IDX(p, c, m)];
                        P[IDX(p, c, m)] = t;
                    }
                float piv = P[IDX(j, j, m)];
                for (int64_t i = j + 1; i < m; ++i)
                    P[IDX(i, j, m)] = P[IDX(i, j, m)] / piv;
            } else if (info == 0) {
                info = (int)(k0 + j + 1);
            }
            for (int64_t c = j + 1; c < kb; ++c) {
                float u = P[IDX(j, c, m)];
                for (int64_t i = j + 1; i < m; ++i)
                    P[IDX(i, c, m)] = fmaf(-P[IDX(i, j, m)], u, P[IDX(i, c, m)]);
            }
        }
        for (int64_t c = 0; c < kb; ++c)
            for (int64_t i = 0; i < m; ++i)
                S[IDX(k0 + i, k0 + c, lds)] = oracle_round((double)P[IDX(i, c, m)], sfmt);
        /* SWAP on the other stored columns */
        if (pivot) {
            for (int64_t j = k0; j < k0 + kb; ++j) {
                int64_t p = ipiv[j];
                if (p == j) continue;
                for (int64_t c = 0; c < n; ++c) {
                    if (c >= k0 && c < k0 + kb) continue;
                    double t = S[IDX(j, c, lds)];
                    S[IDX(j, c, lds)] = S[IDX(p, c, lds)];
                    S[IDX(p, c, lds)] = t;
                }
            }
        }
        int64_t c1 = k0 + kb;
        /* TRSM in FP32 with the unrounded L11 */
        #pragma omp parallel for schedule(static)
        for (int64_t c = c1; c < n; ++c) {
            float u[4096];
            float *uu = (kb <= 4096) ? u : (float *)malloc(sizeof(float) * (size_t)kb);
            for (int64_t k = 0; k < kb; ++k) uu[k] = to_f32(S[IDX(k0 + k, c, lds)]);
            for (int64_t k = 0; k < kb; ++k)
                for (int64_t i = k + 1; i < kb; ++i)
                    uu[i] = fmaf(-P[IDX(i, k, m)], uu[k], uu[i]);
            for (int64_t k = 0; k < kb; ++k)
                S[IDX(k0 + k, c, lds)] = oracle_round((double)uu[k], sfmt);
            if (uu != u) free(uu);
        }
        if (c1 >= n) continue;
        /* trailing update from the stored operands */
        if (prec == 3) {
            /* MX form: every row of L21 and every column of U12 quantised in
               blocks of 32 consecutive k (aligned to the panel) with one
               E8M0 (power-of-two) scale per block; the update sums the
               exactly rescaled products (Lq sL)(Uq sU) in FP32, k ascending
               from zero, and subtracts the sum from fp32(A22) */
            int64_t mt = n - c1, nblk = (kb + 31) / 32;
            for (int64_t i = c1; i < n; ++i)
                for (int64_t b = 0; b < nblk; ++b) {
                    int64_t ka = 32 * b, kz = (ka + 32 < kb) ? ka + 32 : kb;
                    double amax = 0.0;
                    for (int64_t k = ka; k < kz; ++k) {
                        double v = fabs(S[IDX(i, k0 + k, lds)]);
                        if (v > amax) amax = v;
                    }
                    double sc = oracle_mx_scale(amax);
                    sL[(i - c1) * nblk + b] = sc;
                    for (int64_t k = ka; k < kz; ++k)
                        Lq[IDX(i - c1, k, mt)] = (float)oracle_round(
                            S[IDX(i, k0 + k, lds)] / sc, ORACLE_E4M3);
                }
            for (int64_t c = c1; c < n; ++c)
                for (int64_t b = 0; b < nblk; ++b) {
                    int64_t ka = 32 * b, kz = (ka + 32 < kb) ? ka + 32 : kb;
                    double amax = 0.0;
                    for (int64_t k = ka; k < kz; ++k) {
                        double v = fabs(S[IDX(k0 + k, c, lds)]);
                        if (v > amax) amax = v;
                    }
                    double sc = oracle_mx_scale(amax);
                    sU[(c - c1) * nblk + b] = sc;
                    for (int64_t k = ka; k < kz; ++k)
                        Uq[IDX(k, c - c1, kb)] = (float)oracle_round(
                            S[IDX(k0 + k, c, lds)] / sc, ORACLE_E4M3);
                }
            #pragma omp parallel for schedule(static)
            for (int64_t c = c1; c < n; ++c) {
                for (int64_t i = c1; i < n; ++i) {
                    float acc = 0.0f;
                    for (int64_t k = 0; k < kb; ++k) {
                        float l = (float)((double)Lq[IDX(i - c1, k, mt)] *
                                          sL[(i - c1) * nblk + k / 32]);   /* exact */
                        float u = (float)((double)Uq[IDX(k, c - c1, kb)] *
                                          sU[(c - c1) * nblk + k / 32]);   /* exact */
                        acc = fmaf(l, u, acc);
                    }
                    float a = to_f32(S[IDX(i, c, lds)]) - acc;
                    S[IDX(i, c, lds)] = oracle_round((double)a, ORACLE_FP16);
                }
            }
        } else if (prec != 2) {
            #pragma omp parallel for schedule(static)
            for (int64_t c = c1; c < n; ++c) {
                for (int64_t i = c1; i < n; ++i) {
                    float acc = to_f32(S[IDX(i, c, lds)]);
                    for (int64_t k = 0; k < kb; ++k)
                        acc = fmaf(-to_f32(S[IDX(i, k0 + k, lds)]),
                                   to_f32(S[IDX(k0 + k, c, lds)]), acc);
                    S[IDX(i, c, lds)] = oracle_round((double)acc, sfmt);
                }
            }
        } else {
            int64_t mt = n - c1;                 /* rows / cols of A22 */
            int64_t ntile = (mt + tile - 1) / tile;
            for (int64_t t = 0; t < ntile; ++t) {        /* L21 row tiles */
                int64_t r0 = c1 + t * tile, r1 = r0 + tile < n ? r0 + tile : n;
                double amax = 0.0;
                for (int64_t k = 0; k < kb; ++k)
                    for (int64_t i = r0; i < r1; ++i) {
                        double v = fabs(S[IDX(i, k0 + k, lds)]);
                        if (v > amax) amax = v;
                    }
                sL[t] = oracle_fp8_scale(amax);
                for (int64_t k = 0; k < kb; ++k)
                    for (int64_t i = r0; i < r1; ++i)
                        Lq[IDX(i - c1, k, mt)] = (float)oracle_round(
                            S[IDX(i, k0 + k, lds)] / sL[t], ORACLE_E4M3);
            }
            for (int64_t t = 0; t < ntile; ++t) {        /* U12 column tiles */
                int64_t q0 = c1 + t * tile, q1 = q0 + tile < n ? q0 + tile : n;
                double amax = 0.0;
                for (int64_t c = q0; c < q1; ++c)
                    for (int64_t k = 0; k < kb; ++k) {
                        double v = fabs(S[IDX(k0 + k, c, lds)]);
                        if (v > amax) amax = v;
                    }
                sU[t] = oracle_fp8_scale(amax);
                for (int64_t c = q0; c < q1; ++c)
                    for (int64_t k = 0; k < kb; ++k)
                        Uq[IDX(k, c - c1, kb)] = (float)oracle_round(
                            S[IDX(k0 + k, c, lds)] / sU[t], ORACLE_E4M3);
            }
            #pragma omp parallel for schedule(static)
            for (int64_t c = c1; c < n; ++c) {
                double su = sU[(c - c1) / tile];
                for (int64_t i = c1; i < n; ++i) {
                    double sl = sL[(i - c1) / tile];
                    float acc = 0.0f;
                    for (int64_t k = 0; k < kb; ++k)
                        acc = fmaf(Lq[IDX(i - c1, k, mt)], Uq[IDX(k, c - c1, kb)], acc);
                    float upd = (float)((double)acc * sl);    /* exact: power of 2 */
                    upd = (float)((double)upd * su);
                    float a = to_f32(S[IDX(i, c, lds)]) - upd;
                    S[IDX(i, c, lds)] = oracle_round((double)a, ORACLE_FP16);
                }
            }
        }
    }
    free(P); free(Lq); free(Uq); free(sL); free(sU);
    return info;
}

/* The complete low-precision factorization (all panel steps). */
int oracle_lp_getrf(int64_t n, int64_t nb, int prec, int pivot, int64_t tile,
                    double *S, int64_t lds, int32_t *ipiv)
{
    return oracle_lp_getrf_steps(n, nb, prec, pivot, tile, S, lds, ipiv, -1);
}

/*
 * Preconditioner of the refinement: d = M r with M = U^-1 L^-1 P built from
 * the stored low-precision factors (trans = 0), or d = M^T r (trans = 1).
 * The vector is scaled by s = ||r||_inf and rounded to FP32, the triangular
 * solves run in FP32 on the stored factor values (exact in FP32), and the
 * result is rescaled by s in FP64.  ipiv may be NULL (no pivoting).
 */
int oracle_lp_precond(int64_t n, const double *F, int64_t ldf,
                      const int32_t *ipiv, const double *r, double *d, int trans)
{
    if (n < 0 || ldf < (n > 1 ? n : 1)) return -1;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) if (fabs(r[i]) > s) s = fabs(r[i]);
    if (s == 0.0) { for (int64_t i = 0; i < n; ++i) d[i] = 0.0; return 0; }
    float *v = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    if (!v) return -1000;
    for (int64_t i = 0; i < n; ++i) v[i] = (float)(r[i] / s);
    if (trans == 0) {
        if (ipiv)
            for (int64_t j = 0; j < n; ++j) {
                int64_t p = ipiv[j];
                if (p != j) { float t = v[j]; v[j] = v[p]; v[p] = t; }
            }
        for (int64_t k = 0; k < n; ++k)
            for (int64_t i = k + 1; i < n; ++i)
                v[i] = fmaf(-(float)F[IDX(i, k, ldf)], v[k], v[i]);
        for (int64_t k = n - 1; k >= 0; --k) {
            v[k] = v[k] / (float)F[IDX(k, k, ldf)];
            for (int64_t i = 0; i < k; ++i)
                v[i] = fmaf(-(float)F[IDX(i, k, ldf)], v[k], v[i]);
        }
    } else {
        for (int64_t k = 0; k < n; ++k) {
            float acc = v[k];
            for (int64_t i = 0; i < k; ++i)
                acc = fmaf(-(float)F[IDX(i, k, ldf)], v[i], acc);
            v[k] = acc / (float)F[IDX(k, k, ldf)];
        }
        for (int64_t k = n - 1; k >= 0; --k) {
            float acc = v[k];
            for (int64_t i = k + 1; i < n; ++i)
                acc = fmaf(-(float)F[IDX(i, k, ldf)], v[i], acc);
            v[k] = acc;
        }
        if (ipiv)
            for (int64_t j = n - 1; j >= 0; --j) {
                int64_t p = ipiv[j];
                if (p != j) { float t = v[j]; v[j] = v[p]; v[p] = t; }
            }
    }
    for (int64_t i = 0; i < n; ++i) d[i] = s * (double)v[i];
    free(v);
    return 0;
}
