// Mixed-precision solve: low-precision LU + FP64 iterative refinement.
//
// Sec. III-A.2: factorization and trailing updates in reduced precision with
// pivoting omitted, residual evaluation and corrections in FP64, refinement
// restoring double-precision accuracy; Sec. II-B: the refinement is
// non-stationary, based on GMRES.  Here everything runs on the GPU:
//   convert    A (FP64) -> F (bf16 / fp16), round to nearest even from FP64
//   factor     blocked LU of F: FP32 panel and U12 TRSM, MFMA trailing update
//              (16-bit operands or e4m3fn with tile scales), FP32 accumulation
//   x0         = M b,  M = U^-1 L^-1 (P) in FP32 on the stored factors
//   refine     r = b - A x in FP64; stop when the HPL scaled residual
//              ||r||_inf / (eps (||A||_inf ||x||_inf + ||b||_inf) n) < threshold;
//              classical: x += M r;  GMRES-IR: one restarted cycle of
//              left-preconditioned GMRES on A d = r per step (classical
//              Gram-Schmidt applied twice, Givens rotations on the host), x += d.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "lp_common.h"
#include "lp_kernels.h"
#include "profile.h"
#include "refine_kernels.h"

namespace {

using namespace mxlu;

int64_t factor_ld(int64_t n) { return ((n + 63) / 64) * 64 + 64; }

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            (void)hipGetLastError();
            a = b = nullptr;
        }
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start() {
        if (a) (void)hipEventRecord(a, s);
    }
    void stop() {
        if (b) (void)hipEventRecord(b, s);
    }
    double ms() {
        float t = 0.f;
        if (!a || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) {
            (void)hipGetLastError();
            return 0.0;
        }
        return t;
    }
};

// Fork and join of the look-ahead stream p with the factorization stream s;
// joins p back into s when it goes out of scope (also on an error return, so
// that no work of the call still runs when its scratch memory is released).
class AheadJoin {
  public:
    AheadJoin(hipStream_t s, hipStream_t p) : s_(s), p_(p) {}
    ~AheadJoin() {
        if (active_) (void)join();
        for (hipEvent_t e : ev_)
            if (e) (void)hipEventDestroy(e);
    }
    int create() {
        for (hipEvent_t &e : ev_)
            MXLU_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        active_ = true;
        return 0;
    }
    // p continues after everything enqueued so far on s
    int fork() {
        MXLU_HIP_TRY(hipEventRecord(ev_[0], s_));
        MXLU_HIP_TRY(hipStreamWaitEvent(p_, ev_[0], 0));
        return 0;
    }
    // s continues after everything enqueued so far on p
    int join() {
        MXLU_HIP_TRY(hipEventRecord(ev_[1], p_));
        MXLU_HIP_TRY(hipStreamWaitEvent(s_, ev_[1], 0));
        return 0;
    }

  private:
    hipStream_t s_, p_;
    hipEvent_t ev_[2] = {};
    bool active_ = false;
};

// ------------------------------------------------------------------ factor
int lp_factorize(const mxp_opts &o, int64_t n, const ASource &src, uint16_t *F,
                 int64_t ldf, int32_t *ipiv, int *info_host, hipStream_t s, double *t_conv,
                 double *t_fact) {
    const int fmt = (o.prec == MXLU_PREC_BF16) ? kFmtBf16 : kFmtFp16;
    const bool mx = o.prec == MXLU_PREC_FP8_MX;
    const bool fp8 = o.prec == MXLU_PREC_FP8 || mx;
    const int64_t nb = std::min<int64_t>(o.nb, n);
    const int tile = o.scale_tile;
    Scratch scratch(s);
    float *P32 = scratch.alloc_n<float>((size_t)n * nb);
    float *T32 = scratch.alloc_n<float>((size_t)nb * n);
    int *d_info = scratch.alloc_n<int>(4);   // [0] first zero pivot, [2] the leaves' counter
    const int64_t Mp = lp_round_up(n, kLpTileM), Np = lp_round_up(n, kLpTileN);
    const int64_t Mp8 = lp_round_up(n, kLp8Tile), Np8 = lp_round_up(n, kLp8Tile);
    // the packed operands of one step's update (a second set for the step
    // prepared ahead)
    struct Ops {
        uint16_t *LTp = nullptr, *Up = nullptr;   // chunk-packed L21 and U12 (16-bit form)
        uint8_t *LTq = nullptr, *Uq = nullptr;    // e4m3 L21 and U12 (FP8 forms)
        float *sL = nullptr, *sU = nullptr;       // power-of-two tile scales
        uint8_t *sLx = nullptr, *sUx = nullptr;   // MX block scales
    };
    auto alloc_ops = [&](Ops &q) -> int {
        if (fp8) {
            q.LTq = scratch.alloc_n<uint8_t>((size_t)nb * Mp8);
            q.Uq = scratch.alloc_n<uint8_t>((size_t)nb * Np8);
            if (!q.LTq || !q.Uq) return MXLU_E_NOMEM;
            if (mx) {
                q.sLx = scratch.alloc_n<uint8_t>((size_t)(nb / 32) * Mp8);
                q.sUx = scratch.alloc_n<uint8_t>((size_t)(nb / 32) * Np8);
                if (!q.sLx || !q.sUx) return MXLU_E_NOMEM;
            } else {
                q.sL = scratch.alloc_n<float>((size_t)(n / tile + 2));
                q.sU = scratch.alloc_n<float>((size_t)(n / tile + 2));
                if (!q.sL || !q.sU) return MXLU_E_NOMEM;
            }
        } else {
            q.LTp = scratch.alloc_n<uint16_t>((size_t)nb * Mp);
            q.Up = scratch.alloc_n<uint16_t>((size_t)nb * Np);
            if (!q.LTp || !q.Up) return MXLU_E_NOMEM;
        }
        return 0;
    };
    Ops cur, nxt;
    MXLU_TRY(alloc_ops(cur));
    if (!P32 || !T32 || !d_info) return MXLU_E_NOMEM;
    MXLU_HIP_TRY(hipMemsetAsync(d_info, 0, 4 * sizeof(int), s));
    PanelExchange ex{};
    int *moves = nullptr;
    if (o.pivot) {
        MXLU_TRY(alloc_panel_exchange(scratch, n, &ex, s));
        moves = scratch.alloc_n<int>(kSwapMovesInts);
        if (!moves) return MXLU_E_NOMEM;
    }

    Timer tc(s), tf(s);
    tc.start();
    {
        PhaseScope ph(kPhaseConvert, s, 10.0 * (double)n * (double)n);
        MXLU_TRY(lp_convert_src(fmt, n, src, F, ldf, s));
    }
    tc.stop();

    // Depth-1 look-ahead (no pivoting only: the pivoted panel's workgroups
    // must all be resident at once, which a stream shared with the update
    // cannot promise).  The update of step k runs in three parts: the next
    // panel's columns, then the top rows of the other columns (the next
    // step's U12 rows), then the rest.  After the first part the next panel
    // is factored on the look-ahead stream; after the second, the same stream
    // solves and packs the next step's U12 and packs its L21 into the second
    // operand set, all while the third part runs.  Each part is a set of
    // whole tiles of the undivided update (split at multiples of the tile
    // sizes and of the scale tile), so every element takes the same
    // operations in the same order as at depth 0.
    AheadStreams ahs;
    std::unique_lock<std::mutex> ahead_lock;
    const int64_t tile_m = fp8 ? kLp8Tile : kLpTileM;
    const bool la = !o.pivot && n > nb && nb % tile_m == 0 && nb % 128 == 0 &&
                    (!fp8 || mx || nb % tile == 0) && lp_ahead_streams(&ahs, &ahead_lock);
    if (la) MXLU_TRY(alloc_ops(nxt));
    AheadJoin aj(s, la ? ahs.panel : nullptr);
    if (la) MXLU_TRY(aj.create());

    // PFACT of the panel at k0 (width kb) on stream st; the 16-bit form also
    // packs its L21 into q
    auto pfact = [&](int64_t k0, int64_t kb, hipStream_t st, Ops &q) -> int {
        const int64_t m = n - k0, c1 = k0 + kb;
        uint16_t *Fk = F + (size_t)k0 + (size_t)k0 * ldf;
        // work: the panel's bytes in storage precision
        PhaseScope ph(kPhasePfact, st, 2.0 * (double)m * kb);
        MXLU_TRY(lp_load_f32(fmt, m, kb, Fk, ldf, P32, m, st));
        if (o.pivot)   // partial pivoting on the FP32 values of the panel
            MXLU_TRY(panel_factor<float>(P32, m, m, kb, k0, ipiv, ex, moves, st));
        else
            MXLU_TRY(lp_panel_factor_nopiv(m, (int)kb, P32, m, d_info, d_info + 2, k0, st));
        const bool need_lt = !fp8 && c1 < n;
        return lp_panel_store(fmt, m, (int)kb, P32, m, Fk, ldf, need_lt ? q.LTp : nullptr, Mp,
                              st);
    };
    // U12 = L11^-1 A12 of the step at k0 in FP32 (L11 from P32), then the
    // update's operands packed into q (quantised for FP8), on stream st
    auto finish = [&](int64_t k0, int64_t kb, hipStream_t st, Ops &q) -> int {
        const int64_t c1 = k0 + kb, nt = n - c1;
        uint16_t *U12 = F + (size_t)k0 + (size_t)c1 * ldf;
        {
            PhaseScope ph(kPhaseTrsm, st, (double)kb * (kb - 1) * (double)nt);
            MXLU_TRY(lp_load_f32(fmt, kb, nt, U12, ldf, T32, kb, st));
            MXLU_TRY(trsm_f32_llnu(kb, nt, P32, n - k0, T32, kb, st));
            MXLU_TRY(lp_store_f32(fmt, kb, nt, T32, kb, U12, ldf, st));
        }
        const uint16_t *L21 = F + (size_t)c1 + (size_t)k0 * ldf;
        if (mx) {
            MXLU_TRY(lp_quant_l21_mx(fmt, nt, (int)kb, L21, ldf, q.LTq, Mp8, q.sLx, st));
            return lp_quant_u12_mx(fmt, nt, (int)kb, U12, ldf, q.Uq, Np8, q.sUx, st);
        }
        if (fp8) {
            MXLU_TRY(lp_quant_l21(fmt, nt, (int)kb, tile, L21, ldf, q.LTq, Mp8, q.sL, st));
            return lp_quant_u12(fmt, nt, (int)kb, tile, U12, ldf, q.Uq, Np8, q.sU, st);
        }
        return lp_pack_u12(nt, (int)kb, U12, ldf, q.Up, Np, st);
    };
    // rows [i0, i0 + h) x columns [j0, j0 + w) of the trailing update
    // A22 -= L21 U12 of the step at k0, from the operands in q, on stream st
    auto update = [&](int64_t k0, int64_t kb, int64_t i0, int64_t h, int64_t j0, int64_t w,
                      hipStream_t st, const Ops &q) -> int {
        const int64_t c1 = k0 + kb;
        uint16_t *C = F + (size_t)(c1 + i0) + (size_t)(c1 + j0) * ldf;
        // algorithmic bytes: the block of A22 read and written in 16 bits,
        // its L21 rows and U12 columns read once
        const double ob = fp8 ? 1.0 : 2.0;
        PhaseScope ph(kPhaseLpSchur, st, 4.0 * (double)h * (double)w + ob * (double)(h + w) * kb);
        if (mx)
            return lp_schur_update_mx(fmt, h, w, (int)kb, q.LTq, Mp8, q.sLx, i0, q.Uq, Np8, q.sUx,
                                      j0, C, ldf, st);
        if (fp8)
            return lp_schur_update_fp8(fmt, h, w, (int)kb, q.LTq, Mp8, q.sL, i0, q.Uq, Np8, q.sU,
                                       j0, tile, C, ldf, st);
        return lp_schur_update(fmt, h, w, (int)kb, q.LTp, Mp, i0, q.Up, Np, j0, C, ldf, st);
    };

    tf.start();
    {
        PhaseScope ph(kPhaseLpFactor, s, (2.0 / 3.0) * (double)n * n * n);
        int64_t step = 0;
        bool ahead = false;   // the current step was prepared during the previous update
        for (int64_t k0 = 0; k0 < n; k0 += nb, ++step) {
            if (o.factor_steps > 0 && step >= o.factor_steps) break;
            profile_set_step(step);
            const int64_t kb = std::min(nb, n - k0), c1 = k0 + kb;
            if (!ahead) MXLU_TRY(pfact(k0, kb, s, cur));
            if (o.pivot && n > kb) {   // the panel's interchanges on the other stored columns
                PhaseScope ph(kPhaseSwap, s, 8.0 * kb * (double)(n - kb));
                MXLU_TRY(swap_compose(ipiv, k0, (int)kb, n, moves, s));
                MXLU_TRY(swap_apply<uint16_t>(F, ldf, k0, moves, 0, n - kb, k0, kb, s));
            }
            if (c1 >= n) continue;
            if (!ahead) MXLU_TRY(finish(k0, kb, s, cur));
            ahead = false;
            const int64_t nt = n - c1;
            // a factorization stopped after this step leaves the next panel
            // unfactored, so it is not factored ahead
            const bool go_ahead = la && !(o.factor_steps > 0 && step + 1 >= o.factor_steps);
            if (!go_ahead) {
                MXLU_TRY(update(k0, kb, 0, nt, 0, nt, s, cur));
                continue;
            }
            const int64_t kb1 = std::min(nb, nt), rest = nt - kb1;
            MXLU_TRY(update(k0, kb, 0, nt, 0, kb1, s, cur));
            MXLU_TRY(aj.fork());
            profile_set_step(step + 1);   // the next step's panel
            MXLU_TRY(pfact(c1, kb1, ahs.panel, nxt));
            profile_set_step(step);
            if (rest > 0) {
                MXLU_TRY(update(k0, kb, 0, kb1, kb1, rest, s, cur));
                MXLU_TRY(aj.fork());   // the next step's U12 rows are final
                profile_set_step(step + 1);
                MXLU_TRY(finish(c1, kb1, ahs.panel, nxt));
                profile_set_step(step);
                MXLU_TRY(update(k0, kb, kb1, rest, kb1, rest, s, cur));
            }
            MXLU_TRY(aj.join());
            std::swap(cur, nxt);
            ahead = true;
        }
    }
    profile_set_step(-1);
    tf.stop();
    int hinfo[4] = {0, 0, 0, 0};
    MXLU_HIP_TRY(hipMemcpyAsync(hinfo, o.pivot ? ex.flags : d_info, sizeof(hinfo),
                                hipMemcpyDeviceToHost, s));
    MXLU_HIP_TRY(hipStreamSynchronize(s));
    if (o.pivot && hinfo[1]) {
        set_error_msg("mxp_solve: panel grid barrier wait expired");
        return MXLU_E_TIMEOUT;
    }
    *info_host = hinfo[0];
    *t_conv = tc.ms();
    *t_fact = tf.ms();
    return 0;
}

// FP32 factor storage (the first rung of the precision ladder): the factors
// are FP32 numbers in the workspace, so the panel, the interchanges, the U12
// TRSM and the trailing update all work in place on them with the FP32 kernels
// (every element takes its terms in ascending k, one fused multiply-add each).
int lp_factorize_f32(const mxp_opts &o, int64_t n, const ASource &src, float *F, int64_t ldf,
                     int32_t *ipiv, int *info_host, hipStream_t s, double *t_conv,
                     double *t_fact) {
    const int64_t nb = std::min<int64_t>(o.nb, n);
    Scratch scratch(s);
    int *d_info = scratch.alloc_n<int>(4);   // [0] first zero pivot, [2] the leaves' counter
    if (!d_info) return MXLU_E_NOMEM;
    MXLU_HIP_TRY(hipMemsetAsync(d_info, 0, 4 * sizeof(int), s));
    PanelExchange ex{};
    int *moves = nullptr;
    if (o.pivot) {
        MXLU_TRY(alloc_panel_exchange(scratch, n, &ex, s));
        moves = scratch.alloc_n<int>(kSwapMovesInts);
        if (!moves) return MXLU_E_NOMEM;
    }
    Timer tc(s), tf(s);
    tc.start();
    {
        PhaseScope ph(kPhaseConvert, s, 12.0 * (double)n * (double)n);
        MXLU_TRY(lp_convert_src_f32(n, src, F, ldf, s));
    }
    tc.stop();
    tf.start();
    {
        PhaseScope ph(kPhaseLpFactor, s, (2.0 / 3.0) * (double)n * n * n);
        int64_t step = 0;
        for (int64_t k0 = 0; k0 < n; k0 += nb, ++step) {
            if (o.factor_steps > 0 && step >= o.factor_steps) break;
            profile_set_step(step);
            const int64_t kb = std::min(nb, n - k0), m = n - k0, c1 = k0 + kb;
            float *Fk = F + (size_t)k0 + (size_t)k0 * ldf;
            {
                PhaseScope ph(kPhasePfact, s, 4.0 * (double)m * kb);
                if (o.pivot)
                    MXLU_TRY(panel_factor<float>(Fk, ldf, m, kb, k0, ipiv, ex, moves, s));
                else
                    MXLU_TRY(lp_panel_factor_nopiv(m, (int)kb, Fk, ldf, d_info, d_info + 2, k0, s));
            }
            if (o.pivot && n > kb) {
                PhaseScope ph(kPhaseSwap, s, 16.0 * kb * (double)(n - kb));
                MXLU_TRY(swap_compose(ipiv, k0, (int)kb, n, moves, s));
                MXLU_TRY(swap_apply<float>(F, ldf, k0, moves, 0, n - kb, k0, kb, s));
            }
            if (c1 >= n) continue;
            const int64_t nt = n - c1;
            float *U12 = F + (size_t)k0 + (size_t)c1 * ldf;
            {
                PhaseScope ph(kPhaseTrsm, s, (double)kb * (kb - 1) * (double)nt);
                MXLU_TRY(trsm_f32_llnu(kb, nt, Fk, ldf, U12, ldf, s));
            }
            {   // A22 -= L21 U12 in FP32 (work: bytes of A22 read and written)
                PhaseScope ph(kPhaseLpSchur, s, 8.0 * (double)nt * (double)nt);
                MXLU_TRY(gemm_f32_sub(nt, nt, kb, F + (size_t)c1 + (size_t)k0 * ldf, ldf, U12, ldf,
                                      F + (size_t)c1 + (size_t)c1 * ldf, ldf, s));
            }
        }
    }
    profile_set_step(-1);
    tf.stop();
    int hinfo[4] = {0, 0, 0, 0};
    MXLU_HIP_TRY(hipMemcpyAsync(hinfo, o.pivot ? ex.flags : d_info, sizeof(hinfo),
                                hipMemcpyDeviceToHost, s));
    MXLU_HIP_TRY(hipStreamSynchronize(s));
    if (o.pivot && hinfo[1]) {
        set_error_msg("mxp_solve: panel grid barrier wait expired");
        return MXLU_E_TIMEOUT;
    }
    *info_host = hinfo[0];
    *t_conv = tc.ms();
    *t_fact = tf.ms();
    return 0;
}

// ------------------------------------------------------------------ refine
struct RefineCtx {
    int fmt, trans;
    int64_t n, ldf;
    ASource src;   // the FP64 matrix: in memory or regenerated from its seed
    const uint16_t *F;
    const float *F32 = nullptr;   // FP32 factor storage
    const int32_t *perm;
    hipStream_t s;
    const mxp_opts *o;
    // device scratch
    double *r, *z, *w, *V, *part, *apart, *dotp, *hdev;
    float *v32;
    unsigned long long *stats;   // [0] |r|max [1] ||A|| [2] |x|max [3] precond s
    TrsvChain ch{};
    int nsplit, nchunks;
    double anorm = -1.0;
};

int precond(RefineCtx &c, const double *r, double *d) {
    if (c.F32)
        return lp_precond_apply_f32(c.n, c.F32, c.ldf, c.perm, r, d, c.v32, c.stats + 3, c.s);
    return lp_precond_apply(c.fmt, c.trans, c.n, c.F, c.ldf, c.perm, r, d, c.v32, c.stats + 3,
                            c.ch, c.s);
}

// r = b - op(A) x; returns the scaled residual (host sync).
int residual(RefineCtx &c, const double *b, const double *x, double bnorm, double *rho) {
    MXLU_HIP_TRY(hipMemsetAsync(c.stats, 0, 3 * sizeof(unsigned long long), c.s));
    const bool need_anorm = c.anorm < 0.0;
    MXLU_TRY(gemv_f64(c.trans, c.n, c.src, x, b, c.r, c.part, need_anorm ? c.apart : nullptr,
                      c.nsplit, c.stats, c.s));
    unsigned long long h[3];
    MXLU_HIP_TRY(hipMemcpyAsync(h, c.stats, sizeof(h), hipMemcpyDeviceToHost, c.s));
    MXLU_HIP_TRY(hipStreamSynchronize(c.s));
    double v[3];
    std::memcpy(v, h, sizeof(v));
    if (need_anorm) c.anorm = v[1];
    const double eps = 0x1p-53;
    const double den = eps * (c.anorm * v[2] + bnorm) * (double)c.n;
    *rho = den > 0.0 ? v[0] / den : (v[0] > 0.0 ? INFINITY : 0.0);
    return 0;
}

// One GMRES cycle on op(A) d = r (left preconditioned by M); x += d.
int gmres_cycle(RefineCtx &c, double *x, int mmax, int *steps) {
    const int64_t n = c.n;
    const int64_t ldv = n;
    std::vector<double> H((size_t)(mmax + 1) * mmax, 0.0), cs(mmax), sn(mmax), g(mmax + 1, 0.0);
    std::vector<double> hh(2 * (size_t)(mmax + 1) + 2);
    *steps = 0;
    // z = M r; beta = ||z||
    MXLU_TRY(precond(c, c.r, c.z));
    MXLU_TRY(dots_f64(n, 1, c.z, ldv, c.z, c.dotp, c.nchunks, c.hdev, c.s));
    double beta2 = 0.0;
    MXLU_HIP_TRY(hipMemcpyAsync(&beta2, c.hdev, sizeof(double), hipMemcpyDeviceToHost, c.s));
    MXLU_HIP_TRY(hipStreamSynchronize(c.s));
    const double beta = std::sqrt(beta2);
    if (!(beta > 0.0)) return 0;
    MXLU_TRY(scale_copy_f64(n, c.z, 1.0 / beta, c.V, c.s));
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < mmax; ++j) {
        double *vj = c.V + (size_t)j * ldv;
        // w = op(A) v_j ; z = M w
        MXLU_TRY(gemv_f64(c.trans, n, c.src, vj, nullptr, c.w, c.part, nullptr, c.nsplit,
                          nullptr, c.s));
        MXLU_TRY(precond(c, c.w, c.z));
        // classical Gram-Schmidt, twice
        double *h1 = c.hdev, *h2 = c.hdev + (mmax + 1), *hn = c.hdev + 2 * (mmax + 1);
        MXLU_TRY(dots_f64(n, j + 1, c.V, ldv, c.z, c.dotp, c.nchunks, h1, c.s));
        MXLU_TRY(gemv_small_f64(n, j + 1, c.V, ldv, h1, -1.0, c.z, c.s));
        MXLU_TRY(dots_f64(n, j + 1, c.V, ldv, c.z, c.dotp, c.nchunks, h2, c.s));
        MXLU_TRY(gemv_small_f64(n, j + 1, c.V, ldv, h2, -1.0, c.z, c.s));
        MXLU_TRY(dots_f64(n, 1, c.z, ldv, c.z, c.dotp, c.nchunks, hn, c.s));
        MXLU_HIP_TRY(hipMemcpyAsync(hh.data(), c.hdev, sizeof(double) * (2 * (mmax + 1) + 1),
                                    hipMemcpyDeviceToHost, c.s));
        MXLU_HIP_TRY(hipStreamSynchronize(c.s));
        const double hnorm = std::sqrt(hh[2 * (mmax + 1)]);
        for (int i = 0; i <= j; ++i) H[(size_t)j * (mmax + 1) + i] = hh[i] + hh[(mmax + 1) + i];
        H[(size_t)j * (mmax + 1) + j + 1] = hnorm;
        if (hnorm > 0.0)
            MXLU_TRY(scale_copy_f64(n, c.z, 1.0 / hnorm, c.V + (size_t)(j + 1) * ldv, c.s));
        double *col = &H[(size_t)j * (mmax + 1)];
        for (int i = 0; i < j; ++i) {   // previous rotations
            const double t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        cs[j] = col[j] / den;
        sn[j] = col[j + 1] / den;
        col[j] = den;
        col[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        k = j + 1;
        if (std::fabs(g[j + 1]) <= c.o->inner_tol * beta || hnorm == 0.0) break;
    }
    // y = H[:k,:k]^-1 g[:k];  x += V[:, :k] y
    std::vector<double> y(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
        double acc = g[i];
        for (int t = i + 1; t < k; ++t) acc -= H[(size_t)t * (mmax + 1) + i] * y[t];
        y[i] = acc / H[(size_t)i * (mmax + 1) + i];
    }
    MXLU_HIP_TRY(hipMemcpyAsync(c.hdev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, c.s));
    MXLU_HIP_TRY(hipStreamSynchronize(c.s));   // y is a host temporary
    MXLU_TRY(gemv_small_f64(n, k, c.V, ldv, c.hdev, 1.0, x, c.s));
    *steps = k;
    return 0;
}

// Refine one right-hand side.  *conv, *outer, *inner, *rho out.
int refine_column(RefineCtx &c, const double *b, double *x, bool x_init, int *conv, int *outer,
                  int *inner, double *rho_out) {
    const mxp_opts &o = *c.o;
    const int64_t n = c.n;
    unsigned long long hb;
    MXLU_HIP_TRY(hipMemsetAsync(c.stats, 0, sizeof(unsigned long long), c.s));
    MXLU_TRY(absmax_f64(n, b, c.stats, c.s));
    MXLU_HIP_TRY(hipMemcpyAsync(&hb, c.stats, sizeof(hb), hipMemcpyDeviceToHost, c.s));
    MXLU_HIP_TRY(hipStreamSynchronize(c.s));
    double bnorm;
    std::memcpy(&bnorm, &hb, sizeof(double));
    if (!x_init) MXLU_TRY(precond(c, b, x));
    std::vector<double> hist;
    int increases = 0, it = 0, inner_total = 0;
    *conv = 0;
    double rho = 0.0;
    while (true) {
        MXLU_TRY(residual(c, b, x, bnorm, &rho));
        hist.push_back(rho);
        if (rho < o.resid_threshold) {
            *conv = 1;
            break;
        }
        if (hist.size() > 1 && hist[hist.size() - 1] > hist[hist.size() - 2]) ++increases;
        else increases = 0;
        if (it >= o.max_outer || increases >= 3 || inner_total >= o.max_inner_total) break;
        if (o.refine == MXLU_IR_CLASSICAL) {
            MXLU_TRY(precond(c, c.r, c.z));
            MXLU_TRY(axpy_f64(n, c.z, x, c.s));
        } else {
            const int mm = std::min(o.restart, o.max_inner_total - inner_total);
            int steps = 0;
            MXLU_TRY(gmres_cycle(c, x, mm, &steps));
            inner_total += steps;
        }
        ++it;
    }
    *outer = it;
    *inner = inner_total;
    *rho_out = rho;
    return 0;
}

}  // namespace

extern "C" void mxp_default_opts(mxp_opts *o) {
    if (!o) return;
    o->prec = MXLU_PREC_BF16;
    o->pivot = 0;
    o->nb = 512;
    o->refine = MXLU_IR_GMRES;
    o->restart = 30;
    o->max_outer = 20;
    o->max_inner_total = 300;
    o->inner_tol = 1e-6;
    o->resid_threshold = 16.0;
    o->scale_tile = 128;
    o->reuse_factors = 0;
    o->trans = 0;
    o->x_init = 0;
    o->factor_steps = 0;
}

extern "C" size_t mxp_workspace_bytes(int64_t n, int64_t lda, const mxp_opts *o) {
    if (n < 0 || lda < std::max<int64_t>(1, n) || !o) return 0;
    const int64_t ldf = factor_ld(n);
    const size_t esz = o->prec == MXLU_PREC_FP32 ? 4 : 2;   // bytes per stored factor value
    const double bytes = (double)ldf * (double)n * (double)esz + 256.0;
    if (bytes > 9.0e18) return 0;
    return (size_t)ldf * (size_t)n * esz + 256;
}

extern "C" int64_t mxp_factor_ld(int64_t n) { return n < 0 ? 0 : factor_ld(n); }

extern "C" int mxp_convert(int32_t prec, int64_t rows, int64_t cols, const double *A,
                           int64_t lda, uint16_t *F, int64_t ldf, void *stream) {
    if (prec < 0 || prec > 3) return -1;
    if (rows < 0) return -2;
    if (cols < 0) return -3;
    if (rows > 0 && cols > 0 && !A) return -4;
    if (lda < std::max<int64_t>(1, rows)) return -5;
    if (rows > 0 && cols > 0 && !F) return -6;
    if (ldf < std::max<int64_t>(1, rows)) return -7;
    if (rows == 0 || cols == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    return lp_convert(prec == MXLU_PREC_BF16 ? kFmtBf16 : kFmtFp16, rows, cols, A, lda, F, ldf,
                      (hipStream_t)stream);
}

namespace {

// Argument checks shared by both forms (all but the matrix's own arguments).
int mxp_check(int64_t n, int64_t nrhs, const double *B, int64_t ldb, double *X, int64_t ldx,
              void *work, int32_t *ipiv, const mxp_opts *opts) {
    if (n > 0 && nrhs > 0 && !B) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (n > 0 && nrhs > 0 && !X) return -7;
    if (ldx < std::max<int64_t>(1, n)) return -8;
    if (n > 0 && !work) return -9;
    if (!opts) return -12;
    const mxp_opts &o = *opts;
    if (o.prec < 0 || o.prec > 4 || (o.pivot != 0 && o.pivot != 1) || o.nb < 32 ||
        o.nb % 32 != 0 || (o.prec == MXLU_PREC_FP8 && (o.nb % 128 != 0 || o.scale_tile < 4 ||
                                                       o.scale_tile > 256 || o.scale_tile % 4)) ||
        (o.prec == MXLU_PREC_FP8_MX && o.nb % 128 != 0) ||
        (o.prec == MXLU_PREC_FP32 && o.trans != 0) ||
        (o.refine != MXLU_IR_CLASSICAL && o.refine != MXLU_IR_GMRES) || o.restart < 1 ||
        o.restart > 255 || o.max_outer < 0 || o.max_inner_total < 0 || o.trans < 0 ||
        o.trans > 1 || o.factor_steps < 0)
        return -12;
    if (o.pivot && !ipiv) return -11;
    return 0;
}

int mxp_impl(int64_t n, int64_t nrhs, const ASource &src, const double *B, int64_t ldb,
             double *X, int64_t ldx, void *work, size_t work_bytes, int32_t *ipiv,
             const mxp_opts *opts, mxp_report *report, hipStream_t s) {
    const mxp_opts &o = *opts;
    (void)work_bytes;
    const int fmt = (o.prec == MXLU_PREC_BF16) ? kFmtBf16 : kFmtFp16;
    const bool f32 = o.prec == MXLU_PREC_FP32;
    const int64_t ldf = factor_ld(n);
    uint16_t *F = reinterpret_cast<uint16_t *>(work);
    float *F32 = reinterpret_cast<float *>(work);

    double t_conv = 0.0, t_fact = 0.0;
    int info = 0;
    if (!o.reuse_factors) {
        if (f32)
            MXLU_TRY(lp_factorize_f32(o, n, src, F32, ldf, ipiv, &info, s, &t_conv, &t_fact));
        else
            MXLU_TRY(lp_factorize(o, n, src, F, ldf, ipiv, &info, s, &t_conv, &t_fact));
    }

    Scratch scratch(s);
    RefineCtx c;
    c.fmt = fmt;
    c.trans = o.trans;
    c.n = n;
    c.ldf = ldf;
    c.src = src;
    c.F = F;
    c.F32 = f32 ? F32 : nullptr;
    c.perm = nullptr;
    if (o.pivot) {
        int32_t *perm = scratch.alloc_n<int32_t>((size_t)n);
        if (!perm) return MXLU_E_NOMEM;
        MXLU_TRY(perm_from_ipiv(n, ipiv, perm, s));
        c.perm = perm;
    }
    c.s = s;
    c.o = &o;
    c.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(32, n / 2048));
    c.nchunks = (int)std::max<int64_t>(1, std::min<int64_t>(128, n / 1024));
    const int m1 = o.restart + 1;
    c.r = scratch.alloc_n<double>((size_t)n);
    c.z = scratch.alloc_n<double>((size_t)n);
    c.w = scratch.alloc_n<double>((size_t)n);
    c.V = scratch.alloc_n<double>((size_t)n * m1);
    c.part = scratch.alloc_n<double>((size_t)n * c.nsplit);
    c.apart = scratch.alloc_n<double>((size_t)n * c.nsplit);
    c.dotp = scratch.alloc_n<double>((size_t)c.nchunks * m1);
    c.hdev = scratch.alloc_n<double>((size_t)2 * m1 + 8);
    c.v32 = scratch.alloc_n<float>((size_t)n);
    c.stats = scratch.alloc_n<unsigned long long>(8);
    c.ch.xs = scratch.alloc_n<uint64_t>((size_t)n);
    c.ch.expired = scratch.alloc_n<int>(1);
    if (!c.r || !c.z || !c.w || !c.V || !c.part || !c.apart || !c.dotp || !c.hdev || !c.v32 ||
        !c.stats || !c.ch.xs || !c.ch.expired)
        return MXLU_E_NOMEM;
    MXLU_HIP_TRY(hipMemsetAsync(c.ch.xs, 0, sizeof(uint64_t) * (size_t)n, s));
    MXLU_HIP_TRY(hipMemsetAsync(c.ch.expired, 0, sizeof(int), s));

    Timer tr(s);
    tr.start();
    int all_conv = 1, outer_sum = 0, inner_sum = 0;
    double worst = 0.0;
    {
        PhaseScope ph(kPhaseRefine, s, 0.0);
        for (int64_t col = 0; col < nrhs; ++col) {
            int conv = 0, outer = 0, inner = 0;
            double rho = 0.0;
            MXLU_TRY(refine_column(c, B + (size_t)col * ldb, X + (size_t)col * ldx, o.x_init != 0,
                                   &conv, &outer, &inner, &rho));
            all_conv &= conv;
            outer_sum += outer;
            inner_sum += inner;
            worst = std::max(worst, rho);
        }
    }
    tr.stop();
    const double t_ref = tr.ms();
    int expired = 0;
    MXLU_HIP_TRY(hipMemcpyAsync(&expired, c.ch.expired, sizeof(int), hipMemcpyDeviceToHost, s));
    MXLU_HIP_TRY(hipStreamSynchronize(s));
    if (expired) {
        mxlu::set_error_msg("mxp_solve: triangular-solve wait expired");
        return MXLU_E_TIMEOUT;
    }
    if (report) {
        report->converged = all_conv;
        report->outer_iters = outer_sum;
        report->inner_iters = inner_sum;
        report->info = info;
        report->scaled_residual = worst;
        report->t_convert_ms = t_conv;
        report->t_factor_ms = t_fact;
        report->t_refine_ms = t_ref;
    }
    if (!all_conv) {
        mxlu::set_error_msg("mxp_solve: a column did not reach the residual threshold");
        return MXLU_E_NOTCONV;
    }
    return 0;
}

}  // namespace

extern "C" int mxp_solve(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                         int64_t ldb, double *X, int64_t ldx, void *work, size_t work_bytes,
                         int32_t *ipiv, const mxp_opts *opts, mxp_report *report, void *stream) {
    if (n < 0 || n > 0x7fffffff) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (int rc = mxp_check(n, nrhs, B, ldb, X, ldx, work, ipiv, opts)) return rc;
    if (n > 0 && work_bytes < mxp_workspace_bytes(n, lda, opts)) return MXLU_E_WORKSPACE;
    if (report) std::memset(report, 0, sizeof(*report));
    if (n == 0 || nrhs == 0) {
        if (report) report->converged = 1;
        return 0;
    }
    if (int rc = check_device()) return rc;
    clear_error();
    ASource src;
    src.A = A;
    src.lda = lda;
    src.n = n;
    return mxp_impl(n, nrhs, src, B, ldb, X, ldx, work, work_bytes, ipiv, opts, report,
                    (hipStream_t)stream);
}

extern "C" int mxp_solve_seeded(int64_t n, uint64_t seed, uint64_t stream_id, int dominant,
                                int64_t nrhs, const double *B, int64_t ldb, double *X,
                                int64_t ldx, void *work, size_t work_bytes, int32_t *ipiv,
                                const mxp_opts *opts, mxp_report *report, void *stream) {
    if (n < 0 || n > 0x7fffffff) return -1;
    if (dominant != 0 && dominant != 1) return -4;
    if (nrhs < 0) return -5;
    if (int rc = mxp_check(n, nrhs, B, ldb, X, ldx, work, ipiv, opts)) return rc - 1;
    if (n > 0 && work_bytes < mxp_workspace_bytes(n, n, opts)) return MXLU_E_WORKSPACE;
    if (report) std::memset(report, 0, sizeof(*report));
    if (n == 0 || nrhs == 0) {
        if (report) report->converged = 1;
        return 0;
    }
    if (int rc = check_device()) return rc;
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    Scratch scratch(s);
    ASource src;
    src.n = n;
    src.key = gen_key(seed, stream_id);
    if (dominant) {
        double *diag = scratch.alloc_n<double>((size_t)n);
        if (!diag) return MXLU_E_NOMEM;
        MXLU_TRY(gen_dominant_diag(n, src.key, diag, s));
        src.diag = diag;
    }
    return mxp_impl(n, nrhs, src, B, ldb, X, ldx, work, work_bytes, ipiv, opts, report, s);
}
