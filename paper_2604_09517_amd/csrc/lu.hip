// Host driver of the FP64 path: lu_factor and lu_solve (Sec. III-A.1).
//
// lu_factor runs the right-looking blocked algorithm: for each panel of width
// nb, PFACT (recursive panel factorization whose leaves are the
// multi-workgroup pivoting kernel and whose inner nodes are TRSM + MFMA GEMM
// updates inside the panel), SWAP of the panel's interchanges on the columns
// left and right of it, DTRSM for the block row U12, and the MFMA DGEMM
// trailing update A22 -= L21 U12.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>

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
            MXLU_TRY(swap_compose(f.ipiv, f.ibase + c, (int)w, f.ibase + f.m, f.moves, f.s));
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

// Test hook (mxlu_debug_expire_waits): panel exchanges start expired.
std::atomic<int> g_expire_waits{0};

int alloc_panel_exchange(Scratch &scratch, int64_t n, PanelExchange *ex, hipStream_t s) {
    const size_t slot_words = (size_t)2 * kMaxGroups * (2 * kLeafW + 4);
    const size_t rowj_words = (size_t)2 * 2 * kLeafW;
    ex->slots = scratch.alloc_n<uint64_t>(slot_words);
    ex->rowj = scratch.alloc_n<uint64_t>(rowj_words);
    ex->flags = scratch.alloc_n<int>(4);
    ex->group_cap = 0;
    (void)n;
    if (!ex->slots || !ex->rowj || !ex->flags) return MXLU_E_NOMEM;
    // sequence number 0 is never current: zeroed words never match
    MXLU_HIP_TRY(hipMemsetAsync(ex->slots, 0, sizeof(uint64_t) * slot_words, s));
    MXLU_HIP_TRY(hipMemsetAsync(ex->rowj, 0, sizeof(uint64_t) * rowj_words, s));
    MXLU_HIP_TRY(hipMemsetAsync(ex->flags, 0, sizeof(int) * 4, s));
    if (g_expire_waits.load())   // as if a wait had already expired
        MXLU_HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(ex->flags + 1), 1, 1, s));
    return 0;
}
}  // namespace mxlu

namespace {

// Look-ahead depth of lu_factor (0 or 1; Sec. IV-B runs HPL with depth 1).
std::atomic<int> g_lookahead{1};

// Streams of the depth-1 look-ahead: the next panel is factored on `panel`
// while part of the trailing update runs on `update`.  Both carry a CU mask
// so that the two never compete for a CU: the panel's leaf kernel needs all
// of its workgroups resident at once, and it gets CUs that no update
// workgroup holds.  The panel gets mask bits [0, cus/4): the KFD spreads
// mask bits round-robin over the XCDs and then over the shader engines of
// each, so these are the first two CUs of every shader engine (present
// however the engines are harvested); a driver that numbers the bits
// XCD-major would give it two whole XCDs instead, also cus/4 CUs.  Created
// once per device with the default priority; released by mxlu_release (also
// run at process exit, before the HIP runtime's own teardown).
struct OverlapStreams {
    hipStream_t panel = nullptr, update = nullptr;
    int panel_cus = 0, update_cus = 0;
    hipStream_t side = nullptr;   // unmasked (the mixed-precision look-ahead)
};

constexpr int kMaxDev = 64;
std::mutex g_streams_mu;
OverlapStreams g_streams[kMaxDev];
bool g_streams_tried[kMaxDev] = {};
bool g_atexit_registered = false;

// One look-ahead factorization at a time per process: the masked streams and
// their CUs are shared by every call.
std::mutex g_lookahead_mu;

void release_streams() {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    for (int d = 0; d < kMaxDev; ++d) {
        if (g_streams[d].panel) (void)hipStreamDestroy(g_streams[d].panel);
        if (g_streams[d].update) (void)hipStreamDestroy(g_streams[d].update);
        if (g_streams[d].side) (void)hipStreamDestroy(g_streams[d].side);
        g_streams[d] = {};
        g_streams_tried[d] = false;
    }
    (void)hipGetLastError();
}

void release_at_exit() { (void)mxlu_release(); }

const OverlapStreams *device_streams() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_streams_mu);
    if (!g_streams_tried[dev]) {
        g_streams_tried[dev] = true;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        const int np = mxlu_plan_panel_cus(cus);
        if (np > 0) {
            uint32_t pm[32] = {}, um[32] = {};
            for (int i = 0; i < cus; ++i) (i < np ? pm : um)[i / 32] |= 1u << (i % 32);
            const uint32_t words = (uint32_t)((cus + 31) / 32);
            hipStream_t a = nullptr, b = nullptr;
            if (hipExtStreamCreateWithCUMask(&a, words, pm) == hipSuccess &&
                hipExtStreamCreateWithCUMask(&b, words, um) == hipSuccess) {
                g_streams[dev].panel = a;
                g_streams[dev].update = b;
                g_streams[dev].panel_cus = np;
                g_streams[dev].update_cus = cus - np;
            } else {
                if (a) (void)hipStreamDestroy(a);
            }
        }
        hipStream_t c = nullptr;
        if (hipStreamCreateWithFlags(&c, hipStreamNonBlocking) == hipSuccess)
            g_streams[dev].side = c;
        if (!g_atexit_registered && (g_streams[dev].panel || g_streams[dev].side)) {
            // registered after the HIP runtime started, so it runs before the
            // runtime's own exit-time teardown
            g_atexit_registered = std::atexit(release_at_exit) == 0;
        }
        (void)hipGetLastError();
    }
    return &g_streams[dev];
}

const OverlapStreams *overlap_streams() {
    const OverlapStreams *ov = device_streams();
    return ov && ov->panel ? ov : nullptr;
}

// Joins the look-ahead streams back into the factorization stream when it
// goes out of scope (also on an error return, so that no work of the call is
// still running when its scratch memory is released).
class ForkJoin {
  public:
    ForkJoin(hipStream_t s, const OverlapStreams *ov) : s_(s), ov_(ov) {}
    ~ForkJoin() {
        if (!active_) return;
        (void)hipEventRecord(ev_[1], ov_->panel);
        (void)hipStreamWaitEvent(s_, ev_[1], 0);
        (void)hipEventRecord(ev_[2], ov_->update);
        (void)hipStreamWaitEvent(s_, ev_[2], 0);
        for (hipEvent_t e : ev_) (void)hipEventDestroy(e);
    }
    int create() {
        for (hipEvent_t &e : ev_)
            MXLU_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        active_ = true;
        return 0;
    }
    // the look-ahead streams start after everything enqueued so far on s
    int fork() {
        MXLU_HIP_TRY(hipEventRecord(ev_[0], s_));
        MXLU_HIP_TRY(hipStreamWaitEvent(ov_->panel, ev_[0], 0));
        MXLU_HIP_TRY(hipStreamWaitEvent(ov_->update, ev_[0], 0));
        return 0;
    }
    // s continues after everything enqueued so far on the panel stream
    int join_panel() {
        MXLU_HIP_TRY(hipEventRecord(ev_[1], ov_->panel));
        MXLU_HIP_TRY(hipStreamWaitEvent(s_, ev_[1], 0));
        return 0;
    }
    // s continues after everything enqueued so far on the update stream
    int join_update() {
        MXLU_HIP_TRY(hipEventRecord(ev_[2], ov_->update));
        MXLU_HIP_TRY(hipStreamWaitEvent(s_, ev_[2], 0));
        return 0;
    }

  private:
    hipStream_t s_;
    const OverlapStreams *ov_;
    hipEvent_t ev_[3] = {};
    bool active_ = false;
};

// Leaf workgroups allowed on the panel stream: 7/8 of its CUs, so that a
// leaf still fits when a few of them are unavailable.
int lookahead_group_cap(int panel_cus) { return panel_cus * 7 / 8; }

// Depth-1 look-ahead applies when every trailing update can be split at the
// next panel's columns into direct-kernel updates (sizes multiples of 128),
// the first panel's leaf fits on all CUs (it runs on the caller's stream)
// and every later panel's leaf -- at most n - nb rows -- fits within the
// group cap of the panel stream.  Host arithmetic only.
bool lookahead_plan(int64_t n, int64_t nb, const LeafDevice &all, int panel_cus) {
    if (panel_cus <= 0 || nb % 128 != 0 || n % 128 != 0 || n <= nb) return false;
    LeafDevice capped = all;
    capped.cap = lookahead_group_cap(panel_cus);
    int64_t R = 0, G = 0;
    return leaf_plan(n, all, &R, &G) != kLeafNone && leaf_plan(n - nb, capped, &R, &G) != kLeafNone;
}

bool lookahead_fits(int64_t n, int64_t nb, const double *A, int64_t lda,
                    const OverlapStreams *ov) {
    if (!ov || n <= nb || !gemm_f64_update_ok(n - nb, n - nb, nb, A, lda)) return false;
    LeafDevice all;
    if (leaf_device_f64(0, &all)) {
        (void)hipGetLastError();
        clear_error();
        return false;
    }
    return lookahead_plan(n, nb, all, ov->panel_cus);
}

// Columns of the remaining update given to the update stream while the next
// panel is factored: about 1.5x what its CUs finish in the panel's expected
// time (the leaves take ~7 us per column, the update kernel ~0.24 TFLOP/s per
// CU).  The rest runs on all CUs once the panel is done, alongside the tail
// of this part, so erring high costs little and erring low leaves the update
// CUs idle until the panel ends.
int64_t lookahead_split(int64_t nt, int64_t kb, int64_t kb1, const OverlapStreams *ov) {
    constexpr double kPanelSecPerCol = 7.0e-6, kUpdateFlopsPerCu = 2.4e11;
    const double flops = 1.5 * kPanelSecPerCol * (double)kb1 * kUpdateFlopsPerCu * ov->update_cus;
    const int64_t rest = nt - kb1;
    int64_t n1 = (int64_t)(flops / (2.0 * (double)nt * (double)kb));
    n1 = (n1 + 127) / 128 * 128;
    return std::min(rest, std::max<int64_t>(128, n1));
}

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
    // the deferred interchanges left of the panels: two row maps and one
    // panel's rows below it
    int32_t *perm_q = scratch.alloc_n<int32_t>((size_t)n);
    int32_t *perm_r = scratch.alloc_n<int32_t>((size_t)n);
    double *rowsT = n > nb ? scratch.alloc_n<double>((size_t)(n - nb) * (size_t)nb) : nullptr;
    if (!perm_q || !perm_r || (n > nb && !rowsT)) return MXLU_E_NOMEM;

    const OverlapStreams *ov =
        g_lookahead.load() > 0 ? overlap_streams() : nullptr;
    const bool la = lookahead_fits(n, nb, A, lda, ov);
    std::unique_lock<std::mutex> la_lock(g_lookahead_mu, std::defer_lock);
    if (la) la_lock.lock();   // held until the factorization has completed
    ForkJoin fj(s, ov);
    // panels factored on the panel stream may use only its CUs; those on the
    // caller's stream (the first one, and every one at depth 0) use all
    PanelExchange ex_ahead = ex;
    if (la) {
        MXLU_TRY(fj.create());
        ex_ahead.group_cap = lookahead_group_cap(ov->panel_cus);
    }

    bool ahead = false;  // the current panel was factored during the previous update
    for (int64_t k0 = 0; k0 < n; k0 += nb) {
        const int64_t kb = std::min(nb, n - k0);
        const int64_t m = n - k0, c1 = k0 + kb;
        profile_set_step(k0 / nb);
        if (!ahead) {   // PFACT
            PhaseScope ph(kPhasePfact, s, (double)m * kb * 8.0);
            MXLU_TRY(panel_factor<double>(&MXLU_AT(A, k0, k0, lda), lda, m, kb, k0, ipiv, ex, moves,
                                     s));
        }
        ahead = false;
        if (c1 < n) {   // SWAP on the columns right of the panel (those left of it: below)
            PhaseScope ph(kPhaseSwap, s, 32.0 * kb * (double)(n - c1));
            MXLU_TRY(laswp_f64(A, lda, n, ipiv, k0, (int)kb, c1, n - c1, c1, 0, moves, s));
        }
        if (c1 >= n) continue;
        const int64_t nt = n - c1;
        double *L21 = &MXLU_AT(A, c1, k0, lda), *U12 = &MXLU_AT(A, k0, c1, lda);
        const bool direct = la || gemm_f64_update_ok(nt, nt, kb, L21, lda);
        {   // DTRSM: U12 = L11^-1 A12 (then, for the direct kernel, -U12^T packed)
            PhaseScope ph(kPhaseTrsm, s, (double)kb * (kb - 1) * (double)nt);
            MXLU_TRY(PanelOps<double>::trsm(kb, nt, &MXLU_AT(A, k0, k0, lda), lda, U12, lda, s));
            if (direct) MXLU_TRY(pack_neg_transpose_f64(kb, nt, U12, lda, Bn, ldbn, s));
        }
        if (!la) {   // DGEMM: A22 -= L21 U12
            PhaseScope ph(kPhaseGemm, s, 2.0 * (double)nt * (double)nt * (double)kb);
            if (direct)
                MXLU_TRY(gemm_f64_update(nt, nt, kb, L21, lda, Bn, ldbn, &MXLU_AT(A, c1, c1, lda),
                                       lda, s));
            else
                MXLU_TRY(gemm_f64_sub(nt, nt, kb, L21, lda, U12, lda, &MXLU_AT(A, c1, c1, lda),
                                      lda, s, true));
            continue;
        }
        // Look-ahead: update the next panel's columns first, then factor that
        // panel on the panel stream while the update stream takes the next n1
        // columns; the remaining columns follow on all CUs once the panel is
        // done.  The three updates and the panel touch disjoint columns of A;
        // the next SWAP (which reads them all) waits for all of them.
        const int64_t kb1 = std::min(nb, nt);
        {
            PhaseScope ph(kPhaseGemm, s, 2.0 * (double)nt * (double)kb1 * (double)kb);
            MXLU_TRY(gemm_f64_update(nt, kb1, kb, L21, lda, Bn, ldbn, &MXLU_AT(A, c1, c1, lda), lda,
                                   s));
        }
        MXLU_TRY(fj.fork());
        {
            profile_set_step(k0 / nb + 1);   // the next step's panel
            PhaseScope ph(kPhasePfact, ov->panel, (double)nt * kb1 * 8.0);
            MXLU_TRY(panel_factor<double>(&MXLU_AT(A, c1, c1, lda), lda, nt, kb1, c1, ipiv,
                                          ex_ahead, moves, ov->panel));
        }
        profile_set_step(k0 / nb);
        const int64_t n1 = nt > kb1 ? lookahead_split(nt, kb, kb1, ov) : 0;
        if (n1 > 0) {
            PhaseScope ph(kPhaseGemm, ov->update, 2.0 * (double)nt * (double)n1 * (double)kb);
            MXLU_TRY(gemm_f64_update(nt, n1, kb, L21, lda, Bn + kb1, ldbn,
                                   &MXLU_AT(A, c1, c1 + kb1, lda), lda, ov->update));
        }
        MXLU_TRY(fj.join_panel());
        const int64_t n2 = nt - kb1 - n1, j2 = kb1 + n1;
        if (n2 > 0) {
            PhaseScope ph(kPhaseGemm, s, 2.0 * (double)nt * (double)n2 * (double)kb);
            MXLU_TRY(gemm_f64_update(nt, n2, kb, L21, lda, Bn + j2, ldbn,
                                   &MXLU_AT(A, c1, c1 + j2, lda), lda, s));
        }
        MXLU_TRY(fj.join_update());
        ahead = true;
    }
    profile_set_step(-1);
    {   // the interchanges of every step on the L columns left of its panel,
        // applied once now that no step reads those columns any more
        PhaseScope ph(kPhaseSwap, s, 32.0 * (double)n * (double)n / 2.0);
        MXLU_TRY(laswp_left_deferred_f64(A, lda, n, nb, ipiv, moves, perm_q, perm_r, rowsT, s));
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

namespace mxlu {
// The mixed-precision look-ahead factors its panels on the unmasked side
// stream: its panel kernels need no co-resident workgroups, and the update
// it overlaps is bound by memory parallelism, which a CU mask would cut
// (measured at N = 131072, NB = 1024: 654 TFLOP/s with the side stream
// against 477 with the panel on the masked quarter and 566 with the update
// also masked to the other CUs).
bool lp_ahead_streams(AheadStreams *out, std::unique_lock<std::mutex> *lk) {
    if (g_lookahead.load() <= 0) return false;
    const OverlapStreams *ov = device_streams();
    if (!ov || !ov->side) return false;
    out->panel = ov->side;
    *lk = std::unique_lock<std::mutex>(g_lookahead_mu);
    return true;
}
}  // namespace mxlu

extern "C" int mxlu_set_lookahead(int depth) {
    if (depth < 0 || depth > 1) return -1;
    g_lookahead.store(depth);
    return 0;
}

extern "C" int mxlu_debug_expire_waits(int on) {
    if (on != 0 && on != 1) return -1;
    mxlu::g_expire_waits.store(on);
    return 0;
}

extern "C" int mxlu_panel_factor_f64(int64_t m, int64_t nb, double *P, int64_t ldp,
                                     int32_t *ipiv, void *stream) {
    if (m < 0) return -1;
    if (nb < 0 || nb > m || nb > 1024) return -2;
    if (m > 0 && nb > 0 && !P) return -3;
    if (ldp < std::max<int64_t>(1, m)) return -4;
    if (nb > 0 && !ipiv) return -5;
    if (m > 0x7fffffff) return -1;
    if (m == 0 || nb == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    Scratch scratch(s);
    PanelExchange ex;
    MXLU_TRY(alloc_panel_exchange(scratch, m, &ex, s));
    int *moves = scratch.alloc_n<int>(kSwapMovesInts);
    if (!moves) return MXLU_E_NOMEM;
    {
        PhaseScope ph(kPhasePfact, s, (double)m * nb * 8.0);
        MXLU_TRY(panel_factor<double>(P, ldp, m, nb, 0, ipiv, ex, moves, s));
    }
    int flags[4] = {0, 0, 0, 0};
    MXLU_HIP_TRY(hipMemcpyAsync(flags, ex.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    MXLU_HIP_TRY(hipStreamSynchronize(s));
    if (flags[1]) {
        set_error_msg("mxlu_panel_factor_f64: panel grid barrier wait expired");
        return MXLU_E_TIMEOUT;
    }
    return flags[0];
}

extern "C" int mxlu_release(void) {
    release_streams();
    return mxlu::profile_release();
}

extern "C" int mxlu_plan_panel_cus(int cus) {
    if (cus < 128 || cus > 1024) return 0;
    const int np = cus / 4;
    return np % 32 == 0 ? np : 0;
}

extern "C" int mxlu_plan_panel_leaf(int64_t m, int cap, int cus, int occ_reg1, int occ_reg2,
                                    int64_t lds_budget, int elem_bytes, int64_t *rows_per_group,
                                    int64_t *groups) {
    if (cus <= 0 || cap < 0 || (elem_bytes != 4 && elem_bytes != 8)) return -1;
    LeafDevice d{cap, cus, occ_reg1, occ_reg2, elem_bytes, lds_budget};
    int64_t R = 0, G = 0;
    const int form = leaf_plan(m, d, &R, &G);
    if (rows_per_group) *rows_per_group = R;
    if (groups) *groups = G;
    return form;
}

extern "C" int mxlu_plan_lookahead(int64_t n, int64_t nb, int cus, int occ_reg1, int occ_reg2,
                                   int64_t lds_budget) {
    const int np = mxlu_plan_panel_cus(cus);
    LeafDevice all{0, cus, occ_reg1, occ_reg2, 8, lds_budget};
    return lookahead_plan(n, nb, all, np) ? np : 0;
}

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

namespace {

int solve_args(int64_t n, int64_t nrhs, const double *LU, int64_t lda, const int32_t *ipiv,
               const double *B, int64_t ldb, int trans) {
    if (n < 0) return -1;
    if (nrhs < 0) return -2;
    if (n > 0 && !LU) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && !ipiv) return -5;
    if (n > 0 && nrhs > 0 && !B) return -6;
    if (ldb < std::max<int64_t>(1, n)) return -7;
    if (trans != 0 && trans != 1) return -8;
    if (n > 0x7fffffff) return -1;
    return 0;
}

// The solves of lu_solve with caller-provided device scratch: perm (n int32)
// and Y (n x min(16, nrhs) doubles, leading dimension n).
int solve_impl(int64_t n, int64_t nrhs, const double *LU, int64_t lda, const int32_t *ipiv,
               double *B, int64_t ldb, int trans, hipStream_t s, int32_t *perm, double *Y) {
    PhaseScope ph(kPhaseSolve, s, 8.0 * (double)n * (double)n);
    MXLU_TRY(perm_from_ipiv(n, ipiv, perm, s));
    // Work on strips of at most 16 right-hand sides.
    const int64_t bs = 256;
    const int64_t ldy = n;
    for (int64_t r0 = 0; r0 < nrhs; r0 += 16) {
        const int64_t nr = std::min<int64_t>(16, nrhs - r0);
        double *Bc = B + (size_t)r0 * (size_t)ldb;
        if (trans == 0) {
            MXLU_TRY(gather_rows_f64(n, nr, perm, Bc, ldb, Y, ldy, s));
            // L y = P b: diagonal blocks forward, updates below
            for (int64_t b0 = 0; b0 < n; b0 += bs) {
                const int64_t bb = std::min(bs, n - b0);
                if (nr == 1)
                    MXLU_TRY(trsv_block_f64((int)bb, true, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, s));
                else
                    MXLU_TRY(trsm_llnu_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy,
                                           s));
                if (b0 + bb < n && nr == 1)
                    MXLU_TRY(gemv_f64_sub(n - b0 - bb, bb, &MXLU_AT(LU, b0 + bb, b0, lda), lda, Y + b0,
                                          Y + b0 + bb, s));
                else if (b0 + bb < n)
                    MXLU_TRY(gemm_f64_sub(n - b0 - bb, nr, bb, &MXLU_AT(LU, b0 + bb, b0, lda), lda,
                                     Y + b0, ldy, Y + b0 + bb, ldy, s));
            }
            // U x = y: diagonal blocks backward, updates above
            const int64_t nblk = (n + bs - 1) / bs;
            for (int64_t bi = nblk - 1; bi >= 0; --bi) {
                const int64_t b0 = bi * bs, bb = std::min(bs, n - b0);
                if (nr == 1)
                    MXLU_TRY(trsv_block_f64((int)bb, false, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, s));
                else
                    MXLU_TRY(trsm_lunn_f64((int)bb, nr, &MXLU_AT(LU, b0, b0, lda), lda, Y + b0, ldy,
                                           s));
                if (b0 > 0 && nr == 1)
                    MXLU_TRY(gemv_f64_sub(b0, bb, &MXLU_AT(LU, 0, b0, lda), lda, Y + b0, Y, s));
                else if (b0 > 0)
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

// Scratch of lu_solve_noalloc: Y (kNoAllocMaxN x 16 doubles) then perm
// (kNoAllocMaxN int32), one copy per device, held until the process ends.
constexpr int64_t kNoAllocMaxN = 65536;
constexpr size_t kNoAllocYBytes = (size_t)kNoAllocMaxN * 16 * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocYBytes + (size_t)kNoAllocMaxN * sizeof(int32_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDev] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device (the array's name is only a host-side stand-in).
int noalloc_scratch(void **out) {
    int dev = 0;
    MXLU_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) {
        set_error_msg("lu_solve_noalloc: device index out of range");
        return MXLU_E_NODEV;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        MXLU_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return 0;
}

}  // namespace

extern "C" int lu_solve(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                        const int32_t *ipiv, double *B, int64_t ldb, int trans, void *stream) {
    if (int rc = solve_args(n, nrhs, LU, lda, ipiv, B, ldb, trans)) return rc;
    if (n == 0 || nrhs == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    hipStream_t s = (hipStream_t)stream;
    Scratch scratch(s);
    int32_t *perm = scratch.alloc_n<int32_t>((size_t)n);
    double *Y = scratch.alloc_n<double>((size_t)n * (size_t)std::min<int64_t>(16, nrhs));
    if (!perm || !Y) return MXLU_E_NOMEM;
    return solve_impl(n, nrhs, LU, lda, ipiv, B, ldb, trans, s, perm, Y);
}

extern "C" int lu_solve_noalloc(int64_t n, int64_t nrhs, const double *LU, int64_t lda,
                                const int32_t *ipiv, double *B, int64_t ldb, int trans,
                                void *stream) {
    if (int rc = solve_args(n, nrhs, LU, lda, ipiv, B, ldb, trans)) return rc;
    if (n > kNoAllocMaxN) {
        set_error_msg("lu_solve_noalloc: n exceeds the 65536 rows its static scratch holds");
        return MXLU_E_WORKSPACE;
    }
    if (n == 0 || nrhs == 0) return 0;
    if (int rc = check_device()) return rc;
    clear_error();
    void *base = nullptr;
    MXLU_TRY(noalloc_scratch(&base));
    double *Y = static_cast<double *>(base);
    int32_t *perm = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(base) + kNoAllocYBytes);
    return solve_impl(n, nrhs, LU, lda, ipiv, B, ldb, trans, (hipStream_t)stream, perm, Y);
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
