// Optional per-phase timing with HIP events on the work's own stream.
//
// When enabled, each phase of the factorization (PFACT, SWAP, DTRSM, DGEMM
// and the solve; Sec. III-A.1 lists these phases and models the time of each
// step as set by the slowest of them) is bracketed by a pair of events; the
// totals are read back after the caller's work has completed.  Disabled, the
// scopes cost one branch.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "profile.h"

namespace mxlu {

namespace {
struct Pending {
    hipEvent_t start, stop;
    int phase;
    int64_t step;
    double work;
};
struct Done {
    int phase;
    int64_t step;
    double ms, work;
};
std::mutex g_mu;
bool g_enabled = false;
std::vector<Pending> g_pending;
std::vector<Done> g_done;      // resolved intervals since the last reset
std::vector<hipEvent_t> g_free;
thread_local int64_t g_step = -1;

// Resolves the pending intervals into g_done and the per-phase sums.
int resolve_locked() {
    for (auto &p : g_pending) {
        if (hipEventSynchronize(p.stop) != hipSuccess) {
            set_error("hipEventSynchronize", hipGetLastError());
            return MXLU_E_HIP;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.start, p.stop) != hipSuccess) {
            set_error("hipEventElapsedTime", hipGetLastError());
            return MXLU_E_HIP;
        }
        g_done.push_back({p.phase, p.step, (double)t, p.work});
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    return 0;
}

hipEvent_t get_event() {
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}
}  // namespace

bool profiling_enabled() { return g_enabled; }

void profile_set_step(int64_t step) { g_step = step; }

int profile_release() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &p : g_pending) {
        (void)hipEventSynchronize(p.stop);
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    for (hipEvent_t e : g_free) (void)hipEventDestroy(e);
    g_free.clear();
    (void)hipGetLastError();
    return 0;
}

PhaseScope::PhaseScope(int phase, hipStream_t s, double work) : s_(s) {
    if (!g_enabled) return;
    std::lock_guard<std::mutex> lk(g_mu);
    start_ = get_event();
    if (!start_) return;
    phase_ = phase;
    step_ = g_step;
    work_ = work;
    if (hipEventRecord(start_, s_) != hipSuccess) {
        (void)hipGetLastError();
        g_free.push_back(start_);
        start_ = nullptr;
    }
}

PhaseScope::~PhaseScope() {
    if (!start_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t stop = get_event();
    if (!stop || hipEventRecord(stop, s_) != hipSuccess) {
        (void)hipGetLastError();
        g_free.push_back(start_);
        if (stop) g_free.push_back(stop);
        return;
    }
    g_pending.push_back({start_, stop, phase_, step_, work_});
}

}  // namespace mxlu

using namespace mxlu;

extern "C" int mxlu_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = on != 0;
    return 0;
}

extern "C" int mxlu_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &p : g_pending) {
        (void)hipEventSynchronize(p.stop);
        g_free.push_back(p.start);
        g_free.push_back(p.stop);
    }
    g_pending.clear();
    g_done.clear();
    return 0;
}

extern "C" int mxlu_profile_read(double *ms, double *work, int64_t *count, int nphase) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (int rc = resolve_locked()) return rc;
    double sm[kPhaseCount] = {}, sw[kPhaseCount] = {};
    int64_t sc[kPhaseCount] = {};
    for (const Done &d : g_done) {
        sm[d.phase] += d.ms;
        sw[d.phase] += d.work;
        sc[d.phase] += 1;
    }
    for (int i = 0; i < nphase && i < kPhaseCount; ++i) {
        if (ms) ms[i] = sm[i];
        if (work) work[i] = sw[i];
        if (count) count[i] = sc[i];
    }
    return 0;
}

extern "C" int64_t mxlu_profile_intervals(int phase, int64_t *step, double *ms, double *work,
                                          int64_t cap) {
    if (phase < 0 || phase >= kPhaseCount || cap < 0) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (resolve_locked()) return MXLU_E_HIP;
    int64_t k = 0;
    for (const Done &d : g_done) {
        if (d.phase != phase) continue;
        if (k < cap) {
            if (step) step[k] = d.step;
            if (ms) ms[k] = d.ms;
            if (work) work[k] = d.work;
        }
        ++k;
    }
    return k;
}
