// Per-phase event timing (internal interface; see profile.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace mxlu {

// Phase ids, in the order reported by mxlu_profile_read.
enum {
    kPhasePfact = 0,     // panel factorization (leaves, in-panel swaps/TRSM/GEMM)
    kPhaseSwap = 1,      // interchanges on the columns outside the panel
    kPhaseTrsm = 2,      // U12 = L11^-1 A12
    kPhaseGemm = 3,      // trailing update A22 -= L21 U12 (work = flops)
    kPhaseSolve = 4,     // lu_solve
    kPhaseConvert = 5,   // FP64 -> low precision
    kPhaseLpFactor = 6,  // low-precision LU
    kPhaseRefine = 7,    // refinement loop
    kPhaseLpSchur = 8,   // low-precision trailing update (work = algorithmic bytes)
    kPhaseCount = 9
};

bool profiling_enabled();
// Destroys the pooled timing events (pending intervals are dropped).
int profile_release();
// Panel step index recorded with the intervals opened from now on by the
// calling thread (-1: none).
void profile_set_step(int64_t step);

class PhaseScope {
  public:
    PhaseScope(int phase, hipStream_t s, double work = 0.0);
    ~PhaseScope();
    PhaseScope(const PhaseScope &) = delete;
    PhaseScope &operator=(const PhaseScope &) = delete;

  private:
    hipStream_t s_;
    hipEvent_t start_ = nullptr;
    int phase_ = 0;
    int64_t step_ = -1;
    double work_ = 0.0;
};

}  // namespace mxlu
