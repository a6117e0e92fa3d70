// Internal helpers shared by the library's HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mxlu.h"

namespace mxlu {

// Record the last runtime failure of the calling thread (mxlu_last_error).
void set_error(const char *what, hipError_t e);
void set_error_msg(const char *msg);
void clear_error();

// Returns MXLU_E_NODEV when no device is visible, else 0.
int check_device();

// Stream-ordered scratch memory owned by one call; freed by the destructor.
class Scratch {
  public:
    explicit Scratch(hipStream_t s) : stream_(s) {}
    ~Scratch();
    // Returns nullptr and records the error on failure.
    void *alloc(size_t bytes);
    template <class T> T *alloc_n(size_t count) {
        return static_cast<T *>(alloc(count * sizeof(T)));
    }

  private:
    hipStream_t stream_;
    void *ptrs_[32] = {};
    int count_ = 0;
};

}  // namespace mxlu

#define MXLU_HIP_TRY(call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) {                              \
            ::mxlu::set_error(#call, e_);                    \
            return MXLU_E_HIP;                               \
        }                                                    \
    } while (0)

#define MXLU_LAUNCH_CHECK() MXLU_HIP_TRY(hipGetLastError())

#define MXLU_TRY(x)              \
    do {                         \
        int rc_ = (x);           \
        if (rc_) return rc_;     \
    } while (0)

// Offsets are 64-bit everywhere: n^2 exceeds 2^31 for the larger workloads.
#define MXLU_AT(ptr, i, j, ld) ((ptr)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

// Wait until every vector-memory load of the wave has returned (vmcnt(0)).
// Used before a software-pipelined main loop whose accumulators were loaded
// in the prologue: without it, the compiler's wait for those loads lands
// inside the loop on the first use of each accumulator, where the in-order
// counter also makes it wait for the next chunk's prefetch every iteration.
__device__ __forceinline__ void retire_vector_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }
