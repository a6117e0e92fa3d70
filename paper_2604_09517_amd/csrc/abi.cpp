// Status strings, error recording and stream-ordered scratch memory.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>

#include "common.h"

namespace mxlu {

// Test hook: byte value every new scratch buffer is filled with (-1: none).
static std::atomic<int> g_poison_scratch{-1};

static thread_local char g_last_error[512] = "";

void set_error(const char *what, hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what,
                  hipGetErrorString(e));
    // the failure is reported through the return code: do not leave it as
    // the runtime's pending error for the caller's next, unrelated HIP call
    (void)hipGetLastError();
}

void set_error_msg(const char *msg) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
}

void clear_error() { g_last_error[0] = '\0'; }

int check_device() {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        set_error_msg("no HIP device visible");
        return MXLU_E_NODEV;
    }
    return 0;
}

Scratch::~Scratch() {
    for (int i = count_ - 1; i >= 0; --i)
        if (ptrs_[i]) (void)hipFreeAsync(ptrs_[i], stream_);
}

void *Scratch::alloc(size_t bytes) {
    if (count_ >= 32) {
        set_error_msg("internal: too many scratch buffers");
        return nullptr;
    }
    void *p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes ? bytes : 16, stream_);
    if (e != hipSuccess) {
        set_error("hipMallocAsync", e);
        (void)hipGetLastError();
        return nullptr;
    }
    ptrs_[count_++] = p;
    const int poison = g_poison_scratch.load();
    if (poison >= 0 && hipMemsetAsync(p, poison, bytes ? bytes : 16, stream_) != hipSuccess) {
        set_error("hipMemsetAsync", hipGetLastError());
        return nullptr;
    }
    return p;
}

}  // namespace mxlu

extern "C" int mxlu_debug_poison_scratch(int byte) {
    if (byte < -1 || byte > 255) return -1;
    mxlu::g_poison_scratch.store(byte);
    return 0;
}

extern "C" const char *mxlu_status_string(int status) {
    switch (status) {
    case MXLU_OK: return "success";
    case MXLU_E_NODEV: return "no HIP device visible";
    case MXLU_E_HIP: return "HIP runtime error";
    case MXLU_E_NOMEM: return "size overflow or allocation failure";
    case MXLU_E_NOTCONV: return "iterative refinement did not converge";
    case MXLU_E_TIMEOUT: return "a kernel's bounded wait expired";
    case MXLU_E_WORKSPACE: return "workspace too small";
    default: break;
    }
    if (status > 0) return "exactly zero pivot (factorization completed, U singular)";
    if (status < 0 && status > -1000) return "invalid argument";
    return "unknown status";
}

extern "C" const char *mxlu_last_error(void) { return mxlu::g_last_error; }
