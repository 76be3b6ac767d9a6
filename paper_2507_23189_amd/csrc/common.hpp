// Host-side plumbing shared by the library's entry points: the thread-local
// error message behind mc_last_error(), HIP status checks, device queries.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "mcmie.h"

namespace mcmie {

// Records a formatted message for mc_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);

// Clears the calling thread's message (start of every entry point).
void clear_error();

#define MC_HIP_CHECK(expr)                                                          \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::mcmie::fail(MC_EDEVICE, "%s failed: %s", #expr,                \
                                 hipGetErrorString(e_));                            \
    } while (0)

// Compute units of the current device (cached per device).
int device_cu_count(int *out);

}  // namespace mcmie
