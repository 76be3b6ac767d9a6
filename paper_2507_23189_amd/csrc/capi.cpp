// Error reporting and version entry points of the C ABI.
#include "common.hpp"

#include <mutex>

namespace mcmie {

static thread_local char g_msg[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = '\0'; }

int device_cu_count(int *out)
{
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    MC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MC_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int n = 0;
        MC_HIP_CHECK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        cached[dev] = n > 0 ? n : 1;
    }
    *out = cached[dev];
    return MC_OK;
}

}  // namespace mcmie

extern "C" const char *mc_last_error(void) { return mcmie::g_msg; }

extern "C" int mc_version(void) { return 400; }   // 0.4.0
