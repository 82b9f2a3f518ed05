// sb_forward_noalloc: the forward pass with its working arrays in a fixed device array of the
// library instead of the caller's scratch buffer, for callers that cannot allocate device
// memory.  The array's device address is taken once per device with hipGetSymbolAddress;
// host code never passes the array's name itself to a kernel or a copy.
#include "sb_plan.h"

#include <mutex>

namespace sb {
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// The working arrays of sb_forward_noalloc (one copy per device, held until the process ends).
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_mutex;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up on its first use.
sb_status scratch_address(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SB_EUNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return fail(SB_EHIP, "static scratch misaligned");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return SB_OK;
}

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" sb_status sb_forward_noalloc(sb_plan *p, const void *const *delta, double *zeta, void *stream) {
    if (!p) return fail(SB_EINVAL, "null plan");
    if (!delta || !zeta) return fail(SB_EINVAL, "null pointer");
    if (!p->persist) return fail(SB_EWORKSPACE, "persistent workspace not bound");
    if (p->timing) return fail(SB_ESTATE, "per-launch timing creates events; disable it (sb_profile) first");
    if (p->scratch_need > kNoAllocScratchBytes)
        return fail(SB_EWORKSPACE, "the plan needs " + std::to_string(p->scratch_need) +
                                       " bytes of scratch; sb_forward_noalloc holds at most " +
                                       std::to_string(kNoAllocScratchBytes) +
                                       " (lower it with sb_plan_set_scratch_limit or bind a scratch buffer)");
    char *ptr = nullptr;
    if (sb_status st = scratch_address(&ptr); st != SB_OK) return st;
    // run the ordinary forward with the plan's scratch layout placed in the static array
    char *bound = p->scratch;
    p->scratch = ptr;
    const sb_status st = forward(p, delta, zeta, static_cast<hipStream_t>(stream));
    p->scratch = bound;
    p->kept = false;   // whatever this call kept went to the static array
    return st;
}
