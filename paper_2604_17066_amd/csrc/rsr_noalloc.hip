// rsr_eval_unknown_noalloc: Stage-2 evaluation with its scratch memory (the
// list of unclassified samples and its counter) in a file-scope device array
// instead of the context's workspace, so the call never allocates.
//
// `scratch` exists once per device that loads the library and lives until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in symbol): each device's address is looked up
// once with hipGetSymbolAddress, with that device current, when the first
// context on the device is created, and every kernel argument uses that
// address.
#include <mutex>

#include "rsr_internal.h"

namespace rsr {
namespace {

// Counter (8 u64 slots, 64 bytes, of which the first is used) followed by the
// list of up to kNoAllocMaxSamples sample indices.
constexpr int64_t kCounterWords = 16;  // u32 words
constexpr size_t kScratchWords = static_cast<size_t>(kCounterWords) + kNoAllocMaxSamples;

__device__ __align__(256) uint32_t scratch[kScratchWords];

std::mutex g_lock;
void* g_addr[RSR_MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= RSR_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_lock);
    if (!g_addr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace rsr

extern "C" rsr_status rsr_eval_unknown_noalloc(rsr_ctx* ctx, const rsr_system* sys,
                                               const uint32_t* d_samples, int64_t N,
                                               const uint8_t* d_flags, int32_t which,
                                               uint8_t* d_Y, uint64_t* d_n_evaluated) {
    if (!ctx) return RSR_EINVAL;
    if (!sys || !d_samples || !d_Y) return rsr::set_error(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0) return rsr::set_error(ctx, RSR_EINVAL, "N must be > 0");
    if (N > rsr::kNoAllocMaxSamples)
        return rsr::set_error(ctx, RSR_EINVAL,
                              "N exceeds the scratch of rsr_eval_unknown_noalloc (2^22 samples)");
    if (which != RSR_UNKNOWN_ONLY && which != RSR_ALL)
        return rsr::set_error(ctx, RSR_EINVAL, "bad which");
    if (which == RSR_UNKNOWN_ONLY && !d_flags)
        return rsr::set_error(ctx, RSR_EINVAL, "d_flags is NULL with RSR_UNKNOWN_ONLY");
    if (sys->kind == RSR_SYS_HOST_CALLBACK)
        return rsr::set_error(ctx, RSR_EUNSUPPORTED,
                              "host-callback systems stage samples in allocated memory");
    if (!ctx->noalloc_scratch)
        return rsr::set_error(ctx, RSR_EHIP, "no scratch address for this device");
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return rsr::set_error(ctx, RSR_EHIP, "hipGetDevice");
    if (prev != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
        return rsr::set_error(ctx, RSR_EHIP, "hipSetDevice");
    uint64_t* counter = static_cast<uint64_t*>(ctx->noalloc_scratch);
    int32_t* list = reinterpret_cast<int32_t*>(static_cast<uint32_t*>(ctx->noalloc_scratch) +
                                               rsr::kCounterWords);
    const rsr::SegSrc seg = rsr::single_src(d_samples, N, const_cast<uint8_t*>(d_flags), d_Y);
    hipError_t e = hipSuccess;
    if (which == RSR_UNKNOWN_ONLY) {
        // The counter keeps the previous call's value: clear it with a kernel
        // (not a memset node, so the call can also be captured into a graph).
        e = rsr::launch_fill_u64(ctx->stream, counter, 1, 0);
        if (e == hipSuccess)
            e = rsr::launch_label(ctx->stream, seg, list, counter, ctx->cu_count * 16);
    }
    if (e == hipSuccess)
        e = rsr::launch_bfs(ctx->stream, sys, seg, list, counter, which, d_n_evaluated,
                            ctx->cu_count * 8);
    if (prev != ctx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return rsr::hip_error(ctx, e, "rsr_eval_unknown_noalloc launch");
    return RSR_OK;
}
