// crop_item_features for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The per-item statistics that crop_item_features keeps in a
// workspace the library allocates live here in a fixed array in every
// GPU's memory instead.
//
// The array's name is a host-side stand-in in host code: the device copy of
// the array is resolved once per device (noalloc_setup, called when a
// context is created with that device current) and only that resolved
// pointer is handed to kernels.  Every call on one GPU shares that GPU's
// array, which keeps the last call's contents; the statistics are cleared
// at the start of each call.  Calls that overlap on one GPU (other streams,
// other contexts) race on the array.
#include <mutex>

#include "api_util.hpp"
#include "crop_internal.hpp"

namespace crop {

constexpr size_t kScratchWords = (size_t)1 << 21;  // 8 MiB of item statistics
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_resolved[kMaxDevices];
hipError_t g_status[kMaxDevices];
uint32_t *g_ptr[kMaxDevices];

}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_resolved[device]) {
        void *p = nullptr;
        g_status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = g_status[device] == hipSuccess ? static_cast<uint32_t *>(p) : nullptr;
        g_resolved[device] = true;
    }
    return g_status[device];
}

static uint32_t *noalloc_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_resolved[device] ? g_ptr[device] : nullptr;
}

}  // namespace crop

using namespace crop;

crop_status crop_item_features_noalloc(crop_ctx *ctx, uint32_t prefix_T, float *feat)
{
    if (!ctx || !feat) return CROP_E_ARG;
    if (ctx->in.mode != Mode::Tx) return fail(ctx, CROP_E_STATE, "no transaction stream loaded");
    if (prefix_T > ctx->in.T) return fail(ctx, CROP_E_ARG, "prefix longer than the stream");
    const size_t words = item_stats_words(ctx->in.n_items, prefix_T);
    if (words > kScratchWords)
        return fail(ctx, CROP_E_CAPACITY,
                    "crop_item_features_noalloc: 8 n_items + prefix_T + 66 = " +
                        std::to_string(words) + " words exceeds its fixed 2^21-word workspace");
    uint32_t *ws = noalloc_ptr(ctx->device);
    if (!ws) return fail(ctx, CROP_E_HIP, "the fixed workspace of this device is not available");
    DeviceGuard g(ctx->device);
    CK(launch_zero32(ws, (uint32_t)words, ctx->stream));
    CK(launch_item_features(ctx->in.off, ctx->in.items, ctx->in.n_items, prefix_T, ws, feat,
                            ctx->stream));
    return CROP_OK;
}
