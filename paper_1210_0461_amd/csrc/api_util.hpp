// Internal helpers shared by the C ABI translation units (api.hip,
// batch.hip): errors, device selection, input placement, planning and run
// bracketing.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "crop_internal.hpp"

namespace crop {

constexpr uint32_t kMaxP = 8192;             // routing bins of one run (LDS histogram)
constexpr uint32_t kMaxPartitions = 1u << 20; // owners P
constexpr uint32_t kMaxGroupLog2 = 10;        // at most 1024 partitions in one bin
constexpr uint64_t kTermsPerBin = 30000;   // routed terms per bin the auto plan aims at
constexpr size_t kLdsBudget = 64 * 1024;   // enumeration kernels' staging budget
constexpr size_t kStageBudget = 150 * 1024; // scatter kernel: dynamic LDS in total
constexpr size_t kCuLds = 160 * 1024;       // LDS of one CU
constexpr uint64_t kSsMinBins = 2048;       // Space-Saving bins wanted for parallelism
constexpr size_t kSsLdsBudget = 80 * 1024;  // two summary workgroups per CU

crop_status fail(crop_ctx *c, crop_status s, const std::string &msg);
crop_status hip_fail(crop_ctx *c, hipError_t e, const char *what);

#define CK(expr)                                                   \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr);     \
    } while (0)

// Restores the context's hash parameters when a loop over instances, which
// routes with each instance's parameters in turn, ends or returns early.
struct HashGuard {
    crop_ctx *c;
    HashParams saved;
    explicit HashGuard(crop_ctx *ctx) : c(ctx), saved(ctx->hp) {}
    ~HashGuard() { c->hp = saved; }
    HashGuard(const HashGuard &) = delete;
    HashGuard &operator=(const HashGuard &) = delete;
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Copy n elements of T from `src` (host or device) into a host vector.
template <class T>
inline hipError_t fetch(std::vector<T> &dst, const T *src, size_t n, crop_mem where)
{
    dst.resize(n);
    if (n == 0) return hipSuccess;
    if (where == CROP_MEM_HOST) {
        std::memcpy(dst.data(), src, n * sizeof(T));
        return hipSuccess;
    }
    return hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
}

// Place an input array on the device: borrow it, or copy it into buf.
template <class T>
inline hipError_t place(const T *src, size_t n, crop_mem where, crop_own own, DevBuf &buf,
                 const T **out, hipStream_t s)
{
    if (own == CROP_OWN_BORROW) {
        *out = src;
        return hipSuccess;
    }
    hipError_t e = buf.ensure(n * sizeof(T) + 16);
    if (e != hipSuccess) return e;
    if (n) {
        e = hipMemcpyAsync(buf.p, src, n * sizeof(T),
                           where == CROP_MEM_HOST ? hipMemcpyHostToDevice
                                                  : hipMemcpyDeviceToDevice,
                           s);
        if (e != hipSuccess) return e;
    }
    *out = buf.as<T>();
    return hipSuccess;
}

uint64_t tx_terms_of(const std::vector<uint32_t> &off);
crop_status validate_on_device(crop_ctx *ctx, const uint32_t *v_off, uint64_t K,
                               const uint32_t *idx, uint64_t nnz, uint32_t n, int64_t *bad_out);
crop_status check_pairs_on_device(crop_ctx *ctx, const uint32_t *qx, const uint32_t *qy,
                                  uint64_t n, uint32_t n_items, int64_t *bad_out);
crop_status check_offsets(crop_ctx *ctx, const std::vector<uint32_t> &off, uint64_t nnz,
                          const char *name);
void reset_input(crop_ctx *ctx);
void reset_batch(crop_ctx *ctx);
void batch_invalidate_graph(crop_ctx *ctx);
crop_status ensure_route_buffers(crop_ctx *ctx, size_t key_bytes, bool sums);
crop_status require_exact(crop_ctx *ctx);
crop_status run_begin(crop_ctx *ctx);
crop_status stage_end(crop_ctx *ctx, const char *name);
crop_status run_end(crop_ctx *ctx);
size_t spill_entry_bytes(bool wide, bool sums);
size_t tx_scatter_smem_bytes(uint32_t NB, uint32_t max_items, uint32_t cap, bool wide);
size_t tx_count_smem_bytes(uint32_t NB, uint32_t max_items);

#define STAGE(name)                                   \
    do {                                              \
        crop_status st_ = stage_end(ctx, name);       \
        if (st_ != CROP_OK) return st_;               \
    } while (0)


}  // namespace crop
