// Adaptive integration without a caller workspace: the scratch of the persistent
// work queue and of its periapsis work order lives in a file-scope device array.
//
// For callers that cannot allocate device memory around the call (code under HIP
// graph capture, serving loops, harnesses that forbid allocation).  The array is a
// module global, so every GPU the library runs on holds its own copy, at its own
// address, for the life of the process.  Host code never passes the array's name to
// a kernel or a copy (on the host that name is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, looked up once per device with that
// device current, and is what the launches receive.
#include <mutex>

#include "internal.hpp"

namespace malbec {

namespace {

// Largest batch: 2^21 lanes.  Layout (as the workspace of malbec_integrate_adaptive):
// 256 B work counter, then the order's bucket counts and cursors (2 x 1,024 uint32),
// keys (n uint32, padded to 256 B) and the order (n uint32).
constexpr int64_t kNoAllocMaxLanes = MALBEC_NOALLOC_MAX_LANES;
constexpr size_t kNoAllocBytes =
    256 + 2 * MALBEC_SCHED_BUCKETS * sizeof(uint32_t) + 2 * (size_t)kNoAllocMaxLanes * sizeof(uint32_t);
static_assert(kNoAllocMaxLanes % 64 == 0, "the key array must end on a 256-byte boundary");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device, once looked up

// Device address of this device's copy of `scratch` (the current device's).
int scratch_address(void **out)
{
    int dev = 0;
    MALBEC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MALBEC_ENOTSUP, "device %d: the no-allocation scratch table covers %d devices",
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        MALBEC_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MALBEC_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MALBEC_OK;
}

}  // namespace

}  // namespace malbec

using namespace malbec;

extern "C" int malbec_integrate_adaptive_noalloc(const malbec_adaptive *ad, const malbec_batch *b,
                                                 int64_t n, double *state, double *tau, double *h,
                                                 int32_t *status, int32_t *steps, int32_t *rejects,
                                                 void *stream)
{
    clear_error();
    if (!ad) return fail(MALBEC_EINVAL, "ad is NULL");
    if (n > kNoAllocMaxLanes)
        return fail(MALBEC_EINVAL, "n = %lld exceeds the %lld lanes of the no-allocation scratch",
                    (long long)n, (long long)kNoAllocMaxLanes);
    const size_t need =
        malbec_workspace_bytes(MALBEC_OP_ADAPTIVE, n < 0 ? 0 : n, ad->persistent ? 1 + ad->schedule : 0);
    if (need > kNoAllocBytes)
        return fail(MALBEC_EINVAL, "scratch of %zu bytes needed, %zu available", need, kNoAllocBytes);
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    // the work counter and the order's bucket counts are cleared by kernels inside the
    // call; the rest of the scratch is fully written before it is read
    return malbec_integrate_adaptive(ad, b, n, state, tau, h, status, steps, rejects, ws,
                                     kNoAllocBytes, stream);
}
