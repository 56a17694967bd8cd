// Persistent work-queue driver shared by the integrate kernels.
//
// A wavefront keeps 64 items (lanes of the batch) in flight.  After every sub-chunk
// of steps it retires the items that finished, takes a ballot of its idle lanes and
// refills them from a global 64-bit counter with one atomic per wavefront (each idle
// lane's slot is its mbcnt rank in the idle mask).  A wavefront leaves the loop when
// the counter has passed the item count and none of its lanes holds an item; every
// item finishes within a bounded number of steps, so every wavefront exits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace malbec {

// Prog provides:  typename Prog::Lane;
//   bool load(int64_t item, Lane&)   -- false: nothing to do for this item
//   bool step(Lane&)                 -- one step; true when the item is finished
//   void store(int64_t item, const Lane&)
template <class Prog>
__device__ __forceinline__ void persistent_loop(Prog &P, int64_t n_items,
                                                unsigned long long *counter, int32_t chunk)
{
    const unsigned lane = threadIdx.x & 63u;
    typename Prog::Lane L;
    int64_t item = -1;
    bool open = true;  // wavefront-uniform
    while (true) {
        const unsigned long long idle = __ballot(item < 0);
        if (idle != 0ull && open) {
            const int cnt = __popcll(idle);
            const int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0;
            if ((int)lane == leader) base = atomicAdd(counter, (unsigned long long)cnt);
            base = (unsigned long long)__shfl((long long)base, leader, 64);
            if (base + (unsigned long long)cnt >= (unsigned long long)n_items) open = false;
            if (item < 0) {
                const unsigned rank = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(idle >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
                const unsigned long long id = base + rank;
                if (id < (unsigned long long)n_items) {
                    item = (int64_t)id;
                    if (!P.load(item, L)) item = -1;
                }
            }
        }
        const bool busy = __ballot(item >= 0) != 0ull;
        if (!busy && !open) break;
        if (item >= 0) {
            for (int32_t s = 0; s < chunk; ++s) {
                if (P.step(L)) {
                    P.store(item, L);
                    item = -1;
                    break;
                }
            }
        }
    }
}

namespace {
// Clears the work counter (a kernel, not a memset, so that it can sit in a captured
// graph and be replayed).
__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }
}  // namespace

}  // namespace malbec
