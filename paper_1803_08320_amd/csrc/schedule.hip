// Work order of the persistent adaptive kernel: lanes with the smallest periapsis first.
//
// An adaptive integrator spends most of its attempts near the orbit's closest approach,
// so the lanes of one batch need very different numbers of attempts (a factor ~10
// between the 10% and the 100% quantiles on bound Kerr orbits).  The persistent work
// queue hands lanes out in the order it is given; a lane that is long and handed out
// late keeps its wavefront busy after every other has drained the queue.  Handing the
// longest lanes out first (the longest-processing-time rule) removes that tail.  The
// expected length is ranked by the periapsis r_p, read off the Carter-separated radial
// equation of the lane's own constants (E, L_z, Q, mu^2) (Sections 3-4 integrate the
// same constants of motion):
//   (rho^2 dr/dtau)^2 = R(r) = [E (r^2 + a^2) - a L_z]^2 - Delta [mu^2 r^2 + (L_z - a E)^2 + Q],
// R(r_0) >= 0 at the lane's radius; r_p is the first zero of R inward from r_0.
//
// The key of lane i is the bucket j of r_p on the grid r_j = r_+ 2^(j/32) (2.2% wide):
// the largest j <= j_0 (r_j <= r_0) with R(r_j) < 0, found by a march inward one bucket
// at a time (a coarser march can step over the forbidden band of an orbit close to
// marginal stability, whose periapsis is small and whose lane is long).  R(r_+) >= 0
// always (Delta = 0 there), so a lane whose R stays >= 0 down to r_+ plunges (or has a
// band narrower than a bucket); it gets key 0 and goes first with the smallest periapses,
// which costs little when the lane is short and avoids handing out a long one last.
// Every lane the integrator will not load (not ACTIVE, tau >= tau_end, bad spacetime
// index) gets the last key, MALBEC_SCHED_BUCKETS - 1.  The order
// is a counting sort of the keys (a histogram, its exclusive scan, and a scatter that
// ranks the lanes of one block in LDS and reserves their slots with one atomic per
// bucket).  Within a bucket the order depends on the timing of those atomics; the
// integration of a lane does not depend on when it is handed out.
#include "internal.hpp"
#include "monitor.hpp"

namespace malbec {

namespace {

constexpr int kBins = MALBEC_SCHED_BUCKETS;  // 1024
constexpr double kPerOctave = 32.0;

struct KeyArgs {
    int64_t n;
    const double *state;
    const double *tau;
    const int32_t *status;
    const int32_t *st_of_lane;
    double tau_end;
    uint32_t *key;
};

struct RadialPotential {
    double M, a, E, L, Q, mu2;
    __device__ __forceinline__ double operator()(double r) const
    {
        const double r2a2 = r * r + a * a;
        const double Delta = r2a2 - 2.0 * M * r;
        const double P = E * r2a2 - a * L;
        const double K = L - a * E;
        return P * P - Delta * (mu2 * r * r + K * K + Q);
    }
};

template <bool MULTI>
__global__ void __launch_bounds__(256) sched_key_kernel(KeyArgs A, StTable T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    uint32_t key = kBins - 1;
    int32_t sid = 0;
    bool ok = A.status[i] == kActive && A.tau[i] < A.tau_end;
    if (MULTI) {
        sid = A.st_of_lane[i];
        ok = ok && sid >= 0 && sid < T.n_st;
    }
    if (ok) {
        const Spacetime S = T.st[MULTI ? sid : 0];
        double y[8], I[4];
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = A.state[k * A.n + i];
        lane_invariants<false>(S.M, S.a, y, I);
        const RadialPotential R{S.M, S.a, I[0], I[1], I[2], -I[3]};
        const double rp = S.M + sqrt(fmax(S.M * S.M - S.a * S.a, 0.0));
        const double x = kPerOctave * log2(y[1] / rp);  // NaN, +-inf and r_0 <= r_+ fail the test
        if (x >= 1.0 && __builtin_isfinite(R.E) && __builtin_isfinite(R.L) && __builtin_isfinite(R.Q)) {
            int j = (int)fmin(x, (double)(kBins - 2));
            while (j > 0 && !(R(rp * exp2((double)j / kPerOctave)) < 0.0)) --j;
            key = (uint32_t)j;  // j = 0: no turning point above r_+
        }
    }
    A.key[i] = key;
}

__global__ void zero_u32_kernel(uint32_t *p, int m)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) p[k] = 0u;
}

// count[b] += number of keys equal to b (LDS histogram per block, grid-stride).
__global__ void __launch_bounds__(256) sched_hist_kernel(const uint32_t *key, int64_t n,
                                                          uint32_t *count)
{
    __shared__ uint32_t h[kBins];
    for (int k = threadIdx.x; k < kBins; k += blockDim.x) h[k] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[min(key[i], (uint32_t)(kBins - 1))], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < kBins; k += blockDim.x)
        if (h[k]) atomicAdd(&count[k], h[k]);
}

// next[b] = sum of count[b'] over b' < b (one block of kBins threads, Hillis-Steele).
__global__ void __launch_bounds__(kBins) sched_scan_kernel(const uint32_t *count, uint32_t *next)
{
    __shared__ uint32_t v[2][kBins];
    const int t = threadIdx.x;
    int cur = 0;
    v[0][t] = t > 0 ? count[t - 1] : 0u;
    __syncthreads();
    for (int d = 1; d < kBins; d <<= 1) {
        v[cur ^ 1][t] = v[cur][t] + (t >= d ? v[cur][t - d] : 0u);
        __syncthreads();
        cur ^= 1;
    }
    next[t] = v[cur][t];
}

// order[next[b] ...] = the lanes with key b.  Each block takes 256 consecutive lanes at
// a time: LDS ranks within the block, one global atomic per non-empty bucket.
__global__ void __launch_bounds__(256) sched_scatter_kernel(const uint32_t *key, int64_t n,
                                                             uint32_t *next, uint32_t *order)
{
    __shared__ uint32_t cnt[kBins];
    __shared__ uint32_t base[kBins];
    const int64_t n_chunks = (n + 255) / 256;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        for (int k = threadIdx.x; k < kBins; k += 256) cnt[k] = 0u;
        __syncthreads();
        const int64_t i = chunk * 256 + threadIdx.x;
        const bool in = i < n;
        const uint32_t b = in ? min(key[i], (uint32_t)(kBins - 1)) : 0u;
        const uint32_t rank = in ? atomicAdd(&cnt[b], 1u) : 0u;
        __syncthreads();
        for (int k = threadIdx.x; k < kBins; k += 256)
            if (cnt[k]) base[k] = atomicAdd(&next[k], cnt[k]);
        __syncthreads();
        if (in) order[base[b] + rank] = (uint32_t)i;
        __syncthreads();
    }
}

}  // namespace

SchedLayout sched_layout(int64_t n)
{
    SchedLayout L;
    L.count = 0;
    L.next = (size_t)kBins * sizeof(uint32_t);
    L.key = 2 * L.next;
    L.order = L.key + (((size_t)n * sizeof(uint32_t) + 255) / 256) * 256;
    L.bytes = L.order + (size_t)n * sizeof(uint32_t);
    return L;
}

int launch_adaptive_order(const StTable &T, const int32_t *st_of_lane, int64_t n,
                          const double *state, const double *tau, const int32_t *status,
                          double tau_end, uint32_t *order, uint32_t *keys, void *ws,
                          hipStream_t s)
{
    if (n == 0) return MALBEC_OK;
    const SchedLayout Ly = sched_layout(n);
    char *w = (char *)ws;
    uint32_t *count = (uint32_t *)(w + Ly.count);
    uint32_t *next = (uint32_t *)(w + Ly.next);
    uint32_t *key = keys ? keys : (uint32_t *)(w + Ly.key);
    const bool multi = st_of_lane != nullptr && T.n_st > 1;
    KeyArgs A{n, state, tau, status, multi ? st_of_lane : nullptr, tau_end, key};
    if (multi)
        hipLaunchKernelGGL((sched_key_kernel<true>), dim3(grid_for(n, 256)), dim3(256), 0, s, A, T);
    else
        hipLaunchKernelGGL((sched_key_kernel<false>), dim3(grid_for(n, 256)), dim3(256), 0, s, A, T);
    MALBEC_LAUNCH_CHECK("sched_key_kernel");
    hipLaunchKernelGGL(zero_u32_kernel, dim3(kBins / 256), dim3(256), 0, s, count, kBins);
    MALBEC_LAUNCH_CHECK("zero_u32_kernel");
    const unsigned g = (unsigned)std::min<int64_t>(grid_for(n, 256), 1024);
    hipLaunchKernelGGL(sched_hist_kernel, dim3(g), dim3(256), 0, s, key, n, count);
    MALBEC_LAUNCH_CHECK("sched_hist_kernel");
    hipLaunchKernelGGL(sched_scan_kernel, dim3(1), dim3(kBins), 0, s, count, next);
    MALBEC_LAUNCH_CHECK("sched_scan_kernel");
    hipLaunchKernelGGL(sched_scatter_kernel, dim3(g), dim3(256), 0, s, key, n, next, order);
    MALBEC_LAUNCH_CHECK("sched_scatter_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
