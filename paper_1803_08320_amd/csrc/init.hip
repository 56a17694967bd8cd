// Initial-condition construction on the device, one thread per lane.
//
//  CANONICAL  the paper's IC table rows (t, r, theta, phi, p_t, p_r, p_theta, p_phi)
//             with p_t = +E (Section 5); u^mu = g^{mu nu} p_nu with p_t -> -E.
//  CIRCULAR   equatorial circular orbits (Sections 3-4) in the Bardeen-Press-
//             Teukolsky form, with a seeded relative perturbation of L.
//  CONSTANTS  seeded (r0, theta0, E, L_z, Q, signs) accepted when Carter's radial
//             and polar potentials are non-negative; u from the separated equations.
// Random numbers: SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based
// generator, draw k of attempt j of lane i = output (i*2^24 + j*2^4 + k + 1) of the
// sequence started at `seed`.
#include <mutex>

#include "ic_device.hpp"
#include "internal.hpp"

namespace malbec {

namespace {

__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t lane, uint64_t attempt,
                                                 uint64_t k)
{
    uint64_t z = seed + (((lane << 24) | (attempt << 4) | k) + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// lo + (hi - lo) u, rounded after each operation (no fused multiply-add), so that
// the drawn values are the same bits on every implementation of the recipe.
__device__ __forceinline__ double uniform(const double rg[2], uint64_t x)
{
#pragma clang fp contract(off)
    const double span = rg[1] - rg[0];
    const double scaled = span * unit53(x);
    return rg[0] + scaled;
}

// dL (2u - 1) with separately rounded operations.
__device__ __forceinline__ double centred(double dL, uint64_t x)
{
#pragma clang fp contract(off)
    const double twice = 2.0 * unit53(x);
    return dL * (twice - 1.0);
}

struct InitArgs {
    malbec_ic_spec spec;
    const int32_t *st_of_lane;
    int64_t n;
    double *state;
    double *consts;
    int64_t *attempts;
    unsigned long long *exhausted;  // strict mode: count of lanes that exhausted the sampler
};

// Lanes whose rejection sampler ran out of attempts in a strict call (one counter per
// GPU: each device holds its own copy, found through hipGetSymbolAddress).
__device__ unsigned long long g_exhausted;

__global__ void zero_exhausted_kernel(unsigned long long *p) { *p = 0ull; }

__global__ void __launch_bounds__(256) init_kernel(InitArgs A, StTable T)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t sid = A.st_of_lane ? A.st_of_lane[i] : 0;
    const bool bad_sid = sid < 0 || sid >= T.n_st;  // invalid index: NaN state
    if (bad_sid) sid = 0;
    const Spacetime S = T.st[sid];
    const double M = S.M, a = S.a;
    const malbec_ic_spec &P = A.spec;
    const uint64_t lane = (uint64_t)(P.lane0 + i);
    double y[8];
    double cE = 0.0, cL = 0.0, cQ = 0.0, cmu2 = P.mu2;
    int64_t used = 1;

    if (P.mode == MALBEC_IC_CANONICAL) {
        const double *z = P.rows + 8 * i;
        double s, c;
        sincos(z[2], &s, &c);
        double itt, itp, ipp, irr, ithth;
        inverse_metric(M, a, z[1], s, c, itt, itp, ipp, irr, ithth);
        const double pt = -z[4];
        y[0] = z[0]; y[1] = z[1]; y[2] = z[2]; y[3] = z[3];
        y[4] = itt * pt + itp * z[7];
        y[5] = irr * z[5];
        y[6] = ithth * z[6];
        y[7] = itp * pt + ipp * z[7];
        cE = z[4];
        cL = z[7];
        cmu2 = 1.0;
    } else if (P.mode == MALBEC_IC_PARAMS) {
        const double *z = P.rows + 6 * i;  // r0, theta0, u^r0, u^theta0, L_z, E
        double s, c;
        sincos(z[1], &s, &c);
        double itt, itp, ipp, irr, ithth;
        inverse_metric(M, a, z[0], s, c, itt, itp, ipp, irr, ithth);
        y[0] = 0.0; y[1] = z[0]; y[2] = z[1]; y[3] = 0.0;
        y[4] = itt * (-z[5]) + itp * z[4];
        y[5] = z[2];
        y[6] = z[3];
        y[7] = itp * (-z[5]) + ipp * z[4];
        cE = z[5];
        cL = z[4];
        cmu2 = 1.0;
    } else if (P.mode == MALBEC_IC_CIRCULAR) {
        const double rg[2] = {P.r_lo, P.r_hi};
        const double r0 = uniform(rg, splitmix_out(P.seed, lane, 0, 0));
        const double delta = centred(P.dL, splitmix_out(P.seed, lane, 0, 1));
        // Bardeen-Press-Teukolsky circular orbit, upper sign prograde
        const double sg = P.prograde ? 1.0 : -1.0;
        const double sr = sqrt(r0), sM = sqrt(M);
        const double den = pow(r0, 0.75) * sqrt(r0 * sr - 3.0 * M * sr + sg * 2.0 * a * sM);
        const double Ec = (r0 * sr - 2.0 * M * sr + sg * a * sM) / den;
        const double Lc = sg * sM * (r0 * r0 - sg * 2.0 * a * sM * sr + a * a) / den;
        const double L = Lc * (1.0 + delta);
        double itt, itp, ipp, irr, ithth;
        inverse_metric(M, a, r0, 1.0, 0.0, itt, itp, ipp, irr, ithth);
        double E = Ec;
        if (P.e_from_norm) {
            // g^{mu nu} p_mu p_nu = -1 with p = (-E, 0, 0, L): quadratic in E, g^tt < 0
            const double qa = itt, qb = -2.0 * itp * L, qc = ipp * L * L + 1.0;
            E = (-qb - sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa);
        }
        y[0] = 0.0; y[1] = r0; y[2] = 1.57079632679489661923; y[3] = 0.0;
        y[4] = itt * (-E) + itp * L;
        y[5] = 0.0;
        y[6] = 0.0;
        y[7] = itp * (-E) + ipp * L;
        cE = E;
        cL = L;
        cQ = 0.0;
        cmu2 = 1.0;
    } else {
        bool ok = false;
        int64_t att = 0;
        double r0 = 0, th0 = 0, sr = 1, sth = 1, R = 0, Th = 0, s = 0, c = 0;
        for (att = 0; att < P.max_attempts; ++att) {
            r0 = uniform(P.r_range, splitmix_out(P.seed, lane, att, 0));
            th0 = uniform(P.th_range, splitmix_out(P.seed, lane, att, 1));
            cE = uniform(P.E_range, splitmix_out(P.seed, lane, att, 2));
            cL = uniform(P.Lz_range, splitmix_out(P.seed, lane, att, 3));
            cQ = uniform(P.Q_range, splitmix_out(P.seed, lane, att, 4));
            sr = (splitmix_out(P.seed, lane, att, 5) >> 63) ? -1.0 : 1.0;
            sth = (splitmix_out(P.seed, lane, att, 6) >> 63) ? -1.0 : 1.0;
            sincos(th0, &s, &c);
            R = radial_potential(M, a, cE, cL, cQ, P.mu2, r0);
            Th = polar_potential(a, cE, cL, cQ, P.mu2, s, c);
            if (R >= 0.0 && Th >= 0.0) { ok = true; break; }
        }
        if (ok) {
            y[0] = 0.0; y[1] = r0; y[2] = th0; y[3] = 0.0;
            velocity(M, a, cE, cL, cQ, P.mu2, r0, s, c, sr, sth, R, Th, y + 4);
            used = att + 1;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) y[k] = __builtin_nan("");
            used = P.max_attempts;
            if (A.exhausted) atomicAdd(A.exhausted, 1ull);
        }
    }
    if (bad_sid) {
#pragma unroll
        for (int k = 0; k < 8; ++k) y[k] = __builtin_nan("");
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = y[k];
    if (A.consts) {
        A.consts[0 * A.n + i] = cE;
        A.consts[1 * A.n + i] = cL;
        A.consts[2 * A.n + i] = cQ;
        A.consts[3 * A.n + i] = cmu2;
    }
    if (A.attempts) A.attempts[i] = used;
}

}  // namespace

// The device address of g_exhausted on the current device, looked up once per device
// (each GPU holds its own copy at its own address; the name itself is a host-side
// stand-in that must not be passed to a kernel).
static int exhausted_counter(unsigned long long **out)
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static unsigned long long *ptr[kDevices] = {};
    int dev = 0;
    MALBEC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDevices)
        return fail(MALBEC_ENOTSUP, "device %d: the strict sampler count covers %d devices", dev, kDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        MALBEC_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(g_exhausted)));
        if (!p) return fail(MALBEC_EDEVICE, "hipGetSymbolAddress returned NULL for the sampler count");
        ptr[dev] = (unsigned long long *)p;
    }
    *out = ptr[dev];
    return MALBEC_OK;
}

int launch_init(const malbec_ic_spec &spec, const StTable &T, const int32_t *st_of_lane, int64_t n,
                double *state, double *consts, int64_t *attempts, hipStream_t s)
{
    InitArgs A;
    A.spec = spec;
    A.st_of_lane = T.n_st > 1 ? st_of_lane : nullptr;
    A.n = n;
    A.state = state;
    A.consts = consts;
    A.attempts = attempts;
    A.exhausted = nullptr;
    const bool strict = spec.strict != 0 && spec.mode == MALBEC_IC_CONSTANTS;
    if (strict) {
        int rc = exhausted_counter(&A.exhausted);
        if (rc) return rc;
        hipLaunchKernelGGL(zero_exhausted_kernel, dim3(1), dim3(1), 0, s, A.exhausted);
        MALBEC_LAUNCH_CHECK("zero_exhausted_kernel");
    }
    const int block = 256;
    hipLaunchKernelGGL(init_kernel, dim3(grid_for(n, block)), dim3(block), 0, s, A, T);
    MALBEC_LAUNCH_CHECK("init_kernel");
    if (strict) {
        unsigned long long count = 0;
        MALBEC_HIP_CHECK(hipMemcpyAsync(&count, A.exhausted, sizeof(count), hipMemcpyDeviceToHost, s));
        MALBEC_HIP_CHECK(hipStreamSynchronize(s));
        if (count > 0)
            return fail(MALBEC_ESAMPLE, "%llu of %lld lanes exhausted max_attempts = %lld", count,
                        (long long)n, (long long)spec.max_attempts);
    }
    return MALBEC_OK;
}

}  // namespace malbec
