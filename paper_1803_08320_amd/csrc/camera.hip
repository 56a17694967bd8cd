// Camera: backward-traced null geodesics of a Kerr black hole with a thin
// equatorial disk, one photon per lane.
//
// Ray lengths are very uneven (a few hundred steps for rays that miss, many more
// near the photon ring), so the default kernel is persistent: each wavefront keeps
// 64 rays in flight and, after every sub-chunk of steps, retires the lanes whose
// ray ended (ballot of the finished lanes) and refills them from a global work
// counter with one atomic per wavefront (mbcnt prefix over the idle-lane mask
// gives each idle lane its slot).  The rays' initial states are formed beforehand by
// one thread per pixel into the workspace (64 B per pixel, read back once when the
// pixel is taken), which keeps the image-plane arithmetic out of the persistent
// loop and its registers: the loop fits the 128 registers of four waves per SIMD,
// as the one-thread-per-pixel kernel does.  A lane's result depends only on its
// pixel, so the persistent and the one-thread-per-pixel kernels give identical bits.
// Finished rays write their results straight to their pixels' slots: a ray's 24 B
// of results (status, step count, crossing) against its hundreds of steps make the
// scattered writes a negligible share of the traffic, so no staging of results in
// LDS is needed.
#include "ic_device.hpp"
#include "internal.hpp"

namespace malbec {

namespace {

constexpr double kHalfPi = 1.57079632679489661923;  // rounds to the double nearest pi/2

struct CamArgs {
    Spacetime S;          // M, a, r_stop
    double r_obs, incl, sin_i, cos_i, half_width;
    double h0, h_r0, inv_h_r0, r_escape, disk_r_in, disk_r_out;  // inv_h_r0 = RN(1 / h_r0)
    int32_t nx, ny;
    int64_t npix;
    int32_t max_steps;
    int32_t chunk;        // steps between retire/refill checks
    int32_t *status;
    int32_t *steps;
    double *hit;          // 2 * npix, component-major (r_c, phi_c)
    double *final_state;  // 8 * npix or nullptr
};

// Photon of pixel p (Bardeen image plane), traced backward: the arriving photon
// has E = 1, L_z = -alpha sin i, Q = beta^2 + cos^2 i (alpha^2 - a^2), u^r > 0,
// sign(u^theta) = sign(beta); the state carries -u.
__device__ __forceinline__ void pixel_ray(const CamArgs &A, int64_t p, double y[8])
{
    const int64_t i = p % A.nx, j = p / A.nx;
    const double w = A.half_width;
    const double alpha = -w + ((double)i + 0.5) * 2.0 * w / (double)A.nx;
    const double beta = -w + ((double)j + 0.5) * 2.0 * w / (double)A.ny;
    const double M = A.S.M, a = A.S.a;
    const double Lz = -alpha * A.sin_i;
    const double Q = beta * beta + A.cos_i * A.cos_i * (alpha * alpha - a * a);
    const double R = radial_potential(M, a, 1.0, Lz, Q, 0.0, A.r_obs);
    const double Th = polar_potential(a, 1.0, Lz, Q, 0.0, A.sin_i, A.cos_i);
    double u[4];
    velocity(M, a, 1.0, Lz, Q, 0.0, A.r_obs, A.sin_i, A.cos_i, 1.0, beta >= 0.0 ? 1.0 : -1.0, R,
             Th, u);
    y[0] = 0.0; y[1] = A.r_obs; y[2] = A.incl; y[3] = 0.0;
    y[4] = -u[0]; y[5] = -u[1]; y[6] = -u[2]; y[7] = -u[3];
}

// One step of a camera ray (the trigonometry table read from the block's LDS copy,
// which both camera kernels fill first: measured about 1.5 % faster than reading it
// through the vector cache).  Rules in order: a stage point at r <= r_stop ->
// HORIZON (y kept); unusable result -> NONFINITE (y kept); crossing of the
// equatorial plane with r_c in [disk_r_in, disk_r_out] -> DISK; r <= r_stop ->
// HORIZON; r >= r_escape -> ESCAPE.  Crossing: the sign of cos(theta) differs
// between y and y1, which for theta in (0, pi) is (theta > pi/2) differing.
__device__ __forceinline__ int32_t camera_step(const CamArgs &A, double y[8], int32_t &n,
                                               double &rc, double &pc)
{
    const double q0 = y[1] * A.inv_h_r0;
    const double q = fma(fma(-A.h_r0, q0, y[1]), A.inv_h_r0, q0);
    const double h = A.h0 * fmax(1.0, q);
    double y1[8], sr[3];
    rk4_step_f64<false, TabLds>(A.S, h, y, y1, sr);
    ++n;
    if (sr[0] <= A.S.r_stop || sr[1] <= A.S.r_stop || sr[2] <= A.S.r_stop) return kHorizon;
    if (!usable(y1)) return kNonfinite;
    int32_t st = kActive;
    if ((y[2] > kHalfPi) != (y1[2] > kHalfPi)) {
        const double c0 = cos(y[2]), c1 = cos(y1[2]);
        const double f = c0 / (c0 - c1);
        const double rcr = y[1] + (y1[1] - y[1]) * f;
        if (rcr >= A.disk_r_in && rcr <= A.disk_r_out) {
            rc = rcr;
            pc = y[3] + (y1[3] - y[3]) * f;
            st = kDisk;
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = y1[k];
    if (st == kActive) {
        if (y[1] <= A.S.r_stop) st = kHorizon;
        else if (y[1] >= A.r_escape) st = kEscape;
    }
    return st;
}

__device__ __forceinline__ void write_result(const CamArgs &A, int64_t p, int32_t st, int32_t n,
                                             double rc, double pc, const double y[8])
{
    A.status[p] = st;
    A.steps[p] = n;
    A.hit[p] = rc;
    A.hit[A.npix + p] = pc;
    if (A.final_state) {
#pragma unroll
        for (int k = 0; k < 8; ++k) A.final_state[k * A.npix + p] = y[k];
    }
}

// One thread per pixel, each traced to the end.
__global__ void __launch_bounds__(256) camera_plain_kernel(CamArgs A)
{
    TabLds::fill();
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npix) return;
    double y[8];
    pixel_ray(A, p, y);
    int32_t n = 0, st = kActive;
    double rc = __builtin_nan(""), pc = __builtin_nan("");
    while (st == kActive) {
        if (n >= A.max_steps) { st = kBudget; break; }
        st = camera_step(A, y, n, rc, pc);
    }
    write_result(A, p, st, n, rc, pc, y);
}

// Initial states of all rays, component-major y0[k * npix + p].
__global__ void __launch_bounds__(256) camera_rays_kernel(CamArgs A, double *y0)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.npix) return;
    double y[8];
    pixel_ray(A, p, y);
#pragma unroll
    for (int k = 0; k < 8; ++k) y0[k * A.npix + p] = y[k];
}

// Persistent kernel: every wavefront loops until the work counter passes npix and
// all of its lanes are idle; each lane's ray ends within max_steps steps, so every
// wavefront exits.  y0: the rays' initial states (camera_rays_kernel).
__global__ void __launch_bounds__(256) camera_persistent_kernel(CamArgs A,
                                                                unsigned long long *counter,
                                                                const double *y0)
{
    TabLds::fill();
    __syncthreads();
    const unsigned lane = threadIdx.x & 63u;
    int64_t p = -1;  // pixel in flight, -1 = idle
    double y[8];
    int32_t n = 0;
    double rc = 0.0, pc = 0.0;
    bool queue_open = true;  // wave-uniform
    while (true) {
        const unsigned long long idle = __ballot(p < 0);
        if (idle != 0ull && queue_open) {
            const int cnt = __popcll(idle);
            const int leader = __ffsll((long long)idle) - 1;
            unsigned long long base = 0;
            if ((int)lane == leader) base = atomicAdd(counter, (unsigned long long)cnt);
            base = (unsigned long long)__shfl((long long)base, leader, 64);
            if (base + (unsigned long long)cnt >= (unsigned long long)A.npix) queue_open = false;
            if (p < 0) {
                const unsigned rank = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(idle >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)idle, 0u));
                const unsigned long long id = base + rank;
                if (id < (unsigned long long)A.npix) {
                    p = (int64_t)id;
#pragma unroll
                    for (int k = 0; k < 8; ++k) y[k] = y0[k * A.npix + p];
                    n = 0;
                    rc = __builtin_nan("");
                    pc = __builtin_nan("");
                }
            }
        }
        if (__ballot(p >= 0) == 0ull) break;  // nothing in flight and nothing to fetch
        if (p >= 0) {
            int32_t st = kActive;
            for (int32_t s = 0; s < A.chunk && st == kActive; ++s)
                st = n >= A.max_steps ? kBudget : camera_step(A, y, n, rc, pc);
            if (st != kActive) {
                write_result(A, p, st, n, rc, pc, y);
                p = -1;
            }
        }
    }
}

__global__ void zero_counter_kernel(unsigned long long *counter) { *counter = 0ull; }

}  // namespace

int launch_camera(const malbec_camera &cam, double r_stop, double disk_r_in, int32_t *status,
                  int32_t *steps, double *hit, double *final_state, void *ws, hipStream_t s)
{
    CamArgs A;
    A.S.M = cam.M;
    A.S.a = cam.a;
    A.S.r_stop = r_stop;
    A.S.r_zone = 0.0;
    A.r_obs = cam.r_obs;
    A.incl = cam.incl;
    A.sin_i = sin(cam.incl);
    A.cos_i = cos(cam.incl);
    A.half_width = cam.half_width;
    A.h0 = cam.h0;
    A.h_r0 = cam.h_r0;
    A.inv_h_r0 = 1.0 / cam.h_r0;
    A.r_escape = cam.r_escape;
    A.disk_r_in = disk_r_in;
    A.disk_r_out = cam.disk_r_out;
    A.nx = cam.nx;
    A.ny = cam.ny;
    A.npix = (int64_t)cam.nx * cam.ny;
    A.max_steps = (int32_t)cam.max_steps;
    A.chunk = cam.steps_per_chunk > 0 ? cam.steps_per_chunk : 32;
    A.status = status;
    A.steps = steps;
    A.hit = hit;
    A.final_state = final_state;
    const int block = cam.block > 0 ? cam.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    if (!cam.persistent) {
        hipLaunchKernelGGL(camera_plain_kernel, dim3(grid_for(A.npix, block)), dim3(block), 0, s, A);
        MALBEC_LAUNCH_CHECK("camera_plain_kernel");
        return MALBEC_OK;
    }
    int dev = 0;
    MALBEC_HIP_CHECK(hipGetDevice(&dev));
    int n_cu = 0;
    MALBEC_HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0;
    MALBEC_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, camera_persistent_kernel,
                                                                 block, 0));
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)n_cu * per_cu;
    const int64_t need = (A.npix + block - 1) / block;  // no more lanes than pixels
    if (grid > need) grid = need;
    unsigned long long *counter = (unsigned long long *)ws;
    double *y0 = (double *)((char *)ws + 256);
    hipLaunchKernelGGL(camera_rays_kernel, dim3(grid_for(A.npix, 256)), dim3(256), 0, s, A, y0);
    MALBEC_LAUNCH_CHECK("camera_rays_kernel");
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    MALBEC_LAUNCH_CHECK("zero_counter_kernel");
    hipLaunchKernelGGL(camera_persistent_kernel, dim3((unsigned)grid), dim3(block), 0, s, A, counter,
                       (const double *)y0);
    MALBEC_LAUNCH_CHECK("camera_persistent_kernel");
    return MALBEC_OK;
}

}  // namespace malbec
