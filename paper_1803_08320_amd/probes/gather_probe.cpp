// Gather-rate probe for the gridded 3+1 kernel (csrc/grid.hip): every lane loads, per
// "evaluation", four rows of 4 nodes x 5 doubles (160 contiguous bytes each) of an
// 801 x 401 x 5 grid (12.8 MB) at a pseudo-random cell, as one right-hand side of that
// kernel does, and only sums them.  Modes: 0, a fresh random cell per evaluation;
// 1, a random walk of one cell per four evaluations (one RK4 step), one row in flight;
// 2, the same walk with all four rows in flight.  1,048,576 lanes; prints the gathered
// bytes per second.  Not part of the library.
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_1803_08320_amd/probes/gather_probe.cpp -o gather_probe && ./gather_probe 400
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                        \
    do {                                                                \
        hipError_t e_ = (x);                                            \
        if (e_ != hipSuccess) {                                         \
            printf("%s failed: %s\n", #x, hipGetErrorString(e_));        \
            return 1;                                                   \
        }                                                               \
    } while (0)

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

template <int MODE>
__global__ void __launch_bounds__(256) gather(const double *nodes, int nr, int nth, int evals,
                                              double *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    uint32_t s = mix((uint32_t)i * 2654435761u + 12345u);
    int ci = 1 + (int)(s % (uint32_t)(nr - 3));
    int cj = 1 + (int)(mix(s) % (uint32_t)(nth - 3));
    for (int e = 0; e < evals; ++e) {
        if (MODE == 0) {  // a fresh random cell every evaluation
            s = mix(s + (uint32_t)e);
            ci = 1 + (int)(s % (uint32_t)(nr - 3));
            cj = 1 + (int)(mix(s) % (uint32_t)(nth - 3));
        } else if ((e & 3) == 0) {  // modes 1, 2: a random walk of one cell every 4 evaluations (one RK4 step)
            s = mix(s + (uint32_t)e);
            ci = min(max(ci + (int)(s % 3u) - 1, 1), nr - 3);
            cj = min(max(cj + (int)((s >> 8) % 3u) - 1, 1), nth - 3);
        }
        if (MODE < 2) {
#pragma unroll 1
            for (int a = 0; a < 4; ++a) {
                const double *row = nodes + ((int64_t)(ci - 1 + a) * nth + (cj - 1)) * 5;
#pragma unroll
                for (int b = 0; b < 20; ++b) acc += row[b];
            }
        } else {  // all four rows in flight, independent partial sums
            double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double *row = nodes + ((int64_t)(ci - 1 + a) * nth + (cj - 1)) * 5;
#pragma unroll
                for (int b = 0; b < 20; ++b) p[b & 3] += row[b];
            }
            acc += (p[0] + p[1]) + (p[2] + p[3]);
        }
    }
    out[i] = acc;
}

int main(int argc, char **argv)
{
    const int nr = 801, nth = 401;
    const int64_t n = 1 << 20;
    const int evals = argc > 1 ? atoi(argv[1]) : 400;
    std::vector<double> h((size_t)nr * nth * 5, 1.0);
    double *d_nodes, *d_out;
    if (hipMalloc(&d_nodes, h.size() * 8) != hipSuccess || hipMalloc(&d_out, n * 8) != hipSuccess ||
        hipMemcpy(d_nodes, h.data(), h.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
        printf("device allocation or copy failed\n");
        return 1;
    }
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    for (int mode = 0; mode < 3; ++mode) {
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(a, 0));
            if (mode == 0)
                hipLaunchKernelGGL(gather<0>, dim3(n / 256), dim3(256), 0, 0, d_nodes, nr, nth, evals, d_out, n);
            else if (mode == 1)
                hipLaunchKernelGGL(gather<1>, dim3(n / 256), dim3(256), 0, 0, d_nodes, nr, nth, evals, d_out, n);
            else
                hipLaunchKernelGGL(gather<2>, dim3(n / 256), dim3(256), 0, 0, d_nodes, nr, nth, evals, d_out, n);
            CHECK(hipEventRecord(b, 0));
            CHECK(hipEventSynchronize(b));
            float ms = 0;
            CHECK(hipEventElapsedTime(&ms, a, b));
            const double bytes = (double)n * evals * 640.0;
            printf("mode %d (%s) evals %d: %.3f ms, %.2f TB/s gathered, %.3e evaluations/s\n", mode,
                   mode == 0 ? "random cell" : mode == 1 ? "random walk" : "walk, 4 rows in flight", evals, ms, bytes / ms / 1e9,
                   (double)n * evals / ms * 1e3);
        }
    }
    hipError_t e = hipGetLastError();
    printf("status %s\n", hipGetErrorString(e));
    return e == hipSuccess ? 0 : 1;
}
