// Geodesics in a numerical metric given in 3+1 form on an (r, theta) grid.
//
// Section 2 writes the line element in 3+1 form (eq. ADM: lapse alpha, shift
// beta^i, spatial metric gamma_ij), gives them for Kerr, and names the 3+1 form as
// the route to numerically computed metrics.  Here a stationary, axisymmetric metric
// with beta = (0, 0, beta^phi) and diagonal gamma is five functions of (r, theta),
//   F = (alpha, beta^phi, gamma_rr, gamma_thth, gamma_phph / sin^2 theta),
// sampled on a uniform grid (node (i, j) holds its five values contiguously: 40 B as
// doubles, 20 B as floats; the values are widened to FP64 on load).
// At a point the kernel takes the tensor product of 4-point Lagrange interpolants
// (16 nodes: four rows of four consecutive nodes, 160 contiguous bytes each), the
// derivatives of that interpolant, the inverse metric
//   g^tt = -1/alpha^2, g^tphi = beta^phi/alpha^2,
//   g^phph = 1/gamma_phph - (beta^phi)^2/alpha^2, g^rr = 1/gamma_rr, g^thth = 1/gamma_thth
// and its r, theta derivatives, and Hamilton's equations (eq. Ham) on (x^mu, p_mu)
// with classic RK4 (p_t and p_phi are constants).  A right-hand side needs 640 B of
// grid data (320 B as floats); each lane keeps its current cell's stencil in LDS
// (StencilCache), so the rows are gathered from the caches only when a lane moves to
// another cell, and the work per lane-step is ~4 x (interpolation 220 fma + metric
// algebra).
#include <type_traits>

#include "internal.hpp"

namespace malbec {

namespace {

struct GridArgs {
    int64_t n;
    double *state;
    int32_t *status;
    int32_t *steps;
    const void *nodes;  // Node[nr * nth * 5], Node = double or float
    int32_t nr, nth;
    double r0, idr, th0, idth;   // inverse spacings
    double rlo, rhi, tlo, thi;   // interior (stencils and stage points stay inside)
    double r_stop, r_escape, h;
    int32_t n_steps;
};

// Lagrange basis on the nodes -1, 0, 1, 2 at u, and its derivative.
__device__ __forceinline__ void lagrange4(double u, double w[4], double dw[4])
{
    const double um = u - 1.0, u2 = u - 2.0, up = u + 1.0;
    w[0] = -u * um * u2 * (1.0 / 6.0);
    w[1] = up * um * u2 * 0.5;
    w[2] = -up * u * u2 * 0.5;
    w[3] = up * u * um * (1.0 / 6.0);
    const double uu3 = 3.0 * u * u;
    dw[0] = -(uu3 - 6.0 * u + 2.0) * (1.0 / 6.0);
    dw[1] = (uu3 - 4.0 * u - 1.0) * 0.5;
    dw[2] = -(uu3 - 2.0 * u - 2.0) * 0.5;
    dw[3] = (uu3 - 1.0) * (1.0 / 6.0);
}

// Stencil start (node index - 1) and offset u of x on a grid of n nodes; the cell
// index is clamped to [1, n - 3] (NaN-safe), so every access stays inside the grid.
__device__ __forceinline__ int32_t cell(double x, double x0, double ih, int32_t n, double &u)
{
    const double q = (x - x0) * ih;
    const double f = fmin(fmax(floor(q), 1.0), (double)(n - 3));
    u = q - f;
    return (int32_t)f;
}

// Stencil cache of one lane: the 16 nodes x 5 values of the lane's current cell in
// LDS, as 16-byte chunks (4 floats or 2 doubles) with the block's lanes interleaved
// (chunk m of thread t at lds[m * kCacheLanes + t]: conflict-free 16-byte reads), and
// the cell it holds.  The four stage points of a step, and the next steps, mostly lie
// in the same cell (a stage moves a few thousandths in r and theta against cells of
// 0.075 and 0.0075 on the benchmark grid), so most evaluations read LDS instead of
// gathering four rows through the L1.  320 B per lane with float nodes (two blocks of
// 256 fill a CU's 160 KB: two waves per SIMD, as the registers allow) and 640 B with
// double nodes (one block per CU, one wave per SIMD; the LDS reads need little
// latency hiding).
constexpr int kCacheLanes = 256;
template <typename Node>
struct StencilCache {
    typedef typename std::conditional<std::is_same<Node, float>::value, float4, double2>::type Chunk;
    Chunk *lds;      // &cache[threadIdx.x]
    int32_t ci, cj;  // cell held (-1: none)
};

// Lagrange contraction of one stencil row (4 nodes x 5 values, element b * 5 + k,
// widened to FP64 where used).
template <typename V>
__device__ __forceinline__ void contract_row(const V *f, double wra, double dwra,
                                             const double wt[4], const double dwt[4], double F[5],
                                             double Fr[5], double Ft[5])
{
    double v[5], vt[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) { v[k] = 0.0; vt[k] = 0.0; }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double x = (double)f[b * 5 + k];
            v[k] = fma(wt[b], x, v[k]);
            vt[k] = fma(dwt[b], x, vt[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        F[k] = fma(wra, v[k], F[k]);
        Fr[k] = fma(dwra, v[k], Fr[k]);
        Ft[k] = fma(wra, vt[k], Ft[k]);
    }
}

// F, dF/dr, dF/dtheta of the five functions at (r, theta), through the lane's stencil
// cache C (refilled from the grid when the cell changes; double or float node values).
template <typename Node>
__device__ __forceinline__ void grid_eval(const GridArgs &A, double r, double th, double F[5],
                                          double Fr[5], double Ft[5], StencilCache<Node> *C)
{
    typedef typename StencilCache<Node>::Chunk Chunk;
    constexpr int PER = 16 / sizeof(Node);   // values per chunk
    constexpr int CH = 20 / PER;             // chunks per row
    double ur, ut, wr[4], dwr[4], wt[4], dwt[4];
    const int32_t i = cell(r, A.r0, A.idr, A.nr, ur);
    const int32_t j = cell(th, A.th0, A.idth, A.nth, ut);
    lagrange4(ur, wr, dwr);
    lagrange4(ut, wt, dwt);
#pragma unroll
    for (int k = 0; k < 5; ++k) { F[k] = 0.0; Fr[k] = 0.0; Ft[k] = 0.0; }
    if (i != C->ci || j != C->cj) {
#pragma unroll 1
        for (int a = 0; a < 4; ++a) {
            const Node *row = (const Node *)A.nodes + ((int64_t)(i - 1 + a) * A.nth + (j - 1)) * 5;
            Node g[20];
#pragma unroll
            for (int e = 0; e < 20; ++e) g[e] = row[e];
#pragma unroll
            for (int m = 0; m < CH; ++m) {
                Chunk q;
                Node *qp = (Node *)&q;
#pragma unroll
                for (int e = 0; e < PER; ++e) qp[e] = g[PER * m + e];
                C->lds[(a * CH + m) * kCacheLanes] = q;
            }
        }
        C->ci = i;
        C->cj = j;
    }
#pragma unroll 1
    for (int a = 0; a < 4; ++a) {
        Node f[20];
#pragma unroll
        for (int m = 0; m < CH; ++m) {
            const Chunk q = C->lds[(a * CH + m) * kCacheLanes];
            const Node *qp = (const Node *)&q;
#pragma unroll
            for (int e = 0; e < PER; ++e) f[PER * m + e] = qp[e];
        }
        contract_row(f, wr[a], dwr[a], wt, dwt, F, Fr, Ft);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) { Fr[k] *= A.idr; Ft[k] *= A.idth; }
}

// Canonical right-hand side with the gridded metric; records the stage point.
template <typename Node>
struct GridHam {
    const GridArgs &A;
    const HamConst<double> &P;
    StencilCache<Node> *C;  // the lane's stencil cache
    StageTrig trig;
    double st_r[4], st_th[4];
    __device__ __forceinline__ void operator()(int stage, double r, double th, double pr, double pth,
                                               double &dt, double &dr, double &dth, double &dph,
                                               double &dpr, double &dpth)
    {
        st_r[stage] = r;
        st_th[stage] = th;
        double s, c;
        trig(stage, th, s, c);
        double F[5], Fr[5], Ft[5];
        grid_eval<Node>(A, r, th, F, Fr, Ft, C);
        const double s2 = s * s;
        const double al = F[0], be = F[1];
        const double ia = recip(al);
        const double ia2 = ia * ia;
        const double igrr = recip(F[2]), igtt = recip(F[3]), igpp = recip(F[4] * s2);
        // g^{mu nu} p_nu
        const double pt = P.pt, pph = P.pph;
        const double bia2 = be * ia2;
        dt = fma(bia2, pph, -ia2 * pt);
        dph = fma(bia2, pt, (igpp - be * bia2) * pph);
        dr = igrr * pr;
        dth = igtt * pth;
        // -1/2 d_l g^{ab} p_a p_b, l = r, theta
        const double dgpp_r = Fr[4] * s2, dgpp_t = fma(Ft[4], s2, F[4] * 2.0 * s * c);
        const double q_tt = pt * pt, q_tp = pt * pph, q_pp = pph * pph;
        auto dH = [&](double dal, double dbe, double dgrr, double dgtt, double dgpp) {
            const double dia2 = -2.0 * dal * ia2 * ia;       // d(1/alpha^2)
            const double d_tt = -dia2;                       // d g^tt
            const double d_tp = fma(dbe, ia2, be * dia2);    // d g^tphi
            const double d_pp = fma(-dgpp, igpp * igpp, -fma(2.0 * be * dbe, ia2, be * be * dia2));
            const double d_rr = -dgrr * igrr * igrr;
            const double d_hh = -dgtt * igtt * igtt;
            const double sum = fma(d_tt, q_tt, fma(2.0 * d_tp, q_tp, fma(d_pp, q_pp,
                               fma(d_rr, pr * pr, d_hh * pth * pth))));
            return -0.5 * sum;
        };
        dpr = dH(Fr[0], Fr[1], Fr[2], Fr[3], dgpp_r);
        dpth = dH(Ft[0], Ft[1], Ft[2], Ft[3], dgpp_t);
    }
};

__device__ __forceinline__ bool inside(const GridArgs &A, double r, double th)
{
    return r >= A.rlo && r <= A.rhi && th >= A.tlo && th <= A.thi;
}

// At most 256 registers (the two waves per SIMD that the float-node cache's LDS
// allows): left alone the compiler spills a few values to AGPRs past 256 registers.
// The double-node cache takes a CU's whole LDS, so that kernel runs one wave per SIMD.
template <typename Node>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
rk4_grid_kernel(GridArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    int32_t st = A.status[i];
    if (st != kActive) return;
    double y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = A.state[k * A.n + i];
    const HamConst<double> P{y[4], y[7], 0.0, 0.0};
    typedef typename StencilCache<Node>::Chunk Chunk;
    __shared__ Chunk cache[4 * (20 * sizeof(Node) / 16) * kCacheLanes];
    StencilCache<Node> C{&cache[threadIdx.x], -1, -1};
    int32_t taken = 0;
    for (int32_t k = 0; k < A.n_steps && st == kActive; ++k) {
        GridHam<Node> f{A, P, &C, {0.0, 0.0, 1.0}};
        double y1[8], sr[3];
        rk4_ham_step(f, A.h, y, y1, sr);
        ++taken;
        // stage points in order: the first that is in the stop zone or off the grid
        // decides; then the result
        int32_t out = kActive;
#pragma unroll
        for (int s = 1; s < 4; ++s) {
            if (out != kActive) break;
            if (f.st_r[s] <= A.r_stop) out = kHorizon;
            else if (!inside(A, f.st_r[s], f.st_th[s])) out = kNonfinite;
        }
        if (out == kActive && (!usable(y1) || !inside(A, y1[1], y1[2]))) out = kNonfinite;
        if (out != kActive) {
            st = out;
            break;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) y[c] = y1[c];
        if (y[1] <= A.r_stop) st = kHorizon;
        else if (y[1] >= A.r_escape) st = kEscape;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) A.state[k * A.n + i] = y[k];
    A.status[i] = st;
    A.steps[i] += taken;
}

// Kerr's 3+1 functions (Section 2) at every node, computed in FP64 and stored as Node.
template <typename Node>
__global__ void __launch_bounds__(256) grid_fill_kerr_kernel(Node *nodes, int32_t nr, int32_t nth,
                                                             double r0, double dr, double th0,
                                                             double dth, double M, double a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)nr * nth) return;
    const int64_t i = p / nth, j = p % nth;
    const double r = r0 + (double)i * dr, th = th0 + (double)j * dth;
    double s, c;
    sincos(th, &s, &c);
    const double r2a2 = r * r + a * a;
    const double rho2 = r * r + a * a * c * c;
    const double Delta = r * r - 2.0 * M * r + a * a;
    const double Sigma = r2a2 * r2a2 - a * a * Delta * s * s;
    Node *F = nodes + p * 5;
    F[0] = (Node)sqrt(rho2 * Delta / Sigma);
    F[1] = (Node)(-2.0 * M * a * r / Sigma);
    F[2] = (Node)(rho2 / Delta);
    F[3] = (Node)rho2;
    F[4] = (Node)(Sigma / rho2);
}

}  // namespace

int launch_grid_fill_kerr(const malbec_grid &g, double M, double a, void *nodes, hipStream_t s)
{
    const int block = 256;
    const int64_t np = (int64_t)g.nr * g.nth;
    if (g.node_precision == MALBEC_GRID_F32)
        hipLaunchKernelGGL(grid_fill_kerr_kernel<float>, dim3(grid_for(np, block)), dim3(block), 0, s,
                           (float *)nodes, g.nr, g.nth, g.r0, g.dr, g.th0, g.dth, M, a);
    else
        hipLaunchKernelGGL(grid_fill_kerr_kernel<double>, dim3(grid_for(np, block)), dim3(block), 0,
                           s, (double *)nodes, g.nr, g.nth, g.r0, g.dr, g.th0, g.dth, M, a);
    MALBEC_LAUNCH_CHECK("grid_fill_kerr_kernel");
    return MALBEC_OK;
}

int launch_integrate_grid(const malbec_run &run, const malbec_grid &g, int64_t n, double *state,
                          int32_t *status, int32_t *steps, hipStream_t s)
{
    const int block = run.block > 0 ? run.block : 256;
    if (block > 256) return fail(MALBEC_EINVAL, "block %d exceeds the kernel's launch bound 256", block);
    GridArgs A;
    A.n = n;
    A.state = state;
    A.status = status;
    A.steps = steps;
    A.nodes = g.nodes;
    A.nr = g.nr;
    A.nth = g.nth;
    A.r0 = g.r0;
    A.idr = 1.0 / g.dr;
    A.th0 = g.th0;
    A.idth = 1.0 / g.dth;
    A.rlo = g.r0 + g.dr;
    A.rhi = g.r0 + (double)(g.nr - 2) * g.dr;
    A.tlo = g.th0 + g.dth;
    A.thi = g.th0 + (double)(g.nth - 2) * g.dth;
    A.r_stop = g.r_stop;
    A.r_escape = run.r_escape;
    A.h = run.h;
    const int64_t total = run.n_steps;
    const int64_t chunk = run.steps_per_chunk > 0 ? run.steps_per_chunk : total;
    for (int64_t k0 = 0; k0 < total; k0 += chunk) {
        A.n_steps = (int32_t)((total - k0) < chunk ? (total - k0) : chunk);
        if (g.node_precision == MALBEC_GRID_F32)
            hipLaunchKernelGGL(rk4_grid_kernel<float>, dim3(grid_for(n, block)), dim3(block), 0, s, A);
        else
            hipLaunchKernelGGL(rk4_grid_kernel<double>, dim3(grid_for(n, block)), dim3(block), 0, s, A);
        MALBEC_LAUNCH_CHECK("rk4_grid_kernel");
    }
    return MALBEC_OK;
}

}  // namespace malbec
