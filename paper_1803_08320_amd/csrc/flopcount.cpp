// Static operation count of one FP64 RK4 step (host tool).
//
// Instantiates the templates the kernels use (kerr_accel.hpp for the Christoffel
// form, ham_accel.hpp for Hamilton's equations, dp45.hpp for the adaptive pair) with a
// counting scalar type.  Counting rule: add, sub, mul, div = 1 flop each, fma = 2
// flops, sincos = 2 (two results), negation = 0.  The count is independent of the
// data (the code is straight-line), so one evaluation gives the flops per lane-step.
// sin/cos of a stage angle count 2 however the kernel obtains them (library sincos or
// rotation).  The Christoffel form is counted twice: in its direct form
// (kerr_accel_direct: the coefficients, then the contraction), which fixes the work of
// one step for the roofline, and in the regrouped form the kernels evaluate
// (kerr_accel), which needs fewer operations for the same acceleration.
//   g++ -O0 -std=c++17 flopcount.cpp -o flopcount && ./flopcount
#include <cstdio>

struct Counted;
static long g_flops = 0, g_div = 0, g_fma = 0, g_addmul = 0;

struct Counted {
    double v;
    Counted(double x = 0.0) : v(x) {}
};
static Counted op(double v, int flops) { g_flops += flops; if (flops == 1) ++g_addmul; return Counted(v); }
inline Counted operator+(Counted a, Counted b) { return op(a.v + b.v, 1); }
inline Counted operator-(Counted a, Counted b) { return op(a.v - b.v, 1); }
inline Counted operator*(Counted a, Counted b) { return op(a.v * b.v, 1); }
inline Counted operator/(Counted a, Counted b) { ++g_div; g_flops += 1; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted &operator+=(Counted &a, Counted b) { a = a + b; return a; }
inline Counted fma(Counted a, Counted b, Counted c) { ++g_fma; g_flops += 2; return Counted(a.v * b.v + c.v); }
namespace malbec {
inline Counted recip(Counted x) { ++g_div; g_flops += 1; return Counted(1.0 / x.v); }
}

#include <cmath>
#include "dp45.hpp"
#include "ham_accel.hpp"
#include "kerr_accel.hpp"

template <bool DIRECT>
struct AccelCount {
    Counted M, a;
    void operator()(int, Counted r, Counted th, Counted ut, Counted ur, Counted uth, Counted uph,
                    Counted &at, Counted &ar, Counted &ath, Counted &aph) const
    {
        g_flops += 2;  // sincos
        Counted s(std::sin(th.v)), c(std::cos(th.v));
        if (DIRECT)
            malbec::kerr_accel_direct<Counted>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
        else
            malbec::kerr_accel<Counted>(M, a, r, s, c, ut, ur, uth, uph, at, ar, ath, aph);
    }
};

struct HamCount {
    Counted M, a;
    malbec::HamConst<Counted> P;
    void operator()(int, Counted r, Counted th, Counted pr, Counted pth, Counted &dt, Counted &dr,
                    Counted &dth, Counted &dph, Counted &dpr, Counted &dpth) const
    {
        g_flops += 2;  // sincos
        Counted s(std::sin(th.v)), c(std::cos(th.v));
        malbec::kerr_ham<Counted>(M, a, r, s, c, pr, pth, P, dt, dr, dth, dph, dpr, dpth);
    }
};

// flops of the compensated update of one component: d + lo, then the two-sum of hi and
// that (s = a + b, b' = s - a, a' = s - b', e = (a - a') + (b - b'): six additions)
constexpr long kCompensated = 7;

template <bool DIRECT>
void count_christoffel(const char *tag)
{
    Counted y[8] = {0.0, 7.0, 1.1, 0.0, 1.2, 0.1, 0.02, 0.05}, y1[8], sr[3];
    AccelCount<DIRECT> f{Counted(1.0), Counted(0.9)};
    Counted at, ar, ath, aph;
    g_flops = g_div = g_fma = g_addmul = 0;
    f(0, y[1], y[2], y[4], y[5], y[6], y[7], at, ar, ath, aph);
    long rhs = g_flops, rhs_div = g_div, rhs_fma = g_fma, rhs_am = g_addmul;
    g_flops = g_div = g_fma = g_addmul = 0;
    malbec::rk4_step(f, Counted(0.02), y, y1, sr);
    std::printf("rhs_flops%s %ld\nrhs_div%s %ld\nrhs_fma%s %ld\nrhs_addmul%s %ld\n", tag, rhs, tag,
                rhs_div, tag, rhs_fma, tag, rhs_am);
    std::printf("step_flops%s %ld\nstep_fma%s %ld\nstep_addmul%s %ld\nstep_div%s %ld\n", tag,
                g_flops, tag, g_fma, tag, g_addmul, tag, g_div);
    // the FP32-compensated step: the increment h/6 (k1 + 2 k2 + 2 k3 + k4), then per
    // component d + lo and Knuth's two-sum with hi (6 additions): kCompensated
    g_flops = g_div = g_fma = g_addmul = 0;
    Counted d[8];
    malbec::rk4_delta(f, Counted(0.02), y, d, sr);
    std::printf("f32k_step_flops%s %ld\n", tag, g_flops + 8 * kCompensated);
    // one Dormand-Prince attempt (six right-hand sides, the stage points, the
    // 5th-order result and the error estimate; the controller's few operations and
    // the pow are not counted)
    malbec::Deriv<Counted> k1, k7;
    for (int c = 0; c < 4; ++c) k1.u[c] = y[4 + c];
    f(0, y[1], y[2], y[4], y[5], y[6], y[7], k1.acc[0], k1.acc[1], k1.acc[2], k1.acc[3]);
    Counted e[8], sr5[5];
    g_flops = g_div = g_fma = g_addmul = 0;
    malbec::dp45_attempt(f, Counted(0.02), y, k1, y1, e, k7, sr5);
    std::printf("dp45_attempt_flops%s %ld\n", tag, g_flops);
}

int main()
{
    count_christoffel<true>("");          // direct form: the roofline's work per step
    count_christoffel<false>("_kernel");  // regrouped form the kernels evaluate

    // Hamilton's equations: z = (t, r, theta, phi, p_t, p_r, p_theta, p_phi); the
    // products a p_t, a p_phi are formed once per lane, not per step
    Counted z[8] = {0.0, 7.0, 1.1, 0.0, -0.95, 0.1, 0.3, 3.0}, z1[8], sr[3];
    HamCount hf{Counted(1.0), Counted(0.9),
                malbec::HamConst<Counted>{z[4], z[7], Counted(0.9 * z[4].v), Counted(0.9 * z[7].v)}};
    Counted dt, dr, dth, dph, dpr, dpth;
    g_flops = g_div = g_fma = g_addmul = 0;
    hf(0, z[1], z[2], z[5], z[6], dt, dr, dth, dph, dpr, dpth);
    long hrhs = g_flops;
    g_flops = g_div = g_fma = g_addmul = 0;
    malbec::rk4_ham_step(hf, Counted(0.02), z, z1, sr);
    std::printf("ham_rhs_flops %ld\nham_step_flops %ld\nham_step_fma %ld\nham_step_addmul %ld\nham_step_div %ld\n",
                hrhs, g_flops, g_fma, g_addmul, g_div);
    g_flops = g_div = g_fma = g_addmul = 0;
    Counted dz[8];
    malbec::rk4_ham_delta(hf, Counted(0.02), z, dz, sr);
    std::printf("f32k_ham_step_flops %ld\n", g_flops + 8 * kCompensated);
    return 0;
}
