// Embedded Runge-Kutta pair of Dormand and Prince, 5(4) (J. Comput. Appl. Math. 6
// (1980) 19-26), one attempt of the geodesic ODE in the Christoffel form, shared by
// the adaptive kernel and the host flop counter.
//
// Seven stages; the seventh is evaluated at the new point with the 5th-order weights
// (first same as last: it is the first stage of the next step).  The right-hand side
// depends on (r, theta, u) only, so stage points are formed for those six components
// and t, phi only accumulate.  Stage k of an attempt keeps the 4-velocity U_k and the
// acceleration A_k of its stage point; the derivative of (t, r, theta, phi) there is
// U_k.
#pragma once

#include "kerr_accel.hpp"

namespace malbec {

// Butcher tableau: rows 2..7 of A (row 7 = the 5th-order weights b), and the
// weights of the error estimate e = b - b* (b* the 4th-order companion).
struct DP45 {
    static constexpr double a21 = 1.0 / 5;
    static constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
    static constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
    static constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561,
                            a54 = -212.0 / 729;
    static constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247,
                            a64 = 49.0 / 176, a65 = -5103.0 / 18656;
    static constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192,
                            b5 = -2187.0 / 6784, b6 = 11.0 / 84;
    static constexpr double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920,
                            e5 = -17253.0 / 339200, e6 = 22.0 / 525, e7 = -1.0 / 40;
};

// Derivative of the 8-component state at a stage point: (U, A).
template <typename T>
struct Deriv {
    T u[4], acc[4];
};

// One attempt of size h from y, with k1 = f(y) given.  Writes y1 (5th order), the
// error estimate e (y1 minus the 4th-order solution), k7 = f(y1), and the radii of
// stage points 2..6.  accel(stage, r, th, ut, ur, uth, uph, at, ar, ath, aph)
// evaluates the acceleration at stage point `stage` (1..6 here; 0 is the step's
// start, whose derivative is k1).
template <typename T, typename Accel>
MALBEC_HD inline void dp45_attempt(Accel &accel, T h, const T y[8], const Deriv<T> &k1, T y1[8],
                                   T e[8], Deriv<T> &k7, T sr[5])
{
    typedef DP45 D;
    Deriv<T> k2, k3, k4, k5, k6;
    // stage points y + h sum_j a_sj k_j of (r, theta, u); constant weights
    {
        const T r = fma(h * T(D::a21), k1.u[1], y[1]);
        const T th = fma(h * T(D::a21), k1.u[2], y[2]);
        for (int c = 0; c < 4; ++c) k2.u[c] = fma(h * T(D::a21), k1.acc[c], y[4 + c]);
        sr[0] = r;
        accel(1, r, th, k2.u[0], k2.u[1], k2.u[2], k2.u[3], k2.acc[0], k2.acc[1], k2.acc[2], k2.acc[3]);
    }
    {
        const T r = fma(h, fma(T(D::a31), k1.u[1], T(D::a32) * k2.u[1]), y[1]);
        const T th = fma(h, fma(T(D::a31), k1.u[2], T(D::a32) * k2.u[2]), y[2]);
        for (int c = 0; c < 4; ++c)
            k3.u[c] = fma(h, fma(T(D::a31), k1.acc[c], T(D::a32) * k2.acc[c]), y[4 + c]);
        sr[1] = r;
        accel(2, r, th, k3.u[0], k3.u[1], k3.u[2], k3.u[3], k3.acc[0], k3.acc[1], k3.acc[2], k3.acc[3]);
    }
    {
        auto comb = [&](const T &x1, const T &x2, const T &x3) {
            return fma(T(D::a41), x1, fma(T(D::a42), x2, T(D::a43) * x3));
        };
        const T r = fma(h, comb(k1.u[1], k2.u[1], k3.u[1]), y[1]);
        const T th = fma(h, comb(k1.u[2], k2.u[2], k3.u[2]), y[2]);
        for (int c = 0; c < 4; ++c) k4.u[c] = fma(h, comb(k1.acc[c], k2.acc[c], k3.acc[c]), y[4 + c]);
        sr[2] = r;
        accel(3, r, th, k4.u[0], k4.u[1], k4.u[2], k4.u[3], k4.acc[0], k4.acc[1], k4.acc[2], k4.acc[3]);
    }
    {
        auto comb = [&](const T &x1, const T &x2, const T &x3, const T &x4) {
            return fma(T(D::a51), x1, fma(T(D::a52), x2, fma(T(D::a53), x3, T(D::a54) * x4)));
        };
        const T r = fma(h, comb(k1.u[1], k2.u[1], k3.u[1], k4.u[1]), y[1]);
        const T th = fma(h, comb(k1.u[2], k2.u[2], k3.u[2], k4.u[2]), y[2]);
        for (int c = 0; c < 4; ++c)
            k5.u[c] = fma(h, comb(k1.acc[c], k2.acc[c], k3.acc[c], k4.acc[c]), y[4 + c]);
        sr[3] = r;
        accel(4, r, th, k5.u[0], k5.u[1], k5.u[2], k5.u[3], k5.acc[0], k5.acc[1], k5.acc[2], k5.acc[3]);
    }
    {
        auto comb = [&](const T &x1, const T &x2, const T &x3, const T &x4, const T &x5) {
            return fma(T(D::a61), x1,
                       fma(T(D::a62), x2, fma(T(D::a63), x3, fma(T(D::a64), x4, T(D::a65) * x5))));
        };
        const T r = fma(h, comb(k1.u[1], k2.u[1], k3.u[1], k4.u[1], k5.u[1]), y[1]);
        const T th = fma(h, comb(k1.u[2], k2.u[2], k3.u[2], k4.u[2], k5.u[2]), y[2]);
        for (int c = 0; c < 4; ++c)
            k6.u[c] = fma(h, comb(k1.acc[c], k2.acc[c], k3.acc[c], k4.acc[c], k5.acc[c]), y[4 + c]);
        sr[4] = r;
        accel(5, r, th, k6.u[0], k6.u[1], k6.u[2], k6.u[3], k6.acc[0], k6.acc[1], k6.acc[2], k6.acc[3]);
    }
    // 5th-order solution (b2 = 0) for all 8 components: x from U, u from A
    auto bsum = [&](const T &x1, const T &x3, const T &x4, const T &x5, const T &x6) {
        return fma(T(D::b1), x1, fma(T(D::b3), x3, fma(T(D::b4), x4, fma(T(D::b5), x5, T(D::b6) * x6))));
    };
    y1[0] = fma(h, bsum(k1.u[0], k3.u[0], k4.u[0], k5.u[0], k6.u[0]), y[0]);
    y1[1] = fma(h, bsum(k1.u[1], k3.u[1], k4.u[1], k5.u[1], k6.u[1]), y[1]);
    y1[2] = fma(h, bsum(k1.u[2], k3.u[2], k4.u[2], k5.u[2], k6.u[2]), y[2]);
    y1[3] = fma(h, bsum(k1.u[3], k3.u[3], k4.u[3], k5.u[3], k6.u[3]), y[3]);
    for (int c = 0; c < 4; ++c)
        y1[4 + c] = fma(h, bsum(k1.acc[c], k3.acc[c], k4.acc[c], k5.acc[c], k6.acc[c]), y[4 + c]);
    // seventh stage at y1 (first same as last)
    for (int c = 0; c < 4; ++c) k7.u[c] = y1[4 + c];
    accel(6, y1[1], y1[2], k7.u[0], k7.u[1], k7.u[2], k7.u[3], k7.acc[0], k7.acc[1], k7.acc[2],
          k7.acc[3]);
    // error estimate (e2 = 0)
    auto esum = [&](const T &x1, const T &x3, const T &x4, const T &x5, const T &x6, const T &x7) {
        return fma(T(D::e1), x1, fma(T(D::e3), x3, fma(T(D::e4), x4, fma(T(D::e5), x5,
                   fma(T(D::e6), x6, T(D::e7) * x7)))));
    };
    for (int c = 0; c < 4; ++c) {
        e[c] = h * esum(k1.u[c], k3.u[c], k4.u[c], k5.u[c], k6.u[c], k7.u[c]);
        e[4 + c] = h * esum(k1.acc[c], k3.acc[c], k4.acc[c], k5.acc[c], k6.acc[c], k7.acc[c]);
    }
}

}  // namespace malbec
