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
//
// Register economy: k1..k3 are kept whole until the fifth stage point is formed; from
// then on every derivative is folded, as soon as it is known, into running sums of the
// sixth stage point, of the 5th-order weights (yb) and of the error weights (ee), so
// at most three derivatives are live at once and none is live at the seventh stage.
// The operation count is that of the plain weighted sums; only their order differs.
template <typename T, typename Accel>
MALBEC_HD inline void dp45_attempt(Accel &accel, T h, const T y[8], const Deriv<T> &k1, T y1[8],
                                   T e[8], Deriv<T> &k7, T sr[5])
{
    typedef DP45 D;
    Deriv<T> k2, k3;
    T u4[4], a4[4];
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
        for (int c = 0; c < 4; ++c) u4[c] = fma(h, comb(k1.acc[c], k2.acc[c], k3.acc[c]), y[4 + c]);
        sr[2] = r;
        accel(3, r, th, u4[0], u4[1], u4[2], u4[3], a4[0], a4[1], a4[2], a4[3]);
    }
    // the fifth stage point, then k1..k4 folded into the running sums
    T u5[4], a5[4];
    const T r5 = fma(h, fma(T(D::a51), k1.u[1], fma(T(D::a52), k2.u[1],
                            fma(T(D::a53), k3.u[1], T(D::a54) * u4[1]))), y[1]);
    const T th5 = fma(h, fma(T(D::a51), k1.u[2], fma(T(D::a52), k2.u[2],
                             fma(T(D::a53), k3.u[2], T(D::a54) * u4[2]))), y[2]);
    for (int c = 0; c < 4; ++c)
        u5[c] = fma(h, fma(T(D::a51), k1.acc[c], fma(T(D::a52), k2.acc[c],
                           fma(T(D::a53), k3.acc[c], T(D::a54) * a4[c]))), y[4 + c]);
    // p6: a_6j-weighted sum over j <= 4 of the six components a stage point needs
    // (r, theta from U; the four velocities from A); yb, ee: b_j- and e_j-weighted
    // sums of all eight (b2 = e2 = 0)
    T p6[6], yb[8], ee[8];
    {
        auto six = [&](const Deriv<T> &k, int j) { return j < 2 ? k.u[1 + j] : k.acc[j - 2]; };
        for (int j = 0; j < 6; ++j) {
            const T v4 = j < 2 ? u4[1 + j] : a4[j - 2];
            p6[j] = fma(T(D::a64), v4, fma(T(D::a63), six(k3, j),
                        fma(T(D::a62), six(k2, j), T(D::a61) * six(k1, j))));
        }
        for (int c = 0; c < 8; ++c) {
            const T v1 = c < 4 ? k1.u[c] : k1.acc[c - 4];
            const T v3 = c < 4 ? k3.u[c] : k3.acc[c - 4];
            const T v4 = c < 4 ? u4[c] : a4[c - 4];
            yb[c] = fma(T(D::b4), v4, fma(T(D::b3), v3, T(D::b1) * v1));
            ee[c] = fma(T(D::e4), v4, fma(T(D::e3), v3, T(D::e1) * v1));
        }
    }
    sr[3] = r5;
    accel(4, r5, th5, u5[0], u5[1], u5[2], u5[3], a5[0], a5[1], a5[2], a5[3]);
    // the sixth stage point; k5 folded
    T u6[4], a6[4];
    const T r6 = fma(h, fma(T(D::a65), u5[1], p6[0]), y[1]);
    const T th6 = fma(h, fma(T(D::a65), u5[2], p6[1]), y[2]);
    for (int c = 0; c < 4; ++c) u6[c] = fma(h, fma(T(D::a65), a5[c], p6[2 + c]), y[4 + c]);
    for (int c = 0; c < 8; ++c) {
        const T v5 = c < 4 ? u5[c] : a5[c - 4];
        yb[c] = fma(T(D::b5), v5, yb[c]);
        ee[c] = fma(T(D::e5), v5, ee[c]);
    }
    sr[4] = r6;
    accel(5, r6, th6, u6[0], u6[1], u6[2], u6[3], a6[0], a6[1], a6[2], a6[3]);
    // 5th-order solution for all 8 components: x from U, u from A
    for (int c = 0; c < 8; ++c) {
        const T v6 = c < 4 ? u6[c] : a6[c - 4];
        y1[c] = fma(h, fma(T(D::b6), v6, yb[c]), y[c]);
        ee[c] = fma(T(D::e6), v6, ee[c]);
    }
    // seventh stage at y1 (first same as last)
    for (int c = 0; c < 4; ++c) k7.u[c] = y1[4 + c];
    accel(6, y1[1], y1[2], k7.u[0], k7.u[1], k7.u[2], k7.u[3], k7.acc[0], k7.acc[1], k7.acc[2],
          k7.acc[3]);
    // error estimate
    for (int c = 0; c < 4; ++c) {
        e[c] = h * fma(T(D::e7), k7.u[c], ee[c]);
        e[4 + c] = h * fma(T(D::e7), k7.acc[c], ee[4 + c]);
    }
}

}  // namespace malbec
