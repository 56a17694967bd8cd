// Forward-mode dual numbers with two tangent directions (d/dr, d/dtheta), used to
// differentiate the position-dependent coefficients of the acceleration in the
// adjoint.  Exact derivatives of the computed expressions (no truncation).
#pragma once

#include "kerr_accel.hpp"

namespace malbec {

using ::fma;  // keep the scalar overloads visible next to the dual one

template <typename T>
struct Dual2 {
    T v, dr, dth;
    MALBEC_HD Dual2() : v(0), dr(0), dth(0) {}
    MALBEC_HD Dual2(T x) : v(x), dr(0), dth(0) {}
    MALBEC_HD Dual2(T x, T a, T b) : v(x), dr(a), dth(b) {}
};

template <typename T>
MALBEC_HD inline Dual2<T> operator+(Dual2<T> a, Dual2<T> b) { return {a.v + b.v, a.dr + b.dr, a.dth + b.dth}; }
template <typename T>
MALBEC_HD inline Dual2<T> operator-(Dual2<T> a, Dual2<T> b) { return {a.v - b.v, a.dr - b.dr, a.dth - b.dth}; }
template <typename T>
MALBEC_HD inline Dual2<T> operator-(Dual2<T> a) { return {-a.v, -a.dr, -a.dth}; }
template <typename T>
MALBEC_HD inline Dual2<T> operator*(Dual2<T> a, Dual2<T> b)
{
    return {a.v * b.v, fma(a.dr, b.v, a.v * b.dr), fma(a.dth, b.v, a.v * b.dth)};
}
template <typename T>
MALBEC_HD inline Dual2<T> fma(Dual2<T> a, Dual2<T> b, Dual2<T> c)
{
    return {fma(a.v, b.v, c.v), fma(a.dr, b.v, fma(a.v, b.dr, c.dr)),
            fma(a.dth, b.v, fma(a.v, b.dth, c.dth))};
}
template <typename T>
MALBEC_HD inline Dual2<T> recip(Dual2<T> a)
{
    const T iv = recip(a.v);
    const T d = -iv * iv;
    return {iv, d * a.dr, d * a.dth};
}

}  // namespace malbec
