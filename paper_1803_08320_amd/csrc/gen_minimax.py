"""Coefficients of the sin / cos polynomials of kerr_device.hpp (sincos_reduce, FP64)
and mixed.hip (sincos_f32, FP32).

After the reduction x = theta - k pi/2 the kernels evaluate, on |x| <= pi/4,
    sin x = x + x^3 P(x^2),   P of degree 5 (FP64) or 2 (FP32),
    cos x = 1 - x^2 Q(x^2),   Q of degree 6 (FP64) or 3 (FP32).
P and Q are the minimax (equi-oscillating) approximations of (sin x - x) / x^3 and
(1 - cos x) / x^2 as functions of z = x^2 on [0, (pi/4)^2], found with the Remez
exchange algorithm in 60-digit arithmetic (mpmath).  The script prints the
coefficients rounded to double (resp. single) precision, lowest degree first, and
the maximum relative error of sin and cos with the rounded coefficients (exact
arithmetic otherwise).

    python gen_minimax.py
"""
import struct

import mpmath as mp

mp.mp.dps = 60
X = mp.pi / 4 * (1 + mp.mpf(2) ** -40)  # the reduced argument's range, with margin
Z = X * X


def remez(f, n, iters=30, grid=4000):
    """Minimax polynomial of degree n - 1 for f on [0, Z] (coefficients, error)."""
    m = n + 1
    ref = [Z * (1 - mp.cos(mp.pi * i / (m - 1))) / 2 for i in range(m)]
    err_max = None
    for _ in range(iters):
        A = mp.matrix(m, m)
        b = mp.matrix(m, 1)
        for i, z in enumerate(ref):
            for j in range(n):
                A[i, j] = z ** j
            A[i, n] = (-1) ** i
            b[i] = f(z)
        sol = mp.lu_solve(A, b)
        c = [sol[j] for j in range(n)]

        def err(z):
            return sum(c[j] * z ** j for j in range(n)) - f(z)
        zs = [Z * mp.mpf(k) / grid for k in range(grid + 1)]
        es = [err(z) for z in zs]
        # local extrema of |err| (end points included), then one per sign run
        ext = []
        for k, e in enumerate(es):
            lo = es[k - 1] if k > 0 else None
            hi = es[k + 1] if k + 1 < len(es) else None
            if (lo is None or abs(e) >= abs(lo)) and (hi is None or abs(e) >= abs(hi)):
                ext.append((zs[k], e))
        alt = []
        for z, e in ext:
            if alt and mp.sign(alt[-1][1]) == mp.sign(e):
                if abs(e) > abs(alt[-1][1]):
                    alt[-1] = (z, e)
            else:
                alt.append((z, e))
        while len(alt) > m:
            alt.pop(0 if abs(alt[0][1]) < abs(alt[-1][1]) else -1)
        if len(alt) < m:
            break
        ref = [z for z, _ in alt]
        err_max = max(abs(e) for _, e in alt)
    return c, err_max


def f_sin(z):
    if z == 0:
        return mp.mpf(-1) / 6
    x = mp.sqrt(z)
    return (mp.sin(x) - x) / x ** 3


def f_cos(z):
    if z == 0:
        return mp.mpf(1) / 2
    x = mp.sqrt(z)
    return (1 - mp.cos(x)) / z


def to_single(v):
    return struct.unpack("f", struct.pack("f", float(v)))[0]


def report(name, n_sin, n_cos, rnd):
    P, _ = remez(f_sin, n_sin)
    Q, _ = remez(f_cos, n_cos)
    Pr = [mp.mpf(rnd(v)) for v in P]
    Qr = [mp.mpf(rnd(v)) for v in Q]
    xs = [X * mp.mpf(k) / 3000 for k in range(1, 3001)]

    def poly(c, z):
        return sum(c[j] * z ** j for j in range(len(c)))
    es = max(abs((x + x ** 3 * poly(Pr, x * x) - mp.sin(x)) / mp.sin(x)) for x in xs)
    ec = max(abs((1 - x * x * poly(Qr, x * x) - mp.cos(x)) / mp.cos(x)) for x in xs)
    print(name)
    print("  P (sin):", ", ".join(repr(rnd(v)) for v in P))
    print("  Q (cos):", ", ".join(repr(rnd(v)) for v in Q))
    print("  max relative error with rounded coefficients: sin %s, cos %s"
          % (mp.nstr(es, 3), mp.nstr(ec, 3)))


def main():
    report("FP64 (sincos_reduce)", 6, 7, float)
    report("FP32 (sincos_f32)", 3, 4, to_single)


if __name__ == "__main__":
    main()
