"""Coefficients of the float64 sine and cosine polynomials in trig.hpp.

With u = r^2 on |r| <= pi/4 (widened by 1e-4 for the rounding of the
reduction), sin r = r (1 + u P(u)) and cos r = 1 + u Q(u), where P (degree 5)
and Q (degree 6) interpolate (sin r / r - 1) / u and (cos r - 1) / u at the
Chebyshev nodes of [0, (pi/4 * 1.0001)^2].  The target functions come from
their Taylor series summed to 40 terms, everything in 60-digit decimal
arithmetic; the coefficients are then rounded to double.  Printed with the
largest relative error of the rounded polynomials (exact arithmetic, 2001
points): about 2e-17 for the sine and 6e-19 for the cosine, under a quarter
of a double's unit in the last place.

Run: python3 trig_coeffs.py
"""
import math
from decimal import Decimal as D, getcontext

getcontext().prec = 60
PI = D("3.14159265358979323846264338327950288419716939937510582097494459")
U = (PI / 4 * D("1.0001")) ** 2


def sin_target(u):
    """(sin r / r - 1) / u = sum_{k >= 1} (-1)^k u^(k-1) / (2k+1)!"""
    s, t, f = D(0), D(1), D(6)
    for k in range(1, 40):
        s += (-1) ** k * t / f
        t *= u
        f *= (2 * k + 2) * (2 * k + 3)
    return s


def cos_target(u):
    """(cos r - 1) / u = sum_{k >= 1} (-1)^k u^(k-1) / (2k)!"""
    s, t, f = D(0), D(1), D(2)
    for k in range(1, 40):
        s += (-1) ** k * t / f
        t *= u
        f *= (2 * k + 1) * (2 * k + 2)
    return s


def interpolate(g, n):
    """Coefficients (lowest degree first) of the degree-n polynomial through g
    at the n + 1 Chebyshev nodes of [0, U] (Gaussian elimination, partial pivoting)."""
    nodes = [U / 2 * (1 - D(math.cos(math.pi * (2 * i + 1) / (2 * (n + 1))))) for i in range(n + 1)]
    a = [[D(1)] + [x ** j for j in range(1, n + 1)] for x in nodes]
    b = [g(x) for x in nodes]
    m = n + 1
    for c in range(m):
        p = max(range(c, m), key=lambda r: abs(a[r][c]))
        a[c], a[p] = a[p], a[c]
        b[c], b[p] = b[p], b[c]
        for r in range(c + 1, m):
            f = a[r][c] / a[c][c]
            for k in range(c, m):
                a[r][k] -= f * a[c][k]
            b[r] -= f * b[c]
    x = [D(0)] * m
    for r in range(m - 1, -1, -1):
        x[r] = (b[r] - sum(a[r][k] * x[k] for k in range(r + 1, m))) / a[r][r]
    return x


def max_rel_error(coef, g):
    worst = 0.0
    for i in range(1, 2001):
        u = U * i / 2000
        p = D(0)
        for c in reversed(coef):
            p = p * u + D(c)
        exact = 1 + u * g(u)   # sin r / r or cos r
        worst = max(worst, float(abs(u * (p - g(u))) / exact))
    return worst


def main():
    for name, g, n in (("sin", sin_target, 5), ("cos", cos_target, 6)):
        coef = [float(c) for c in interpolate(g, n)]
        print(f"{name}: max rel error {max_rel_error(coef, g):.2e}")
        for j, c in enumerate(coef):
            print(f"  u^{j}: {c!r}")


if __name__ == "__main__":
    main()
