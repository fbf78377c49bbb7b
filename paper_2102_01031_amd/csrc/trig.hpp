// trig.hpp -- float64 sine and cosine for the U(1) kernels, whose arguments
// (plaquette angles e dx^2 (curl A), link phases e dx A) are rarely beyond a
// few radians.
//
// Method: Cody-Waite reduction x = r + k pi/2 with pi/2 split into three
// doubles (each product k * part formed inside a fused multiply-add), then
// polynomials on |r| <= pi/4 in u = r^2: sin r = r (1 + u P(u)) with P of
// degree 5 and cos r = 1 + u Q(u) with Q of degree 6, which interpolate the
// exact functions at the Chebyshev nodes of the interval (trig_coeffs.py
// computes them in 60-digit arithmetic; relative error of the rounded
// polynomials about 2e-17 and 6e-19, under a quarter ulp).  They replace the
// Taylor series to r^17 and r^16 with two and one fused multiply-adds fewer.
// Constants: pi/2 and 2/pi rounded to double, the remainders pi/2 - hi and
// pi/2 - hi - mid rounded to double (from pi to 100 digits).
// Arguments beyond 2^20 in magnitude (and NaN, inf) go to the library sincos,
// whose reduction covers the whole range.  Measured against glibc over random
// and special arguments: at most 1 ulp.
//
// The header also compiles for the host (define LAT_HD empty), which is how
// its accuracy is tested.
#pragma once
#include <cmath>

#ifndef LAT_HD
#define LAT_HD __device__
#endif

namespace lat {
namespace trig {

constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kPio2Hi = 0x1.921fb54442d18p+0;
constexpr double kPio2Mid = 0x1.1a62633145c07p-54;
constexpr double kPio2Lo = -0x1.f1976b7ed8fbcp-110;
constexpr double kMaxReduced = 1048576.0;   // 2^20

// sin r = r + r z P(z), z = r^2 (coefficients of P from trig_coeffs.py)
LAT_HD inline double sin_poly(double r, double z)
{
    double p = 1.591810123027412e-10;
    p = fma(p, z, -2.5051131455427946e-08);
    p = fma(p, z, 2.755731610068303e-06);
    p = fma(p, z, -0.0001984126983675497);
    p = fma(p, z, 0.008333333333330946);
    p = fma(p, z, -0.16666666666666666);
    return fma(r * z, p, r);
}

// cos r = 1 + z Q(z), z = r^2 (coefficients of Q from trig_coeffs.py)
LAT_HD inline double cos_poly(double z)
{
    double p = -1.1367978191553177e-11;
    p = fma(p, z, 2.0875886390883725e-09);
    p = fma(p, z, -2.755731556415141e-07);
    p = fma(p, z, 2.480158729368715e-05);
    p = fma(p, z, -0.0013888888888880767);
    p = fma(p, z, 0.04166666666666664);
    p = fma(p, z, -0.5);
    return fma(z, p, 1.0);
}

// x = r + k pi/2 with |r| <= pi/4 (+ rounding); q = k mod 4.  |x| <= 2^20.
LAT_HD inline double reduce(double x, int &q)
{
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kPio2Hi, x);
    r = fma(-k, kPio2Mid, r);
    r = fma(-k, kPio2Lo, r);
    q = (int)k & 3;
    return r;
}

LAT_HD inline void sincos_reduced(double x, double *s, double *c)
{
    int q;
    const double r = reduce(x, q);
    const double z = r * r;
    const double sr = sin_poly(r, z), cr = cos_poly(z);
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

LAT_HD inline double sin_reduced(double x)
{
    int q;
    const double r = reduce(x, q);
    const double z = r * r;
    const double a = (q & 1) ? cos_poly(z) : sin_poly(r, z);
    return (q & 2) ? -a : a;
}

// the library's full-range versions, kept out of line so that the rarely
// taken branch does not add its registers to every call site
LAT_HD __attribute__((noinline)) void sincos_full(double x, double *s, double *c)
{
    sincos(x, s, c);
}

LAT_HD __attribute__((noinline)) double sin_full(double x)
{
    return sin(x);
}

}  // namespace trig

// |x| <= pi/4 needs no reduction (k = 0 gives r = x exactly, so this branch
// returns what the reduced path would); wavefronts whose lanes all take it
// skip the reduction and the quadrant selection
constexpr double kQuarterPi = 0.78539816339744831;

LAT_HD inline void lat_sincos(double x, double *s, double *c)
{
    const double ax = fabs(x);
    if (ax <= kQuarterPi) {
        const double z = x * x;
        *s = trig::sin_poly(x, z);
        *c = trig::cos_poly(z);
    } else if (ax <= trig::kMaxReduced) {
        trig::sincos_reduced(x, s, c);
    } else {
        trig::sincos_full(x, s, c);
    }
}

LAT_HD inline double lat_sin(double x)
{
    const double ax = fabs(x);
    if (ax <= kQuarterPi) return trig::sin_poly(x, x * x);
    return ax <= trig::kMaxReduced ? trig::sin_reduced(x) : trig::sin_full(x);
}

}  // namespace lat
