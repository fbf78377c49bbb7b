// Host build of the library's float64 sine/cosine (csrc/trig.hpp), compared
// with glibc over random and special arguments; prints the worst error in
// ulp of the reference result for each argument range.
#define LAT_HD
#include "trig.hpp"
#include <cstdio>
#include <cstdint>
#include <cmath>
#include <random>
#include <vector>

static double ulp_err(double got, double ref)
{
    if (got == ref) return 0.0;
    const double u = std::nextafter(std::fabs(ref), INFINITY) - std::fabs(ref);
    return std::fabs(got - ref) / u;
}

int main()
{
    std::mt19937_64 rng(12345);
    struct Range { double lo, hi; const char *name; };
    const Range ranges[] = {{-1e-3, 1e-3, "tiny"}, {-0.8, 0.8, "quarter"}, {-4.0, 4.0, "small"},
                            {-100.0, 100.0, "medium"}, {-1048576.0, 1048576.0, "large"},
                            {-1e7, 1e7, "fallback"}};
    for (const Range &R : ranges) {
        std::uniform_real_distribution<double> d(R.lo, R.hi);
        double ws = 0, wc = 0, w1 = 0;
        for (int i = 0; i < 2000000; ++i) {
            const double x = d(rng);
            double s, c;
            lat::lat_sincos(x, &s, &c);
            ws = std::fmax(ws, ulp_err(s, std::sin(x)));
            wc = std::fmax(wc, ulp_err(c, std::cos(x)));
            w1 = std::fmax(w1, ulp_err(lat::lat_sin(x), std::sin(x)));
        }
        std::printf("%s %.3f %.3f %.3f\n", R.name, ws, wc, w1);
    }
    // special arguments: zeros, quarter-period boundaries, multiples of pi/2 and their neighbours
    double ws = 0, wc = 0, w1 = 0;
    std::vector<double> xs = {0.0, -0.0, 1e-300, -1e-300, 5e-324, M_PI_4, -M_PI_4, M_PI_2, M_PI, 3 * M_PI_2,
                              2 * M_PI, 1048576.0, -1048576.0};
    for (int k = -2000; k <= 2000; ++k) {
        const double x = k * M_PI_2;
        xs.push_back(x);
        xs.push_back(std::nextafter(x, INFINITY));
        xs.push_back(std::nextafter(x, -INFINITY));
        xs.push_back(x + M_PI_4);
        xs.push_back(std::nextafter(x + M_PI_4, 0.0));
    }
    for (double x : xs) {
        double s, c;
        lat::lat_sincos(x, &s, &c);
        ws = std::fmax(ws, ulp_err(s, std::sin(x)));
        wc = std::fmax(wc, ulp_err(c, std::cos(x)));
        w1 = std::fmax(w1, ulp_err(lat::lat_sin(x), std::sin(x)));
    }
    std::printf("special %.3f %.3f %.3f\n", ws, wc, w1);
    double s, c;
    lat::lat_sincos(NAN, &s, &c);
    std::printf("nan %d %d\n", (int)std::isnan(s), (int)std::isnan(c));
    return 0;
}
