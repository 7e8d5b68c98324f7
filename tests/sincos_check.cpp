// Host accuracy check of the FP64 link sincos against long-double sin and
// cos: prints, per argument range, the largest error in ulps and absolute.
#include <cmath>
#include <cstdio>
#include <random>

#define AH_SINCOS_QUAL
#include "ah_sincos.h"

static double ulps(double got, long double ref)
{
    const double r = (double)ref;
    const double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    return (double)(fabsl((long double)got - ref) / u);
}

int main()
{
    std::mt19937_64 g(7);
    const double ranges[] = {1e-8, 1.0, 10.0, 1000.0, 1e5, 1e9};
    for (double R : ranges) {
        std::uniform_real_distribution<double> U(-R, R);
        double mu = 0.0, ma = 0.0;
        for (int i = 0; i < 1000000; ++i) {
            const double x = U(g);
            double s, c;
            ah::sincos_reduced(x, &s, &c);
            const long double rs = sinl((long double)x), rc = cosl((long double)x);
            if (std::fabs((double)rs) > 1e-300) mu = std::fmax(mu, ulps(s, rs));
            mu = std::fmax(mu, ulps(c, rc));
            ma = std::fmax(ma, (double)std::fmax(fabsl(s - rs), fabsl(c - rc)));
        }
        std::printf("range %g ulp %.4f abs %.4e\n", R, mu, ma);
    }
    // arguments next to multiples of pi/2, where the reduction cancels: the
    // small one of sin and cos must keep its relative accuracy
    double mu = 0.0;
    for (long long k = -600000000LL; k <= 600000000LL; k += 600013LL) {
        double x = (double)((long double)k * 1.5707963267948966192313216916397514L);
        for (int j = 0; j < 4; ++j) {
            double s, c;
            ah::sincos_reduced(x, &s, &c);
            mu = std::fmax(mu, std::fmax(ulps(s, sinl((long double)x)), ulps(c, cosl((long double)x))));
            x = std::nextafter(x, INFINITY);
        }
    }
    std::printf("nearcut ulp %.4f\n", mu);
    return 0;
}
