// sin and cos in FP64 for |x| <= 1e9, written for the link variables of the
// FP64 step (exp(-i dx A) once per link), cheaper than the general library
// routine, whose range reduction covers every double.
//
// x = k pi/2 + r with |r| <= pi/4: k = rint(2x/pi), and pi/2 in five parts
// (Cody-Waite) whose first four carry 22 significant bits, so that k * part
// is exact for |k| < 2^31 and the reduction keeps ~140 bits of pi/2.
// sin r and cos r come from their Taylor series to degree 17 and 18: on
// |r| <= pi/4 the first omitted terms are below 1e-19.  Measured against
// long-double sin and cos: within 1.6 ulp for |x| <= 1e3 and 2.4 ulp (1.5e-16
// absolute) for |x| <= 1e9.
//
// The including file defines AH_SINCOS_QUAL (__device__ for kernels, empty
// for the host accuracy test).
#pragma once

#include <cmath>

#ifndef AH_SINCOS_QUAL
#error "define AH_SINCOS_QUAL before including ah_sincos.h"
#endif

namespace ah {

AH_SINCOS_QUAL inline void sincos_reduced(double x, double* s, double* c)
{
    // 2/pi, and pi/2 = p1 + ... + p5 (from pi to 90 digits by Machin's formula)
    const double two_over_pi = 0x1.45f306dc9c883p-1;
    const double p1 = 0x1.921fb00000000p+0, p2 = 0x1.5110b00000000p-22, p3 = 0x1.1846980000000p-44;
    const double p4 = 0x1.3198a00000000p-69, p5 = 0x1.701b839a25205p-92;
    const double k = rint(x * two_over_pi);
    double r = fma(-k, p1, x);
    r = fma(-k, p2, r);
    r = fma(-k, p3, r);
    r = fma(-k, p4, r);
    r = fma(-k, p5, r);
    const double z = r * r;
    // sin r = r + r z (-1/3! + z (1/5! + z (-1/7! + ...)))
    double ps = 1.0 / 355687428096000.0;  // 1/17!
    ps = fma(ps, z, -1.0 / 1307674368000.0);
    ps = fma(ps, z, 1.0 / 6227020800.0);
    ps = fma(ps, z, -1.0 / 39916800.0);
    ps = fma(ps, z, 1.0 / 362880.0);
    ps = fma(ps, z, -1.0 / 5040.0);
    ps = fma(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double sr = fma(r * z, ps, r);
    // cos r = 1 - z/2 + z^2 (1/4! + z (-1/6! + ...)), with the rounding error
    // of 1 - z/2 carried into the tail
    double pc = -1.0 / 6402373705728000.0;  // -1/18!
    pc = fma(pc, z, 1.0 / 20922789888000.0);
    pc = fma(pc, z, -1.0 / 87178291200.0);
    pc = fma(pc, z, 1.0 / 479001600.0);
    pc = fma(pc, z, -1.0 / 3628800.0);
    pc = fma(pc, z, 1.0 / 40320.0);
    pc = fma(pc, z, -1.0 / 720.0);
    pc = fma(pc, z, 1.0 / 24.0);
    const double hz = 0.5 * z;
    const double w = 1.0 - hz;
    const double cr = w + (((1.0 - w) - hz) + (z * z) * pc);
    // quadrant k mod 4
    const int q = (int)((long long)k & 3);
    const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}

}  // namespace ah
