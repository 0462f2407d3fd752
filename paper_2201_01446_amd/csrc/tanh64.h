// tanh64.h -- FP64 tanh for the network activations (host and device).
//
// gfx950 has no FP64 exponential instruction, and the library tanh spends
// about 160 FP64 instructions per call on a double-double exponential.  The
// activations need a few ulp, not a correctly rounded result, so:
//
//   tanh|x| = u / (u + 2),  u = e^y - 1,  y = 2|x|,  sign restored;
//
// and 1 for |x| >= 20 (1 - tanh 20 < 2^-57); a NaN stays a NaN.  e^y - 1
// uses the Cody-Waite reduction y = n ln2 + r with ln2 split into a high
// part whose last 11 bits are zero (n ln2_hi is exact for |n| < 2^11) and a
// low part, |r| <= ln2/2; e^r - 1 from its Taylor series to r^14 in Horner
// form (the remainder is below 2^-60 relative there); then
// e^y - 1 = 2^n (e^r - 1) + (2^n - 1), which for n >= 1 cancels at most 1.3
// bits (u >= 0.41).  Against the C library's tanh over [-25, 25] and random
// points down to 1e-300: at most 3 ulp (the tests hold it to 4).  About 40
// FP64 instructions, no branches.
#pragma once

#include <hip/hip_runtime.h>

namespace dp {

__host__ __device__ inline double tanh_f64(double x)
{
    const double ax = fabs(x);
    const double y = 2.0 * ax > 40.0 ? 40.0 : 2.0 * ax;   // (a NaN goes through)
    const double ln2_hi = 0x1.62e42fefa3800p-1;   // ln 2 to 42 bits
    const double ln2_lo = 0x1.ef35793c76730p-45;  // ln 2 - ln2_hi
    const double n = rint(y * 0x1.71547652b82fep0);   // y / ln 2
    double r = fma(-n, ln2_hi, y);
    r = fma(-n, ln2_lo, r);
    // e^r - 1 = r (1 + r/2! + r^2/3! + ... + r^13/14!)
    double q = 1.0 / 87178291200.0;   // 1/14!
    q = fma(q, r, 1.0 / 6227020800.0);
    q = fma(q, r, 1.0 / 479001600.0);
    q = fma(q, r, 1.0 / 39916800.0);
    q = fma(q, r, 1.0 / 3628800.0);
    q = fma(q, r, 1.0 / 362880.0);
    q = fma(q, r, 1.0 / 40320.0);
    q = fma(q, r, 1.0 / 5040.0);
    q = fma(q, r, 1.0 / 720.0);
    q = fma(q, r, 1.0 / 120.0);
    q = fma(q, r, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    const double em1 = q * r;
    const int ni = (int)n;
    const double p2 = ldexp(1.0, ni);
    const double u = fma(p2, em1, p2 - 1.0);   // 2^n (e^r - 1) + (2^n - 1)
    const double t = ax >= 20.0 ? 1.0 : u / (u + 2.0);
    return copysign(t, x);
}

}  // namespace dp
