// perrk_log.h -- double-precision logarithms for the kernels' entropy arithmetic
// (entropy variables, entropy densities, the relaxation residual, the
// logarithmic mean's fallback).  The runtime library's log and log1p in double
// precision take about 100 and 135 vector instructions; these take about 30
// and 40, with an error of a few units in the last place.
//
// log(x), x = m 2^e with m in [sqrt(1/2), sqrt(2)):
//   log x = e ln 2 + 2 atanh(t),  t = (m - 1) / (m + 1),  |t| <= 3 - 2 sqrt 2 < 0.1716,
//   atanh(t) = t (1 + s/3 + s^2/5 + ... + s^10/21),  s = t^2 <= 0.0295
// (the first omitted term, s^11/23, is below 1e-18 relative).  m - 1 is exact
// (Sterbenz), so t carries the rounding of m + 1 and of the reciprocal only.
// ln 2 is split into a head of 32 significant bits (e ln2_hi is exact for
// |e| < 2^21) and a tail.
// log1p(x) = x log(u) / (u - 1) with u = 1 + x rounded (u != 1), x where
// u == 1: the rounding of u cancels to first order between log(u) and u - 1.
//
// Both are templates on the reciprocal in use (a functor), so that the same
// arithmetic compiles for the device (hardware reciprocal refined by Newton
// steps) and for a host-side accuracy test.
#pragma once

#include <math.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#define __forceinline__ inline
#endif

namespace perrk_log {

constexpr double LN2_HI = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
constexpr double LN2_LO = 1.90821492927058770002e-10;  // ln 2 - LN2_HI
constexpr double SQRT_HALF = 0.70710678118654752440;

template <typename Rcp>
__host__ __device__ __forceinline__ double log_f64(double x, Rcp rcp)
{
    int e = 0;
    double m = frexp(x, &e);  // m in [1/2, 1) for finite nonzero x
    const bool low = m < SQRT_HALF;
    m = low ? m + m : m;
    e = low ? e - 1 : e;
    const double t = (m - 1.0) * rcp(m + 1.0);
    const double s = t * t;
    // 2 atanh(t) / t = 2 (1 + s/3 + ... + s^10/21)
    double P = 2.0 / 21.0;
    P = fma(P, s, 2.0 / 19.0);
    P = fma(P, s, 2.0 / 17.0);
    P = fma(P, s, 2.0 / 15.0);
    P = fma(P, s, 2.0 / 13.0);
    P = fma(P, s, 2.0 / 11.0);
    P = fma(P, s, 2.0 / 9.0);
    P = fma(P, s, 2.0 / 7.0);
    P = fma(P, s, 2.0 / 5.0);
    P = fma(P, s, 2.0 / 3.0);
    P = fma(P, s, 2.0);
    const double de = (double)e;
    double r = fma(de, LN2_LO, t * P);
    r = fma(de, LN2_HI, r);
    // zero, negative, NaN and infinite arguments
    r = x > 0.0 ? r : (x == 0.0 ? -INFINITY : NAN);
    return x == INFINITY ? x : r;
}

template <typename Rcp>
__host__ __device__ __forceinline__ double log1p_f64(double x, Rcp rcp)
{
    const double u = 1.0 + x;
    const double um1 = u - 1.0;
    const double r = log_f64(u, rcp) * (x * rcp(um1));
    return (um1 == 0.0 || x == INFINITY) ? x : r;
}

}  // namespace perrk_log
