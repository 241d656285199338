// dmath.h -- double-precision sine and cosine for the residual evaluation.
//
// Reduction modulo pi/2 by the Cody-Waite method with pi/2 split into three doubles
// (P1 + P2 + P3 agrees with pi/2 to about 160 bits; each product k*Pi is subtracted
// with one fused multiply-add, so the reduced argument r carries a relative error of
// about 2^-53 for |x| up to 2^30), then the Taylor series of sin (through x^17) and cos
// (through x^16) on |r| <= pi/4, whose truncation error there is below 2^-55.  Larger
// arguments fall back to the library routine.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace comet {

__host__ __device__ inline void sincos_d(double x, double* s, double* c) {
  if (!(fabs(x) < 1073741824.0)) {  // 2^30, and NaN / inf
    *s = sin(x);
    *c = cos(x);
    return;
  }
  const double P1 = 1.5707963267948966, P2 = 6.123233995736766e-17, P3 = -1.4973849048591698e-33;
  const double k = rint(x * 0.6366197723675814);
  double r = fma(-k, P1, x);
  r = fma(-k, P2, r);
  r = fma(-k, P3, r);
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ... + r^16/17!)
  double ps = 2.8114572543455206e-15;  // 1/17!
  ps = fma(ps, r2, -7.647163731819816e-13);   // 1/15!
  ps = fma(ps, r2, 1.6059043836821613e-10);   // 1/13!
  ps = fma(ps, r2, -2.505210838544172e-08);   // 1/11!
  ps = fma(ps, r2, 2.7557319223985893e-06);   // 1/9!
  ps = fma(ps, r2, -1.984126984126984e-04);   // 1/7!
  ps = fma(ps, r2, 8.333333333333333e-03);    // 1/5!
  ps = fma(ps, r2, -1.6666666666666666e-01);  // 1/3!
  const double sr = fma(r * r2, ps, r);
  // cos r = 1 - r^2/2! + r^4/4! - ... + r^16/16!
  double pc = 4.779477332387385e-14;   // 1/16!
  pc = fma(pc, r2, -1.1470745597729725e-11);  // 1/14!
  pc = fma(pc, r2, 2.08767569878681e-09);     // 1/12!
  pc = fma(pc, r2, -2.755731922398589e-07);   // 1/10!
  pc = fma(pc, r2, 2.48015873015873e-05);     // 1/8!
  pc = fma(pc, r2, -1.388888888888889e-03);   // 1/6!
  pc = fma(pc, r2, 4.1666666666666664e-02);   // 1/4!
  pc = fma(pc, r2, -0.5);                     // 1/2!
  const double cr = fma(r2, pc, 1.0);
  const int q = ((int)(long long)k) & 3;
  const double s0 = (q & 1) ? cr : sr;
  const double c0 = (q & 1) ? sr : cr;
  *s = (q & 2) ? -s0 : s0;
  *c = ((q + 1) & 2) ? -c0 : c0;
}

}  // namespace comet
