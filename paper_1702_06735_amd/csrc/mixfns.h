// cosh, sinh, cos and sin in FP64 for the time dependence of Eq. (1)
// (arguments y Gamma t and x Gamma t). Usable on the host (tests) and the
// device.
//
// The device library versions carry a wide-argument path that costs tens of
// registers per lane across a whole kernel; these use Cody-Waite argument
// reduction with fused multiply-adds (exact for |k| < 2^40) and Taylor series
// whose truncation error on the reduced interval is below 1e-17. Accurate to a
// few ulp for |x Gamma t| < 1e6 and |y Gamma t| < 700.
#pragma once

#include <math.h>

#if defined(__HIPCC__)
#define MXA_HD __host__ __device__
#else
#define MXA_HD
#endif

namespace mxa {

constexpr double MIX_LOG2E = 1.4426950408889634;
constexpr double MIX_LN2_HI = 0x1.62e42fefa39efp-1;    // ln 2 rounded to double
constexpr double MIX_LN2_LO = 0x1.abc9e3b39803fp-56;   // ln 2 - MIX_LN2_HI
constexpr double MIX_TWO_OVER_PI = 0.6366197723675814;
constexpr double MIX_PIO2_HI = 0x1.921fb54442d18p+0;   // pi/2 rounded to double
constexpr double MIX_PIO2_LO = 0x1.1a62633145c07p-54;  // pi/2 - MIX_PIO2_HI

// e^u = 2^k e^r with |r| <= ln2 / 2; sum_{n<=13} r^n / n!
MXA_HD inline double mix_exp(double u) {
  const double k = rint(u * MIX_LOG2E);
  double r = fma(-k, MIX_LN2_HI, u);
  r = fma(-k, MIX_LN2_LO, r);
  double p = 1.0 / 6227020800.0;  // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, static_cast<int>(k));
}

// sinh(u) = sum_n u^(2n+1) / (2n+1)! to u^17, for |u| <= 1/2
MXA_HD inline double mix_sinh_small(double u) {
  const double u2 = u * u;
  double p = 1.0 / 355687428096000.0;  // 1/17!
  p = fma(p, u2, 1.0 / 1307674368000.0);
  p = fma(p, u2, 1.0 / 6227020800.0);
  p = fma(p, u2, 1.0 / 39916800.0);
  p = fma(p, u2, 1.0 / 362880.0);
  p = fma(p, u2, 1.0 / 5040.0);
  p = fma(p, u2, 1.0 / 120.0);
  p = fma(p, u2, 1.0 / 6.0);
  return fma(p * u2, u, u);
}

MXA_HD inline void mix_cosh_sinh(double u, double* ch, double* sh) {
  const double e = mix_exp(u), ie = 1.0 / e;
  *ch = 0.5 * (e + ie);
  *sh = fabs(u) <= 0.5 ? mix_sinh_small(u) : 0.5 * (e - ie);
}

// v = k pi/2 + r with |r| <= pi/4:
// sin r = sum_n (-1)^n r^(2n+1) / (2n+1)! to r^19,
// cos r = sum_n (-1)^n r^(2n) / (2n)! to r^18.
MXA_HD inline void mix_sincos(double v, double* sn, double* cs) {
  const double k = rint(v * MIX_TWO_OVER_PI);
  double r = fma(-k, MIX_PIO2_HI, v);
  r = fma(-k, MIX_PIO2_LO, r);
  const double r2 = r * r;
  double s = -1.0 / 121645100408832000.0;  // -1/19!
  s = fma(s, r2, 1.0 / 355687428096000.0);
  s = fma(s, r2, -1.0 / 1307674368000.0);
  s = fma(s, r2, 1.0 / 6227020800.0);
  s = fma(s, r2, -1.0 / 39916800.0);
  s = fma(s, r2, 1.0 / 362880.0);
  s = fma(s, r2, -1.0 / 5040.0);
  s = fma(s, r2, 1.0 / 120.0);
  s = fma(s, r2, -1.0 / 6.0);
  s = fma(s * r2, r, r);
  double c = -1.0 / 6402373705728000.0;  // -1/18!
  c = fma(c, r2, 1.0 / 20922789888000.0);
  c = fma(c, r2, -1.0 / 87178291200.0);
  c = fma(c, r2, 1.0 / 479001600.0);
  c = fma(c, r2, -1.0 / 3628800.0);
  c = fma(c, r2, 1.0 / 40320.0);
  c = fma(c, r2, -1.0 / 720.0);
  c = fma(c, r2, 1.0 / 24.0);
  c = fma(c, r2, -0.5);
  c = fma(c, r2, 1.0);
  const int q = static_cast<int>(static_cast<long long>(k) & 3);
  const double ss = (q & 1) ? c : s, cc = (q & 1) ? s : c;
  *sn = (q & 2) ? -ss : ss;
  *cs = ((q + 1) & 2) ? -cc : cc;
}

}  // namespace mxa
