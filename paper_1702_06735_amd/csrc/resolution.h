// Gaussian decay-time resolution (an extension of Eq. (1), which is stated
// for perfectly measured decay times). Usable on the host (tests) and the
// device.
//
// With resolution width sigma, each exponential of the rate is replaced by its
// convolution with the Gaussian,
//   E(a; t) = int_0^inf e^{-a t'} G(t - t'; sigma) dt'
//           = 1/2 exp(a^2 sigma^2 / 2 - a t) erfc(u),  u = (a sigma^2 - t) / (sqrt 2 sigma),
// for complex a with Re a > 0. With the Faddeeva function w(z) = exp(-z^2)
// erfc(-i z): E = 1/2 exp(-t^2 / (2 sigma^2)) w(i u) when Re u >= 0, and
// E = exp(a^2 sigma^2 / 2 - a t) - 1/2 exp(-t^2 / (2 sigma^2)) w(-i u) when
// Re u < 0 (from erfc(u) = 2 - erfc(-u)), so that w is only taken in the upper
// half plane and nothing overflows. The derivative in a follows from the first
// form: dE/da = (a sigma^2 - t) E - sigma / sqrt(2 pi) exp(-t^2 / (2 sigma^2)).
#pragma once

#include "faddeeva_coef.h"
#include "mixfns.h"

namespace mxa {

struct Cd {
  double re, im;
};
MXA_HD inline Cd cd_mul(Cd a, Cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
MXA_HD inline Cd cd_div(Cd a, Cd b) {
  const double d = 1.0 / (b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}

// w(z) for Im z >= 0 by Weideman's rational series (N = 36; relative error
// below 3e-14 against a reference implementation over the upper half plane).
MXA_HD inline Cd faddeeva_upper(Cd z) {
  const double L = FADDEEVA_L;
  const Cd lp = {L - z.im, z.re};   // L + i z
  const Cd lm = {L + z.im, -z.re};  // L - i z
  const Cd Z = cd_div(lp, lm);
  Cd p = {FADDEEVA_A[0], 0.0};
  for (int k = 1; k < FADDEEVA_N; ++k) {
    p = cd_mul(p, Z);
    p.re += FADDEEVA_A[k];
  }
  const Cd inv = cd_div({1.0, 0.0}, lm);
  const Cd inv2 = cd_mul(inv, inv);
  const double rsqpi = 0.5641895835477563;  // 1 / sqrt(pi)
  const Cd t1 = cd_mul(p, inv2);
  return {2.0 * t1.re + rsqpi * inv.re, 2.0 * t1.im + rsqpi * inv.im};
}

// E(a; t) and dE/da for a = (ar, ai), resolution width sigma > 0.
MXA_HD inline void conv_exp(double ar, double ai, double t, double sigma, Cd* e, Cd* de) {
  const double s2 = sigma * sigma;
  const double k = 0.7071067811865476 / sigma;  // 1 / (sqrt 2 sigma)
  const Cd u = {(ar * s2 - t) * k, ai * s2 * k};
  const double g = mix_exp(fmax(-0.5 * t * t / s2, -746.0));
  Cd E;
  if (u.re >= 0.0) {
    const Cd w = faddeeva_upper({-u.im, u.re});  // i u
    E = {0.5 * g * w.re, 0.5 * g * w.im};
  } else {
    const Cd w = faddeeva_upper({u.im, -u.re});  // -i u
    // exp(a^2 sigma^2 / 2 - a t)
    const double qr = 0.5 * (ar * ar - ai * ai) * s2 - ar * t;
    const double qi = ar * ai * s2 - ai * t;
    double sn, cs;
    mix_sincos(qi, &sn, &cs);
    const double eq = mix_exp(fmax(qr, -746.0));
    E = {eq * cs - 0.5 * g * w.re, eq * sn - 0.5 * g * w.im};
  }
  *e = E;
  const Cd f = {ar * s2 - t, ai * s2};
  const Cd fe = cd_mul(f, E);
  const double c = 0.3989422804014327 * sigma * g;  // sigma / sqrt(2 pi) exp(-t^2/(2 sigma^2))
  *de = {fe.re - c, fe.im};
}

}  // namespace mxa
