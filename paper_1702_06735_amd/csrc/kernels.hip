// HIP kernels for gfx950 (MI355X): tier-0 precompute, the likelihood passes
// over data and MC events with their adjoint, the deterministic reduction and
// finalisation, and a per-event diagnostics kernel.
//
// Method: Hasse et al., arXiv:1702.06735 -- Eq. (1) (time-dependent rate),
// Eq. (2) (coherent sums over decay chains), Sec. 3 (chains built from spin
// factors, form factors, lineshapes, Bose symmetrisation) and Sec. 3.1 (Monte
// Carlo normalisation over uniform phase space).
#include <math.h>

#include <type_traits>

#include "finalize.h"
#include "internal.h"
#include "mixfns.h"
#include "resolution.h"

namespace mxa {
namespace {

// ===========================================================================
// Tier-0 precompute (once per sample, FP64).
// ===========================================================================
struct F4 {
  double e, x, y, z;
};
__device__ inline F4 add(F4 a, F4 b) { return {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline F4 sub(F4 a, F4 b) { return {a.e - b.e, a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline F4 smul(double c, F4 a) { return {c * a.e, c * a.x, c * a.y, c * a.z}; }
__device__ inline double mdot(F4 a, F4 b) { return a.e * b.e - a.x * b.x - a.y * b.y - a.z * b.z; }

// Break-up momentum squared from invariants, lambda(M2, a2, b2) / (4 M2),
// clamped at zero.
__device__ inline double q2_inv(double M2, double a2, double b2) {
  const double d = M2 - a2 - b2;
  const double v = (d * d - 4.0 * a2 * b2) / (4.0 * M2);
  return v > 0.0 ? v : 0.0;
}

// Orbital tensors of a vertex P -> u v: rank 1 is u - v made orthogonal to P;
// rank 2 (contracted with a, b) is its traceless symmetric square in the P
// rest frame. p2 = P.P.
__device__ inline F4 orb1(F4 P, F4 u, F4 v) {
  const F4 w = sub(u, v);
  return sub(w, smul(mdot(w, P) / mdot(P, P), P));
}
__device__ inline double proj(F4 P, F4 a, F4 b, double p2) {
  return mdot(a, b) - mdot(a, P) * mdot(b, P) / p2;
}
__device__ inline double orb2(F4 P, F4 l, F4 a, F4 b, double p2) {
  return mdot(a, l) * mdot(b, l) - mdot(l, l) * proj(P, a, b, p2) / 3.0;
}
// eps_{mu nu rho sigma} a^mu b^nu c^rho d^sigma with eps_{0123} = +1, by
// Laplace expansion over the 2x2 minors of rows (a, b) and (c, d).
__device__ inline double levi(F4 a, F4 b, F4 c, F4 d) {
  const double s0 = a.e * b.x - a.x * b.e, s1 = a.e * b.y - a.y * b.e, s2 = a.e * b.z - a.z * b.e;
  const double s3 = a.x * b.y - a.y * b.x, s4 = a.x * b.z - a.z * b.x, s5 = a.y * b.z - a.z * b.y;
  const double c5 = c.y * d.z - c.z * d.y, c4 = c.x * d.z - c.z * d.x, c3 = c.x * d.y - c.y * d.x;
  const double c2 = c.e * d.z - c.z * d.e, c1 = c.e * d.y - c.y * d.e, c0 = c.e * d.x - c.x * d.e;
  return s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
}
// Blatt-Weisskopf factors without q^L, z = (r q)^2.
__device__ inline double bw1(double z) { return 1.0 / sqrt(1.0 + z); }
__device__ inline double bw2(double z) { return 1.0 / sqrt(9.0 + z * (3.0 + z)); }

// The 12 columns of one Bose configuration. pi_s is the pi- paired with the
// K+ (and the a1 bachelor), pi_o the one paired with the pi+.
__device__ void tier0_sigma(const Tier0Const& k, F4 kp, F4 ps, F4 pip, F4 po, F4 pD, double pD2,
                            F4 pa1, double s3, F4 lDa, double fDa, double* out) {
  const double mK2 = k.m_K * k.m_K, mpi2 = k.m_pi * k.m_pi, r2 = k.r * k.r, mD2 = k.m_D * k.m_D;
  const F4 P1 = add(kp, ps), P2 = add(pip, po), PK = add(P1, pip);
  const double s1 = mdot(P1, P1), s2 = mdot(P2, P2), sk = mdot(PK, PK);
  // two-body resonance vertices K*0 -> K+ pi_s and rho0 -> pi+ pi_o
  const double qk2 = q2_inv(s1, mK2, mpi2), qr2 = q2_inv(s2, mpi2, mpi2);
  const double fk = bw1(r2 * qk2), fr = bw1(r2 * qr2);
  const double gk = qk2 * sqrt(qk2) * fk * fk / sqrt(s1);
  const double gr = qr2 * sqrt(qr2) * fr * fr / sqrt(s2);
  // D -> V1 V2 and D -> S V2
  const F4 t1 = orb1(P1, kp, ps), t2 = orb1(P2, pip, po), lD = orb1(pD, P1, P2);
  const double zD = r2 * q2_inv(mD2, s1, s2);
  const double f1D = bw1(zD), f2D = bw2(zD), fkr = fk * fr;
  out[C_SKPI] = s1;
  out[C_GKS] = gk;
  out[C_SPIPI] = s2;
  out[C_GRHO] = gr;
  out[C_SKPIPI] = sk;
  out[C_SF1] = mdot(t1, t2) * fkr;
  out[C_SF2] = levi(lD, pD, t1, t2) * f1D * fkr;
  out[C_SF3] = orb2(pD, lD, t1, t2, pD2) * f2D * fkr;
  out[C_SF4] = mdot(lD, t2) * f1D * fr;
  // D -> a1- K+, a1- -> rho0 pi_s (S and D wave)
  const F4 lA = orb1(pa1, P2, ps);
  const double za = r2 * q2_inv(s3, s2, mpi2);
  out[C_SF5] = proj(pa1, lDa, t2, s3) * fDa * fr;
  out[C_SF6] = orb2(pa1, lA, lDa, t2, s3) * fDa * fr * bw2(za);
  // D -> K1+ pi_o, K1+ -> K*0 pi+
  const F4 lDk = orb1(pD, PK, po);
  const double fDk = bw1(r2 * q2_inv(mD2, sk, mpi2));
  out[C_SF7] = proj(PK, lDk, t1, sk) * fDk * fk;
}

// The 25 tier-0 values of one event p[4] = (K+, pi-(a), pi+, pi-(b)).
__device__ inline void tier0_event(const Tier0Const& k, const F4 p[4], double o[NCOL]) {
  // pi- pair formed first so that nothing shared depends on which pi- is "a"
  const F4 pim = add(p[1], p[3]);
  const F4 pD = add(add(p[0], p[2]), pim);
  const F4 pa1 = add(p[2], pim);
  const double pD2 = mdot(pD, pD), s3 = mdot(pa1, pa1);
  const F4 lDa = orb1(pD, pa1, p[0]);
  const double fDa = bw1(k.r * k.r * q2_inv(k.m_D * k.m_D, s3, k.m_K * k.m_K));
  tier0_sigma(k, p[0], p[1], p[2], p[3], pD, pD2, pa1, s3, lDa, fDa, o);
  tier0_sigma(k, p[0], p[3], p[2], p[1], pD, pD2, pa1, s3, lDa, fDa, o + CPS);
  o[C_S3PI] = s3;
}

__global__ __launch_bounds__(BLOCK) void tier0_kernel(Tier0Const k, const double* __restrict__ p4,
                                                      const double* __restrict__ t, int64_t n,
                                                      int64_t ld, double* __restrict__ c64,
                                                      float* __restrict__ c32,
                                                      double* __restrict__ t64,
                                                      unsigned* __restrict__ n_bad) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  double v[16];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    v[j] = p4[16 * i + j];
    ok = ok && isfinite(v[j]);
  }
  F4 p[4];
  const double sg = k.parity ? -1.0 : 1.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) p[j] = {v[4 * j], sg * v[4 * j + 1], sg * v[4 * j + 2], sg * v[4 * j + 3]};
  // validation: four-momentum conservation and mass shells
  const F4 pD = add(add(p[0], p[2]), add(p[1], p[3]));
  ok = ok && fabs(pD.e - k.m_D) <= k.tol_p && fabs(pD.x) <= k.tol_p && fabs(pD.y) <= k.tol_p &&
       fabs(pD.z) <= k.tol_p;
  const double m2[4] = {k.m_K * k.m_K, k.m_pi * k.m_pi, k.m_pi * k.m_pi, k.m_pi * k.m_pi};
#pragma unroll
  for (int j = 0; j < 4; ++j) ok = ok && fabs(mdot(p[j], p[j]) - m2[j]) <= k.tol_m2;
  if (t) {
    const double tt = t[i];
    ok = ok && isfinite(tt) && (tt >= 0.0 || k.allow_neg_t);
    t64[i] = tt;
  }
  if (!ok) atomicAdd(n_bad, 1u);
  double o[NCOL];
  tier0_event(k, p, o);
  // either copy may be omitted (NULL)
  if (c64) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) c64[c * ld + i] = o[c];
  }
  if (c32) {
#pragma unroll
    for (int c = 0; c < NCOL; ++c) c32[c * ld + i] = static_cast<float>(o[c]);
  }
}

// ===========================================================================
// Amplitudes (Sec. 3, Eq. (2)) in the amplitude precision R.
// ===========================================================================
template <class R> struct Cp {
  R re, im;
};
// Explicit fused multiply-adds. A sum of two products a b + c d can be
// contracted either way (a b fused, or c d); left to the compiler, the choice
// can differ between two copies of the same code, and the two Bose
// configurations would then round differently. Written out, both
// configurations compute the same operations, so exchanging the two pi- gives
// bit-identical sums.
template <class R> __device__ inline R fmr(R a, R b, R c);
template <> __device__ inline float fmr<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ inline double fmr<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class R> __device__ inline Cp<R> cmul(Cp<R> a, Cp<R> b) {
  return {fmr<R>(a.re, b.re, -(a.im * b.im)), fmr<R>(a.re, b.im, a.im * b.re)};
}
template <class R> __device__ inline Cp<R> cscale(Cp<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R> __device__ inline Cp<R> cadd(Cp<R> a, Cp<R> b) { return {a.re + b.re, a.im + b.im}; }

template <class R> __device__ inline R rcp(R x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// 1/x from the hardware estimate refined by two Newton steps, each
// r <- r + r (1 - x r): within about an ulp of the correctly rounded quotient
// for the positive, normal squared moduli it is applied to, at half the
// instructions of an IEEE division
template <> __device__ inline double rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
template <class R> __device__ inline R root(R x);
template <> __device__ inline float root<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ inline double root<double>(double x) { return sqrt(x); }

// acc += (cr + i ci) b as four fused multiply-adds
template <class R> __device__ inline void cfma(Cp<R>& acc, R cr, R ci, const Cp<R>& b) {
  acc.re = fmr<R>(cr, b.re, acc.re);
  acc.re = fmr<R>(-ci, b.im, acc.re);
  acc.im = fmr<R>(cr, b.im, acc.im);
  acc.im = fmr<R>(ci, b.re, acc.im);
}
// acc = a b for the first term of a sum (first = true), else acc += a b
template <class R> __device__ inline void cacc(Cp<R>& acc, bool& first, R cr, R ci, const Cp<R>& b) {
  if (first) {
    acc = cmul(Cp<R>{cr, ci}, b);
    first = false;
  } else {
    cfma(acc, cr, ci, b);
  }
}

// 1 / (re - i im)
template <class R> __device__ inline Cp<R> inv_den(R re, R im) {
  const R n = rcp<R>(fmr<R>(re, re, im * im));
  return {re * n, im * n};
}

// Value barrier: the compiler may not fuse the producing multiply into the
// consuming add. Keeps b(sigma=a) + b(sigma=b) a plain, commutative sum, so
// exchanging the two pi- gives bit-identical results.
__device__ inline float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ inline double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <class R> __device__ inline const LsConst<R>& ls_of(const EvalParams& p);
template <> __device__ inline const LsConst<double>& ls_of<double>(const EvalParams& p) { return p.ld; }
template <> __device__ inline const LsConst<float>& ls_of<float>(const EvalParams& p) { return p.lf; }

// Two-body lineshape with running width from s alone (RW passes):
// l = 1/D, D = (m0^2 - s) - i K g(s), g = N / Dg with N = P sqrt(P),
// P = s (s - t_sum) + t_prod and Dg = s (8 s + 2 r^2 P); multiplying
// through by Dg leaves one reciprocal inv = 1 / (re^2 + im^2):
//   l = Dg inv (re + i im),  re = (m0^2 - s) Dg,  im = K N,
// and g l = u (re + i im) with u = N inv for the lineshape adjoint.
template <class R>
__device__ inline void running_ls(R m2, R K, R tsum, R tprod, R r2x2, R s, Cp<R>& l, Cp<R>& r,
                                  R& u) {
  R P = fmr<R>(s, s - tsum, tprod);
  P = P > R(0) ? P : R(0);
  const R N = P * root<R>(P);
  const R Dg = s * fmr<R>(r2x2, P, R(8) * s);
  const R re = (m2 - s) * Dg, im = K * N;
  const R inv = rcp<R>(fmr<R>(re, re, im * im));
  const R w = Dg * inv;
  l = {re * w, im * w};
  r = {re, im};
  u = N * inv;
}

// Per-event values loaded from the tier-0 cache.
template <class R> struct EventIn {
  R v[2][CPS];
  R s3;
};

// Column c of the cache starts at the wave-uniform address cache + c * ld.
// The column bases are pinned in scalar registers (the empty asm also stops
// the compiler from re-deriving them from one per-lane pointer) and the lane
// offset is a 32-bit byte count, so each load is the "scalar base + 32-bit
// vector offset" form: one offset register for all columns instead of a
// 64-bit address pair per column. Requires i * sizeof(R) < 2^32.
template <class R> using gptr = const __attribute__((address_space(1))) R*;
template <class R> struct Cols {
  gptr<char> p[NCOL];
};
template <class R>
__device__ inline Cols<R> columns(const R* __restrict__ c, int64_t ld) {
  Cols<R> k;
#pragma unroll
  for (int j = 0; j < NCOL; ++j) {
    gptr<char> q = (gptr<char>)(c + static_cast<int64_t>(j) * ld);
    asm volatile("" : "+s"(q));
    k.p[j] = q;
  }
  return k;
}
template <class R> __device__ inline R ld_col(gptr<char> base, uint32_t off) {
  return *reinterpret_cast<gptr<R>>(base + off);
}

// RW: the running-width columns are not read (the pass forms g from s).
template <class R, int U, bool RW = false>
__device__ inline void load_event(const Cols<R>& c, uint32_t i, EventIn<R>& e) {
  constexpr bool ks = U & KS_SET, rho = U & RHO_SET;
  const uint32_t off = i * static_cast<uint32_t>(sizeof(R));
#pragma unroll
  for (int sg = 0; sg < 2; ++sg) {
    const int o = CPS * sg;
    if (ks) {
      e.v[sg][C_SKPI] = ld_col<R>(c.p[o + C_SKPI], off);
      if (!RW) e.v[sg][C_GKS] = ld_col<R>(c.p[o + C_GKS], off);
    }
    if (rho) {
      e.v[sg][C_SPIPI] = ld_col<R>(c.p[o + C_SPIPI], off);
      if (!RW) e.v[sg][C_GRHO] = ld_col<R>(c.p[o + C_GRHO], off);
    }
    if (U & K1_SET) e.v[sg][C_SKPIPI] = ld_col<R>(c.p[o + C_SKPIPI], off);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (U & (1 << k)) e.v[sg][C_SF1 + k] = ld_col<R>(c.p[o + C_SF1 + k], off);
    if (U & K1_SET) e.v[sg][C_SF7] = ld_col<R>(c.p[o + C_SF7], off);
  }
  if (U & A1_SET) e.s3 = ld_col<R>(c.p[C_S3PI], off);
}

// Reduced chain amplitudes beta_k of one Bose configuration and the reduced
// lineshapes they are built from.
template <class R> struct Sigma {
  Cp<R> b[8];
  Cp<R> lks, lrho;
  Cp<R> kr;           // l_K* l_rho, the lineshape product of chains 1-3
  Cp<R> rks, rrho;    // RW passes: g l = u r for K*0 and rho0
  R uks, urho;
};

template <class R, int U, bool RW = false>
__device__ inline void chains(const LsConst<R>& L, const R* v, Cp<R> la1, Sigma<R>& o) {
  if constexpr (RW) {
    if (U & KS_SET)
      running_ls<R>(L.ks_m2, L.ks_k, L.ks_tsum, L.ks_tprod, L.r2x2, v[C_SKPI], o.lks, o.rks, o.uks);
    if (U & RHO_SET)
      running_ls<R>(L.rho_m2, L.rho_k, L.rho_tsum, L.rho_tprod, L.r2x2, v[C_SPIPI], o.lrho, o.rrho,
                    o.urho);
  } else {
    if (U & KS_SET) o.lks = inv_den<R>(L.ks_m2 - v[C_SKPI], L.ks_k * v[C_GKS]);
    if (U & RHO_SET) o.lrho = inv_den<R>(L.rho_m2 - v[C_SPIPI], L.rho_k * v[C_GRHO]);
  }
  if (U & 0x07) {
    o.kr = cmul(o.lks, o.lrho);
    if (U & 0x01) o.b[0] = cscale(o.kr, v[C_SF1]);
    if (U & 0x02) o.b[1] = cscale(o.kr, v[C_SF2]);
    if (U & 0x04) o.b[2] = cscale(o.kr, v[C_SF3]);
  }
  if (U & 0x08) o.b[3] = cscale(o.lrho, v[C_SF4]);
  if (U & A1_SET) {
    const Cp<R> ar = cmul(la1, o.lrho);
    if (U & 0x10) o.b[4] = cscale(ar, v[C_SF5]);
    if (U & 0x20) o.b[5] = cscale(ar, v[C_SF6]);
  }
  if (U & K1_SET) {
    const Cp<R> k7 = cscale(o.lks, v[C_SF7]);
    if (U & 0x40) o.b[6] = cmul(k7, inv_den<R>(L.k1a_m2 - v[C_SKPIPI], L.k1a_mg));
    if (U & 0x80) o.b[7] = cmul(k7, inv_den<R>(L.k1b_m2 - v[C_SKPIPI], L.k1b_mg));
  }
  // every b_k is a finished, rounded value from here on (see opaque)
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (U & (1 << k)) {
      o.b[k].re = opaque(o.b[k].re);
      o.b[k].im = opaque(o.b[k].im);
    }
}

template <class R> struct Amps {
  Sigma<R> sg[2];
  Cp<R> la1;
  Cp<R> B[8];  // Bose-symmetrised reduced chain amplitudes
  Cp<R> A, Ab;
};

template <class R, int MA, int MB, bool RW = false>
__device__ inline void amplitudes(const LsConst<R>& L, const EventIn<R>& e, Amps<R>& a) {
  constexpr int U = MA | MB;
  if (U & A1_SET) a.la1 = inv_den<R>(L.a1_m2 - e.s3, L.a1_mg);
  chains<R, U, RW>(L, e.v[0], a.la1, a.sg[0]);
  chains<R, U, RW>(L, e.v[1], a.la1, a.sg[1]);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (U & (1 << k)) {
      a.B[k].re = a.sg[0].b[k].re + a.sg[1].b[k].re;
      a.B[k].im = a.sg[0].b[k].im + a.sg[1].b[k].im;
    }
  // Eq. (2) as chains of fused multiply-adds
  a.A = {R(0), R(0)};
  a.Ab = {R(0), R(0)};
  bool fa = true, fb = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (MA & (1 << k)) cacc(a.A, fa, L.ca[k][0], L.ca[k][1], a.B[k]);
    if (MB & (1 << k)) cacc(a.Ab, fb, L.cb[k][0], L.cb[k][1], a.B[k]);
  }
}

// Moments of Eq. (1) in FP64.
struct Mom {
  double ar, ai, br, bi;
  double a2, b2, xr, xi;  // |A|^2, |Ab|^2, Re(A Ab*), Im(A Ab*)
};
template <class R> __device__ inline Mom moments(const Cp<R>& A, const Cp<R>& Ab) {
  Mom m;
  m.ar = A.re; m.ai = A.im; m.br = Ab.re; m.bi = Ab.im;
  m.a2 = m.ar * m.ar + m.ai * m.ai;
  m.b2 = m.br * m.br + m.bi * m.bi;
  m.xr = m.ar * m.br + m.ai * m.bi;
  m.xi = m.ai * m.br - m.ar * m.bi;
  return m;
}

struct TimeFns {
  double ch, sh, cs, sn;
};
__device__ inline TimeFns time_fns(const MixConst& x, double t) {
  TimeFns f;
  mix_cosh_sinh(x.yg * t, &f.ch, &f.sh);
  mix_sincos(x.xg * t, &f.sn, &f.cs);
  return f;
}
// Eq. (1) divided by exp(-Gamma t) N_f
__device__ inline double rate_eq1(const Mom& m, const TimeFns& f) {
  return (m.a2 + m.b2) * f.ch + (m.a2 - m.b2) * f.cs - 2.0 * m.xr * f.sh - 2.0 * m.xi * f.sn;
}
// its integral over t in [0, inf) with exp(-Gamma t)
__device__ inline double rate_int(const Mom& m, const MixConst& x) {
  return x.h_sum * (m.a2 + m.b2) + x.h_diff * (m.a2 - m.b2) - x.h_re * m.xr - x.h_im * m.xi;
}
// With a Gaussian decay-time resolution: e^{-Gamma t} times the four time
// functions, each convolved with the resolution (cosh, sinh from the
// exponentials of Gamma (1 -+ y), cos, sin from that of Gamma (1 - i x)), at
// the measured time t, and their x and y derivatives. rate_eq1 with these is
// the resolved density R(t) (its integral over t is unchanged).
struct ResFns {
  TimeFns f;
  double dcs_dx, dsn_dx, dch_dy, dsh_dy;
};
__device__ inline ResFns res_fns(const MixConst& x, double t) {
  const double G = x.gamma;
  Cd e1, d1, e2, d2, e3, d3;
  conv_exp(G - x.yg, 0.0, t, x.sigma_t, &e1, &d1);
  conv_exp(G + x.yg, 0.0, t, x.sigma_t, &e2, &d2);
  conv_exp(G, -x.xg, t, x.sigma_t, &e3, &d3);
  ResFns r;
  r.f.ch = 0.5 * (e1.re + e2.re);
  r.f.sh = 0.5 * (e1.re - e2.re);
  r.f.cs = e3.re;
  r.f.sn = e3.im;
  // d a3 / dx = -i Gamma; d a1 / dy = -Gamma, d a2 / dy = +Gamma
  r.dcs_dx = G * d3.im;
  r.dsn_dx = -G * d3.re;
  r.dch_dy = 0.5 * G * (d2.re - d1.re);
  r.dsh_dy = -0.5 * G * (d1.re + d2.re);
  return r;
}

// ===========================================================================
// Reductions: per-thread FP64 sums -> wave reduce-scatter -> workgroup
// (TwoSum-compensated across waves) -> one row per workgroup -> per-slot
// totals over the rows (slot_reduce_kernel), each level in a fixed order, so
// results are bitwise reproducible.
// ===========================================================================
struct Pair {
  double s, e;
};
__device__ inline Pair two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline Pair padd(Pair x, Pair y) {
  Pair r = two_sum(x.s, y.s);
  r.e += x.e + y.e;
  return r;
}

// One reduce-scatter step at lane distance D on M live slots: lanes with bit
// D set keep the upper half, the others the lower half, adding the partner's
// copy of that half. With M = 1 it is a plain butterfly step.
template <int M, int D, int P>
__device__ inline void rs_steps(double (&v)[P], int lane) {
  if constexpr (D >= 1) {
    if constexpr (M > 1) {
      constexpr int H = M / 2;
      const bool up = (lane & D) != 0;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const double keep = up ? v[H + j] : v[j];
        const double send = up ? v[j] : v[H + j];
        v[j] = keep + __shfl_xor(send, D, 64);
      }
      rs_steps<H, D / 2, P>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], D, 64);
      rs_steps<1, D / 2, P>(v, lane);
    }
  }
}

// Reduce the block's per-thread accumulators acc[0..NS) into (sum, error)
// pairs; thread t < NS returns slot t in *out (valid in wave 0 only).
template <int NS, int P>
__device__ inline Pair block_reduce(double (&acc)[P], double* lds /* [4][P] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  rs_steps<P, 32, P>(acc, lane);
  constexpr int SHIFT = 6 - (P == 1 ? 0 : (P == 2 ? 1 : (P == 4 ? 2 : (P == 8 ? 3 : (P == 16 ? 4 : (P == 32 ? 5 : 6))))));
  if ((lane & ((1 << SHIFT) - 1)) == 0) lds[wave * P + (lane >> SHIFT)] = acc[0];
  __syncthreads();
  Pair r = {0.0, 0.0};
  if (threadIdx.x < NS) {
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) r = padd(r, Pair{lds[w * P + threadIdx.x], 0.0});
  }
  return r;
}

// ===========================================================================
// Likelihood passes. Each workgroup takes a contiguous range of data (or MC)
// events and sums into the accumulator slots of Slots (finalize.h).
// Slots 0..4 are per-thread FP64 registers. The adjoint slots (5..) are
// per-thread partial sums over the thread's events (a few tens), combined in
// FP64 across threads and workgroups like every other slot:
//  * FP32 amplitudes: FP32 registers (34 VGPRs for the fourteen-chain model).
//    No LDS is then needed, and the pass runs 14% faster than with the FP64
//    LDS words below (fourteen-chain MC pass over 4M events, 76 against
//    88 us). The FP32 LDS atomic add is no alternative: it measured an order
//    of magnitude slower than the FP64 one on this chip.
//  * FP64: private FP64 words in LDS, added to with FP64 LDS atomics (in
//    registers they would take ~70 VGPRs for the whole event loop).
// A thread's slots are touched only by that thread, in program order, so the
// sums are deterministic.
// ===========================================================================
// add v to adjoint slot s (>= 5) of this thread: FP32 register slots ...
template <class R, int N> __device__ inline void gadd(float (&gr)[N], int s, R v) {
  gr[s - 5] += static_cast<float>(v);
}
// ... or FP64 LDS words (stride BLOCK)
template <class R> __device__ inline void gadd(double* __restrict__ gl, int s, R v) {
  __hip_atomic_fetch_add(gl + (s - 5) * BLOCK, static_cast<double>(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
}
// add a1 b1 + a2 b2: two fused multiply-adds into an FP32 register slot, one
// LDS add of the value for an FP64 slot
template <class R, int N> __device__ inline void gadd2(float (&gr)[N], int s, R a1, R b1, R a2, R b2) {
  gr[s - 5] = __builtin_fmaf(a2, b2, __builtin_fmaf(a1, b1, gr[s - 5]));
}
template <class R> __device__ inline void gadd2(double* __restrict__ gl, int s, R a1, R b1, R a2, R b2) {
  gadd<R>(gl, s, a1 * b1 + a2 * b2);
}
// ... or FP64 registers (the basis pass, whose coefficient adjoints fit in
// registers beside its light per-event work): the same value added in the
// same order as to an FP64 LDS word
template <int N> struct Reg64 {
  double v[N];
};
template <class R, int N> __device__ inline void gadd(Reg64<N>& gr, int s, R v) {
  gr.v[s - 5] += static_cast<double>(v);
}
template <class R, int N> __device__ inline void gadd2(Reg64<N>& gr, int s, R a1, R b1, R a2, R b2) {
  gadd<R>(gr, s, a1 * b1 + a2 * b2);
}

// BKG: data with a background component (an extension of the paper's model):
// the event's density is p = (1 - f) B e^{-Gamma t} / Nhat + f Gamma_b
// e^{-Gamma_b t} (inv_nhat = 1 / Nhat from the MC pass), its term -ln p, and
// the adjoint weight w = (1 - f) e^{-Gamma t} / (Nhat p) takes the place of
// 1 / B.
// RES: data with a Gaussian decay-time resolution: the resolved density R(t)
// takes the place of B, the event's term is -ln R (no Gamma t: R holds the
// exponential), and the x, y derivatives come from the convolved functions.
// Both: p = (1 - f) R(t) / Nhat + f Gamma_b E(Gamma_b; t), E the background's
// exponential convolved with the resolution.
// SHAPES: also the lineshape adjoints (slots 5..10); without, e is not read.
template <class R, int MA, int MB, bool GRAD, bool DATA, int P, class G, bool BKG = false,
          bool RES = false, bool RW = false, bool SHAPES = true>
__device__ inline void accumulate(const EvalParams& p, const Amps<R>& a, const EventIn<R>& e,
                                  double t, double (&acc)[P], G&& gl, double inv_nhat = 0.0) {
  const Mom m = moments(a.A, a.Ab);
  // adjoint weights G_A, G_Ab: FP64 on data events (from Eq. (1)), R on MC
  using GT = std::conditional_t<DATA, double, R>;
  Cp<GT> GA, GB;
  if constexpr (DATA) {
    ResFns rf;
    if constexpr (RES) rf = res_fns(p.mix, t);
    const TimeFns f = RES ? rf.f : time_fns(p.mix, t);
    const double B = rate_eq1(m, f);
    const bool ok = B > 0.0 && B < INFINITY;
    double l, wb = 0.0;
    if constexpr (BKG) {
      // the signal's e^{-Gamma t} / Nhat and the background's density at t;
      // with a resolution B already holds the resolved exponential, and the
      // background's exponential is convolved too
      double es, eb;
      if constexpr (RES) {
        Cd E, dE;
        conv_exp(p.mix.g_bkg, 0.0, t, p.mix.sigma_t, &E, &dE);
        es = inv_nhat;
        eb = p.mix.g_bkg * E.re;
      } else {
        es = mix_exp(-p.mix.gamma * t) * inv_nhat;
        eb = p.mix.g_bkg * mix_exp(-p.mix.g_bkg * t);
      }
      const double sg = (1.0 - p.mix.f_bkg) * B * es;
      const double dens = sg + p.mix.f_bkg * eb;
      l = ok ? -log(dens) : 0.0;
      wb = ok ? (1.0 - p.mix.f_bkg) * es / dens : 0.0;
      if constexpr (GRAD) {
        constexpr int X = Slots<GRAD, MA, MB>::NS;
        acc[X] += ok ? sg / dens : 0.0;
        acc[X + 1] += ok ? (B * es - eb) / dens : 0.0;
      }
    } else if constexpr (RES) {
      l = ok ? -log(B) : 0.0;
    } else {
      l = ok ? p.mix.gamma * t - log(B) : 0.0;
    }
    acc[0] += l;
    acc[1] += fabs(l);
    acc[2] += ok ? 0.0 : 1.0;
    if constexpr (GRAD) {
      const double w = BKG ? wb : (ok ? 1.0 / B : 0.0);
      const double cp = f.ch + f.cs, cm = f.ch - f.cs;
      GA.re = w * (cp * m.ar - (f.sh * m.br - f.sn * m.bi));
      GA.im = w * (cp * m.ai - (f.sh * m.bi + f.sn * m.br));
      GB.re = w * (cm * m.br - (f.sh * m.ar + f.sn * m.ai));
      GB.im = w * (cm * m.bi - (f.sh * m.ai - f.sn * m.ar));
      if constexpr (RES) {
        acc[3] += w * ((m.a2 - m.b2) * rf.dcs_dx - 2.0 * m.xi * rf.dsn_dx);
        acc[4] += w * ((m.a2 + m.b2) * rf.dch_dy - 2.0 * m.xr * rf.dsh_dy);
      } else {
        const double gt = p.mix.gamma * t;
        acc[3] += w * (-gt * ((m.a2 - m.b2) * f.sn + 2.0 * m.xi * f.cs));
        acc[4] += w * (gt * ((m.a2 + m.b2) * f.sh - 2.0 * m.xr * f.ch));
      }
    }
  } else {
    acc[0] += m.a2;
    acc[1] += m.b2;
    acc[2] += m.xr;
    acc[3] += m.xi;
    if constexpr (GRAD) {
      // the weights in the amplitudes' own precision: G_A = hp A - h Ab,
      // G_Ab = hm Ab - conj(h) A with h = (h_re + i h_im) / 2
      const LsConst<R>& L = ls_of<R>(p);
      const Cp<R> A = a.A, Ab = a.Ab;
      GA.re = fmr<R>(L.mc_hp, A.re, -fmr<R>(L.mc_hr, Ab.re, -(L.mc_hi * Ab.im)));
      GA.im = fmr<R>(L.mc_hp, A.im, -fmr<R>(L.mc_hr, Ab.im, L.mc_hi * Ab.re));
      GB.re = fmr<R>(L.mc_hm, Ab.re, -fmr<R>(L.mc_hr, A.re, L.mc_hi * A.im));
      GB.im = fmr<R>(L.mc_hm, Ab.im, -fmr<R>(L.mc_hr, A.im, -(L.mc_hi * A.re)));
    }
  }
  if constexpr (GRAD) {
    constexpr int U = MA | MB;
    const R gar = static_cast<R>(GA.re), gai = static_cast<R>(GA.im);
    const R gbr = static_cast<R>(GB.re), gbi = static_cast<R>(GB.im);
    // coefficient adjoints W_k
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const R br = a.B[k].re, bi = a.B[k].im;
      if (MA & (1 << k)) {
        const int sl = 11 + 2 * rank_in(MA, k);
        gadd2<R>(gl, sl, gar, br, gai, bi);
        gadd2<R>(gl, sl + 1, gar, bi, -gai, br);
      }
      if (MB & (1 << k)) {
        const int sl = 11 + 2 * popc(MA) + 2 * rank_in(MB, k);
        gadd2<R>(gl, sl, gbr, br, gbi, bi);
        gadd2<R>(gl, sl + 1, gbr, bi, -gbi, br);
      }
    }
    if constexpr (!SHAPES) return;
    // h_k = conj(G_A) c'_k + conj(G_Ab) cbar'_k, with the terms of chains
    // outside A_f or Abar_f left out (not multiplied by zero)
    const LsConst<R>& L = ls_of<R>(p);
    Cp<R> h[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (U & (1 << k)) {
        const bool ia = MA & (1 << k), ib = MB & (1 << k);
        const R car = L.ca[k][0], cai = L.ca[k][1], cbr = L.cb[k][0], cbi = L.cb[k][1];
        R hr, hi;
        if (ia) {
          hr = fmr<R>(gai, cai, gar * car);
          hi = fmr<R>(-gai, car, gar * cai);
          if (ib) {
            hr = fmr<R>(gbi, cbi, fmr<R>(gbr, cbr, hr));
            hi = fmr<R>(-gbi, cbr, fmr<R>(gbr, cbi, hi));
          }
        } else {
          hr = fmr<R>(gbi, cbi, gbr * cbr);
          hi = fmr<R>(-gbi, cbr, gbr * cbi);
        }
        h[k] = {hr, hi};
      }
    // lineshape adjoints: Q_R = l_R sum_{k in R} h_k beta_k per configuration.
    // The sums share their terms: chains 1-3 carry both the K*0 and the rho0
    // lineshape, 7-8 the K*0 only, 4 the rho0 only, 5-6 the rho0 and the a1.
    // The two configurations are combined by one commutative add so that
    // exchanging the pi- leaves every sum bit-identical.
    Cp<R> hks[2], hrho[2], ha1[2];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const Sigma<R>& S = a.sg[sg];
      Cp<R> vv = {R(0), R(0)}, ka = {R(0), R(0)}, a1 = {R(0), R(0)};
      bool fv = true, fa = true;
      if (U & 0x07) {
        // chains 1-3 share l_K* l_rho: sum h_k beta_k = kr sum_k sf_k h_k
        Cp<R> t = {R(0), R(0)};
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (U & (1 << k)) {
            const R f = e.v[sg][C_SF1 + k];
            if (fv) {
              t = {h[k].re * f, h[k].im * f};
              fv = false;
            } else {
              t = {fmr<R>(h[k].re, f, t.re), fmr<R>(h[k].im, f, t.im)};
            }
          }
        vv = cmul(S.kr, t);
      }
#pragma unroll
      for (int k = 4; k < 6; ++k)
        if (U & (1 << k)) cacc(a1, fa, h[k].re, h[k].im, S.b[k]);
      ka = vv;
      bool fk = fv;
#pragma unroll
      for (int k = 6; k < 8; ++k)
        if (U & (1 << k)) cacc(ka, fk, h[k].re, h[k].im, S.b[k]);
      Cp<R> rh = vv;
      bool fr = fv;
      if (U & 0x08) cacc(rh, fr, h[3].re, h[3].im, S.b[3]);
      if (!fa) {
        if (fr) rh = a1; else rh = cadd(rh, a1);
        fr = false;
      }
      hks[sg] = fk ? Cp<R>{R(0), R(0)} : ka;
      hrho[sg] = fr ? Cp<R>{R(0), R(0)} : rh;
      ha1[sg] = fa ? Cp<R>{R(0), R(0)} : a1;
    }
    // one IEEE add of two values behind barriers is commutative, so the
    // sum is the same whichever pi- is "a"
    auto sym = [](R x0, R x1) { return opaque(x0) + opaque(x1); };
    // the width slots take g Im(l h): in RW passes u Im(r h) with g l = u r
    // from the lineshape
    auto gim = [](const Cp<R>& r, R u, const Cp<R>& hh) {
      return u * fmr<R>(r.re, hh.im, r.im * hh.re);
    };
    if (U & KS_SET) {
      if constexpr (RW) {
        const Sigma<R>& S0 = a.sg[0];
        const Sigma<R>& S1 = a.sg[1];
        gadd<R>(gl, 5, sym(cmul(S0.lks, hks[0]).re, cmul(S1.lks, hks[1]).re));
        gadd<R>(gl, 6, sym(gim(S0.rks, S0.uks, hks[0]), gim(S1.rks, S1.uks, hks[1])));
      } else {
        const Cp<R> q0 = cmul(a.sg[0].lks, hks[0]), q1 = cmul(a.sg[1].lks, hks[1]);
        gadd<R>(gl, 5, sym(q0.re, q1.re));
        gadd<R>(gl, 6, sym(e.v[0][C_GKS] * q0.im, e.v[1][C_GKS] * q1.im));
      }
    }
    if (U & RHO_SET) {
      if constexpr (RW) {
        const Sigma<R>& S0 = a.sg[0];
        const Sigma<R>& S1 = a.sg[1];
        gadd<R>(gl, 7, sym(cmul(S0.lrho, hrho[0]).re, cmul(S1.lrho, hrho[1]).re));
        gadd<R>(gl, 8, sym(gim(S0.rrho, S0.urho, hrho[0]), gim(S1.rrho, S1.urho, hrho[1])));
      } else {
        const Cp<R> q0 = cmul(a.sg[0].lrho, hrho[0]), q1 = cmul(a.sg[1].lrho, hrho[1]);
        gadd<R>(gl, 7, sym(q0.re, q1.re));
        gadd<R>(gl, 8, sym(e.v[0][C_GRHO] * q0.im, e.v[1][C_GRHO] * q1.im));
      }
    }
    if (U & A1_SET) {
      const Cp<R> hsum = {sym(ha1[0].re, ha1[1].re), sym(ha1[0].im, ha1[1].im)};
      const Cp<R> q = cmul(a.la1, hsum);
      gadd<R>(gl, 9, q.re);
      gadd<R>(gl, 10, q.im);
    }
  }
}

// Event loop of one workgroup. With PREFETCH the next event's cache values
// are loaded before the current event is computed (software pipelining), so
// the load latency hides behind arithmetic even at low occupancy.
template <class R, int MA, int MB, bool GRAD, bool DATA, bool PREFETCH, int P, class G,
          bool BKG = false, bool RES = false, bool RW = false>
__device__ inline void run_events(const EvalParams& p, const R* __restrict__ cache,
                                  const double* __restrict__ tt, int64_t ld, int64_t lo,
                                  int64_t hi, double (&acc)[P], G&& gl, double inv_nhat = 0.0) {
  constexpr int U = MA | MB;
  const LsConst<R>& L = ls_of<R>(p);
  const Cols<R> cols = columns<R>(cache, ld);
  const uint32_t end = static_cast<uint32_t>(hi);
  uint32_t i = static_cast<uint32_t>(lo) + threadIdx.x;
  if constexpr (PREFETCH) {
    // two event buffers used in turn, so that no values are copied between
    // iterations
    if (i >= end) return;
    EventIn<R> e0, e1;
    load_event<R, U, RW>(cols, i, e0);
    double t0 = DATA ? tt[i] : 0.0, t1 = 0.0;
    while (true) {
      const uint32_t n1 = i + BLOCK < end ? i + BLOCK : i;
      load_event<R, U, RW>(cols, n1, e1);
      if (DATA) t1 = tt[n1];
      {
        Amps<R> a;
        amplitudes<R, MA, MB, RW>(L, e0, a);
        accumulate<R, MA, MB, GRAD, DATA, P, G, BKG, RES, RW>(p, a, e0, t0, acc, gl, inv_nhat);
      }
      i += BLOCK;
      if (i >= end) break;
      const uint32_t n2 = i + BLOCK < end ? i + BLOCK : i;
      load_event<R, U, RW>(cols, n2, e0);
      if (DATA) t0 = tt[n2];
      {
        Amps<R> a;
        amplitudes<R, MA, MB, RW>(L, e1, a);
        accumulate<R, MA, MB, GRAD, DATA, P, G, BKG, RES, RW>(p, a, e1, t1, acc, gl, inv_nhat);
      }
      i += BLOCK;
      if (i >= end) break;
    }
  } else {
    for (; i < end; i += BLOCK) {
      EventIn<R> e;
      load_event<R, U, RW>(cols, i, e);
      const double t = DATA ? tt[i] : 0.0;
      Amps<R> a;
      amplitudes<R, MA, MB, RW>(L, e, a);
      accumulate<R, MA, MB, GRAD, DATA, P, G, BKG, RES, RW>(p, a, e, t, acc, gl, inv_nhat);
    }
  }
}

// Which passes form the running-width factors from s instead of reading
// them: 21 columns read instead of 25, for one square root per factor. Measured
// on the 50k + 4M-event evaluation (kernel medians): FP32 NLL+gradient 73.6 ->
// 67.4 us, FP32 NLL 68.2 -> 58.1 us, FP64 NLL 148.5 -> 125.7 us, FP64
// NLL+gradient 142.6 -> 133.4 us (its MC pass; eval_both_kernel held to two
// waves per SIMD, which the extra registers would otherwise halve). The FP64
// data pass of the gradient, which holds the time functions as well, keeps
// reading them.
template <class R, bool GRAD, bool DATA>
constexpr bool recompute_widths() { return sizeof(R) == 4 || !GRAD || !DATA; }

// ===========================================================================
// The basis of a fit with fixed lineshapes: with the masses and widths fixed,
// each event's Bose-symmetrised reduced chain amplitudes B_k (Eq. (2) without
// the coefficients) are fixed too, and only the coefficients and x, y change
// from one evaluation to the next. The fit server stores them once per fit
// (column 2 r holds Re B_k and column 2 r + 1 Im B_k, r = rank of chain k in
// U = MA | MB) in place of the tier-0 record, and each evaluation forms A_f,
// Abar_f as their coefficient sums: no lineshape, barrier or spin-factor
// arithmetic per evaluation, and 2 |U| values read per event instead of the
// record's 21. B_k is computed by the same code as in the passes, with the
// same width policy as the data pass (recompute_widths), and A_f, Abar_f are
// summed in the same order, so the NLL and its coefficient and x, y adjoints
// are those of the tier-0 data pass; the lineshape adjoints are not formed.
// ===========================================================================
template <class R, int MA, int MB>
__global__ __launch_bounds__(BLOCK) void basis_kernel(const R* __restrict__ cache, int64_t ld, int64_t n,
                                                      EvalParams p, R* __restrict__ basis, int64_t bld) {
  constexpr int U = MA | MB;
  constexpr bool RW = recompute_widths<R, true, true>();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (i >= n) return;
  EventIn<R> e;
  load_event<R, U, RW>(columns<R>(cache, ld), static_cast<uint32_t>(i), e);
  Amps<R> a;
  amplitudes<R, MA, MB, RW>(ls_of<R>(p), e, a);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (U & (1 << k)) {
      const int c = 2 * rank_in(U, k);
      basis[c * bld + i] = a.B[k].re;
      basis[(c + 1) * bld + i] = a.B[k].im;
    }
}

// Data event loop over a basis (the run_events of a fit with fixed
// lineshapes): the next event's values are loaded before the current one is
// computed. The column bases sit in scalar registers.
template <int NB> struct BCols {
  gptr<char> p[NB];
};
template <class R, int NB>
__device__ __attribute__((always_inline)) inline BCols<NB> basis_columns_of(const R* __restrict__ c, int64_t ld) {
  BCols<NB> k;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    // uniform: read from the first lane, so that it is held in scalar
    // registers (the builtin takes and returns a signed 32-bit int: each half
    // goes back through uint32_t, so that the low half is not sign-extended)
    const uint64_t q = reinterpret_cast<uint64_t>(c + static_cast<int64_t>(j) * ld);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(q))));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(static_cast<uint32_t>(q >> 32))));
    k.p[j] = (gptr<char>)((static_cast<uint64_t>(hi) << 32) | lo);
  }
  return k;
}
template <class R, int NB>
__device__ __attribute__((always_inline)) inline void load_basis(const BCols<NB>& c, uint32_t i, R (&b)[NB]) {
  const uint32_t off = i * static_cast<uint32_t>(sizeof(R));
#pragma unroll
  for (int j = 0; j < NB; ++j) b[j] = ld_col<R>(c.p[j], off);
}
template <class R, int MA, int MB, int P, class G, bool BKG, bool RES, int NB, class T>
__device__ __attribute__((always_inline)) inline void basis_event(const EvalParams& p, const LsConst<R>& L, const T (&b)[NB], double t,
                                   double (&acc)[P], G&& gl, double inv_nhat) {
  constexpr int U = MA | MB;
  Amps<R> a;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (U & (1 << k))
      a.B[k] = {static_cast<R>(b[2 * rank_in(U, k)]), static_cast<R>(b[2 * rank_in(U, k) + 1])};
  a.A = {R(0), R(0)};
  a.Ab = {R(0), R(0)};
  bool fa = true, fb = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (MA & (1 << k)) cacc(a.A, fa, L.ca[k][0], L.ca[k][1], a.B[k]);
    if (MB & (1 << k)) cacc(a.Ab, fb, L.cb[k][0], L.cb[k][1], a.B[k]);
  }
  const EventIn<R> e = {};  // not read without the lineshape adjoints
  accumulate<R, MA, MB, true, true, P, G, BKG, RES, false, false>(p, a, e, t, acc, gl, inv_nhat);
}
// T: the basis's storage precision; the sums of Eq. (2) and everything after
// them run in FP64 (the per-event work is light, and an FP64 evaluation of an
// FP32-stored basis is a smooth function of the parameters, which the
// minimiser's line searches need).
template <class T, int MA, int MB, int P, class G, bool BKG, bool RES>
__device__ __attribute__((always_inline)) inline void run_basis(const EvalParams& p, const T* __restrict__ basis,
                                 const double* __restrict__ tt, int64_t ld, int64_t lo, int64_t hi,
                                 double (&acc)[P], G&& gl, double inv_nhat) {
  constexpr int NB = 2 * popc(MA | MB);
  const LsConst<double>& L = ls_of<double>(p);
  const BCols<NB> cols = basis_columns_of<T, NB>(basis, ld);
  const uint32_t end = static_cast<uint32_t>(hi);
  uint32_t i = static_cast<uint32_t>(lo) + threadIdx.x;
  if (i >= end) return;
  T b0[NB], b1[NB];
  load_basis<T, NB>(cols, i, b0);
  double t0 = tt[i], t1 = 0.0;
  while (true) {
    const uint32_t n1 = i + BLOCK < end ? i + BLOCK : i;
    load_basis<T, NB>(cols, n1, b1);
    t1 = tt[n1];
    basis_event<double, MA, MB, P, G, BKG, RES, NB>(p, L, b0, t0, acc, gl, inv_nhat);
    i += BLOCK;
    if (i >= end) break;
    const uint32_t n2 = i + BLOCK < end ? i + BLOCK : i;
    load_basis<T, NB>(cols, n2, b0);
    t0 = tt[n2];
    basis_event<double, MA, MB, P, G, BKG, RES, NB>(p, L, b1, t1, acc, gl, inv_nhat);
    i += BLOCK;
    if (i >= end) break;
  }
}

// One workgroup's share of a pass: events [blk epb, (blk+1) epb) of the data
// (DATA) or MC sample, partial sums to row blk (+ nb_d for MC).
// PF: prefetch the next event in an NLL-only MC pass as well (the combined
// launch, whose data workgroups set its occupancy anyway).
template <class R, int MA, int MB, bool GRAD, bool DATA, bool BKG = false, bool RES = false,
          bool PF = false>
__device__ inline void eval_block(const EvalArgs& a, const EvalParams& p, int blk, double* lds,
                                  double* gacc) {
  using S = Slots<GRAD, MA, MB, BKG>;
  constexpr int NS = S::NS, NT = S::NT, P = S::P;
  double acc[P];
#pragma unroll
  for (int s = 0; s < P; ++s) acc[s] = 0.0;
  // with a background component the data pass needs Nhat: from the host (Gram
  // mode), or from the MC totals of this evaluation, complete (reduced by the
  // preceding launch)
  double inv_nhat = a.inv_nhat;
  if (BKG && !(inv_nhat > 0.0)) {
    const double* M = a.totals + 64;
    const MixConst& x = p.mix;
    const double sumT = x.h_sum * (M[0] + M[1]) + x.h_diff * (M[0] - M[1]) - x.h_re * M[2] - x.h_im * M[3];
    inv_nhat = static_cast<double>(a.n_m) / sumT;
  }
  const int64_t epb = DATA ? a.epb_d : a.epb_m, n = DATA ? a.n_d : a.n_m;
  const int64_t lo = static_cast<int64_t>(blk) * epb;
  const int64_t hi = lo + epb < n ? lo + epb : n;
  // prefetch in the adjoint passes, whose arithmetic per event is long enough
  // to cover the load latency of the next one (not in the FP64 data pass,
  // where the extra registers would spill)
  constexpr bool PREFETCH = (GRAD || PF) && !(DATA && sizeof(R) == 8);
  const R* cache = static_cast<const R*>(DATA ? a.cache_d : a.cache_m);
  const double* tt = DATA ? a.t_d : nullptr;
  const int64_t ld = DATA ? a.ld_d : a.ld_m;
  constexpr bool RW = recompute_widths<R, GRAD, DATA>();
  if constexpr (GRAD && sizeof(R) == 4) {
    float gr[S::NADJ];
#pragma unroll
    for (int s = 0; s < S::NADJ; ++s) gr[s] = 0.0f;
    run_events<R, MA, MB, GRAD, DATA, PREFETCH, P, float (&)[S::NADJ], BKG, RES, RW>(
        p, cache, tt, ld, lo, hi, acc, gr, inv_nhat);
#pragma unroll
    for (int s = S::NREG; s < NS; ++s) acc[s] = static_cast<double>(gr[s - S::NREG]);
  } else if constexpr (GRAD) {
    double* gl = gacc + threadIdx.x;
#pragma unroll
    for (int s = 0; s < S::NADJ; ++s) gl[s * BLOCK] = 0.0;
    run_events<R, MA, MB, GRAD, DATA, PREFETCH, P, double*&, BKG, RES, RW>(p, cache, tt, ld, lo, hi,
                                                                          acc, gl, inv_nhat);
#pragma unroll
    for (int s = S::NREG; s < NS; ++s) acc[s] = gl[(s - S::NREG) * BLOCK];
  } else {
    run_events<R, MA, MB, GRAD, DATA, PREFETCH, P, double*&, BKG, RES, RW>(p, cache, tt, ld, lo, hi,
                                                                          acc, gacc, inv_nhat);
  }
  const Pair r = block_reduce<NT, P>(acc, lds);
  if (threadIdx.x < NT) {
    // slot-major rows: the rows of one slot are contiguous for the reduction
    const int row = DATA ? blk : a.nb_d + blk;
    const int64_t o = (static_cast<int64_t>(threadIdx.x) * (a.nb_d + a.nb_m) + row) * 2;
    a.rows[o] = r.s;
    a.rows[o + 1] = r.e;
  }
}

// MC workgroups walk the ranges in reverse order on alternate evaluations
// (a.rev): the ranges read last by one evaluation, still in the 256 MB
// memory-side cache, are then read first by the next. Each range keeps its
// workgroup row, so the sums do not depend on the order.
__device__ inline int mc_range(const EvalArgs& a, int b) { return a.rev ? a.nb_m - 1 - b : b; }

template <class R, int MA, int MB, bool GRAD, bool DATA, bool BKG = false, bool RES = false>
__global__ __launch_bounds__(BLOCK) void eval_kernel(EvalArgs a, EvalParams p) {
  using S = Slots<GRAD, MA, MB, BKG>;
  __shared__ double lds[(BLOCK / 64) * S::P];
  __shared__ double gacc[S::template lds_words<R>() * BLOCK];
  eval_block<R, MA, MB, GRAD, DATA, BKG, RES>(a, p, DATA ? blockIdx.x : mc_range(a, blockIdx.x), lds,
                                              gacc);
}

// Both passes of an evaluation in one launch: workgroups 0 .. nb_m - 1 take
// the MC sample, the rest the data. The data workgroups (one event per
// thread, latency-bound) come last, where they fill the compute units the MC
// workgroups' last round leaves idle: NLL+gradient 65.4 -> 62.4 us for 50k
// data + 4M MC events in FP32 (135.7 -> 132.3 us in FP64) against data
// first. The adjoint passes run at two waves per SIMD (registers in FP32,
// LDS slots in FP64), so sharing a launch costs them none. In the NLL-only
// form the data path's registers set the occupancy (122 VGPRs in FP32, 163
// in FP64), and the MC part prefetches its next event to make up for it:
// against separate data and MC launches the step went 69.8 -> 65.6 us (FP32)
// and 135.2 -> 122.8 us (FP64), the MC part itself faster in FP64 (115 against
// 121 us without prefetch at four waves per SIMD).
template <class R, int MA, int MB, bool GRAD = true>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
void eval_both_kernel(EvalArgs a, EvalParams p) {
  using S = Slots<GRAD, MA, MB>;
  __shared__ double lds[(BLOCK / 64) * S::P];
  __shared__ double gacc[S::template lds_words<R>() * BLOCK];
  if (static_cast<int>(blockIdx.x) < a.nb_m)
    eval_block<R, MA, MB, GRAD, false, false, false, true>(a, p, mc_range(a, blockIdx.x), lds, gacc);
  else
    eval_block<R, MA, MB, GRAD, true>(a, p, blockIdx.x - a.nb_m, lds, gacc);
}

// Second kernel of an evaluation: one workgroup per (slot, pass) combines
// that slot's workgroup rows in a fixed order -- each thread a fixed strided
// subset, then a binary tree of compensated pairs -- so the totals do not
// depend on timing. The kernel boundary makes the first kernels' rows visible
// without device-scope fences (on this chip a fence writes back the L2 of an
// XCD).
__global__ __launch_bounds__(BLOCK) void slot_reduce_kernel(EvalArgs a, int kind0) {
  __shared__ Pair part[BLOCK];
  const int sl = blockIdx.x, kind = kind0 + static_cast<int>(blockIdx.y);
  const int nrows = a.nb_d + a.nb_m;
  const int r0 = kind == 0 ? 0 : a.nb_d, r1 = kind == 0 ? a.nb_d : nrows;
  const double2* base = reinterpret_cast<const double2*>(a.rows) + static_cast<int64_t>(sl) * nrows;
  // rows loaded four ahead of their in-order additions
  Pair q = {0.0, 0.0};
  for (int r = r0 + threadIdx.x; r < r1; r += 4 * BLOCK) {
    double2 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = r + j * BLOCK < r1 ? base[r + j * BLOCK] : double2{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (r + j * BLOCK < r1) q = padd(q, Pair{v[j].x, v[j].y});
  }
  part[threadIdx.x] = q;
  __syncthreads();
#pragma unroll
  for (int st = BLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) part[threadIdx.x] = padd(part[threadIdx.x], part[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = part[0].s + part[0].e;
    a.totals[kind * 64 + sl] = v;
    if (a.host_totals) a.host_totals[kind * 64 + sl] = v;
  }
}

// Third kernel of a context's evaluation: the sequence word, after the slot
// totals that the reduction wrote to mapped host memory (the kernel boundary
// completes those writes), behind a system-scope release; the host forms the
// NLL and gradient from the totals (finalize() in finalize.h). Assembling the
// gradient on the device instead took 3.3 us of a 79 us step: 64 lanes on
// diverging paths, each a chain of dependent steps, where the host needs well
// under a microsecond.
__global__ __launch_bounds__(64) void publish_kernel(EvalArgs a) {
  if (a.seq > 0.0 && threadIdx.x == 0)
    __hip_atomic_store(a.result + 7, a.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Per-event diagnostics: |A|^2, |Ab|^2, Re(A Ab*), Im(A Ab*), rate.
template <class R, int MA, int MB>
__global__ __launch_bounds__(BLOCK) void terms_kernel(TermsArgs a, EvalParams p) {
  const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= a.n) return;
  const LsConst<R>& L = ls_of<R>(p);
  EventIn<R> e;
  load_event<R, MA | MB>(columns<R>(static_cast<const R*>(a.cache), a.ld), i, e);
  Amps<R> am;
  amplitudes<R, MA, MB>(L, e, am);
  const Mom m = moments(am.A, am.Ab);
  double* o = a.out + 5 * i;
  o[0] = m.a2;
  o[1] = m.b2;
  o[2] = m.xr;
  o[3] = m.xi;
  o[4] = a.t ? rate_eq1(m, time_fns(p.mix, a.t[i])) : rate_int(m, p.mix);
}

// ===========================================================================
// Batched passes of the fit server (see BatchArgs).
// ===========================================================================
// The parameter table, the active list and the rows are passed again as
// restrict-qualified arguments: knowing that the row stores do not write the
// parameters, the compiler loads those (uniform) with scalar loads into
// SGPRs, as it does kernel arguments, and not per use into VGPRs.
// BKG: data with a background component; the pass takes 1 / Nhat of each
// fit from its parameters (the host forms it from the Gram matrix) and
// writes the two extra sums.
// RES: data with a Gaussian decay-time resolution.
// BASIS: the fits hold their bases (fixed lineshapes; v.cache is the basis)
// instead of tier-0 records.
template <class R, int MA, int MB, bool BKG = false, bool RES = false, bool BASIS = false>
__global__ __launch_bounds__(BLOCK) void batch_data_kernel(BatchArgs a,
                                                           const EvalParams* __restrict__ params,
                                                           double* __restrict__ rows) {
  using S = Slots<true, MA, MB, BKG>;
  constexpr int NS = S::NS, NT = S::NT, P = S::P;
  __shared__ double lds[(BLOCK / 64) * P];
  __shared__ double gacc[BASIS ? 1 : S::template lds_words<R>() * BLOCK];
  const int n_items = *a.n_items;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {  // uniform trip count
    const FitItem item = a.items[it];
    const FitView v = a.views[item.slot];
    const EvalParams& p = params[item.slot];
    const R* cache = static_cast<const R*>(v.cache);
    const double inv_nhat = BKG ? p.mix.inv_nhat : 0.0;
    double acc[P];
#pragma unroll
    for (int s = 0; s < P; ++s) acc[s] = 0.0;
    // the data pass of eval_block: next-event prefetch and the running
    // widths formed from s with FP32 amplitudes
    if constexpr (BASIS) {
      // the basis in the server's precision, the evaluation in FP64
      Reg64<S::NADJ> gr;
#pragma unroll
      for (int s = 0; s < S::NADJ; ++s) gr.v[s] = 0.0;
      run_basis<R, MA, MB, P, Reg64<S::NADJ>&, BKG, RES>(p, cache, v.t, v.ld, item.lo, item.hi, acc, gr,
                                                          inv_nhat);
#pragma unroll
      for (int s = S::NREG; s < NS; ++s) acc[s] = gr.v[s - S::NREG];
    } else if constexpr (sizeof(R) == 4) {
      float gr[S::NADJ];
#pragma unroll
      for (int s = 0; s < S::NADJ; ++s) gr[s] = 0.0f;
      run_events<R, MA, MB, true, true, true, P, float (&)[S::NADJ], BKG, RES,
                 recompute_widths<R, true, true>()>(p, cache, v.t, v.ld, item.lo, item.hi, acc, gr,
                                                    inv_nhat);
#pragma unroll
      for (int s = S::NREG; s < NS; ++s) acc[s] = static_cast<double>(gr[s - S::NREG]);
    } else {
      double* gl = gacc + threadIdx.x;
#pragma unroll
      for (int s = 0; s < S::NADJ; ++s) gl[s * BLOCK] = 0.0;
      run_events<R, MA, MB, true, true, false, P, double*&, BKG, RES>(p, cache, v.t, v.ld, item.lo, item.hi,
                                                                    acc, gl, inv_nhat);
#pragma unroll
      for (int s = S::NREG; s < NS; ++s) acc[s] = gl[(s - S::NREG) * BLOCK];
    }
    const Pair r = block_reduce<NT, P>(acc, lds);
    if (threadIdx.x < NT) {
      const int64_t o = (static_cast<int64_t>(threadIdx.x) * a.max_rows + item.row) * 2;
      rows[o] = r.s;
      rows[o + 1] = r.e;
    }
    __syncthreads();  // lds is reused by the next item
  }
}

// MC pass of a server with floating lineshapes: every active fit's MC sums at
// its own point, over one shared MC sample. Item it = 8 q + x of the walk is
// (range, fit) = (8 (q / K) + x, q mod K) for K active fits. Workgroups go to
// the eight XCDs in turn and the grid is a multiple of 8, so workgroup b
// stays on XCD b mod 8 and only takes items with x = b mod 8: the K fits of
// a range run one after another on one XCD, whose L2 (or the memory-side
// cache) serves the later reads, and HBM serves each range about once per
// tick. The arithmetic is that of the MC adjoint pass, K times. The running
// widths are read from the cache: forming them from s, as the single
// evaluation does, saves reads that the later fits of a range take from
// cache anyway, and costs arithmetic K times (measured at 4M MC events, FP32:
// 124 -> 114 us per tick at K = 1, 245 -> 281 us at K = 4).
template <class R, int MA, int MB>
__global__ __launch_bounds__(BLOCK) void batch_mc_kernel(BatchArgs a, const EvalParams* __restrict__ params,
                                                         const int32_t* __restrict__ active,
                                                         double* __restrict__ mc_rows) {
  using S = Slots<true, MA, MB>;
  constexpr int NS = S::NS, P = S::P;
  __shared__ double lds[(BLOCK / 64) * P];
  __shared__ double gacc[S::template lds_words<R>() * BLOCK];
  const int K = *a.n_active;
  const int64_t n_it = static_cast<int64_t>(a.nb_mc) * K;
  const R* cache = static_cast<const R*>(a.mc_cache);
  for (int64_t it = blockIdx.x; it < n_it; it += gridDim.x) {  // uniform trip count
    const int64_t q = it >> 3;
    const int slot = active[q % K];
    const int range = static_cast<int>(q / K) * 8 + static_cast<int>(it & 7);
    const EvalParams& p = params[slot];
    const int64_t lo = std::min<int64_t>(static_cast<int64_t>(range) * a.epb_mc, a.n_mc);
    const int64_t hi = std::min<int64_t>(lo + a.epb_mc, a.n_mc);
    double acc[P];
#pragma unroll
    for (int s = 0; s < P; ++s) acc[s] = 0.0;
    if constexpr (sizeof(R) == 4) {
      float gr[S::NADJ];
#pragma unroll
      for (int s = 0; s < S::NADJ; ++s) gr[s] = 0.0f;
      run_events<R, MA, MB, true, false, true, P>(p, cache, nullptr, a.mc_ld, lo, hi, acc, gr);
#pragma unroll
      for (int s = S::NREG; s < NS; ++s) acc[s] = static_cast<double>(gr[s - S::NREG]);
    } else {
      double* gl = gacc + threadIdx.x;
#pragma unroll
      for (int s = 0; s < S::NADJ; ++s) gl[s * BLOCK] = 0.0;
      run_events<R, MA, MB, true, false, true, P>(p, cache, nullptr, a.mc_ld, lo, hi, acc, gl);
#pragma unroll
      for (int s = S::NREG; s < NS; ++s) acc[s] = gl[(s - S::NREG) * BLOCK];
    }
    const Pair r = block_reduce<NS, P>(acc, lds);
    if (threadIdx.x < NS) {
      const int64_t o =
          ((static_cast<int64_t>(threadIdx.x) * a.max_slots + slot) * a.nb_mc + range) * 2;
      mc_rows[o] = r.s;
      mc_rows[o + 1] = r.e;
    }
    __syncthreads();  // lds and gacc are reused by the next item
  }
}

// Totals of a batched evaluation: one workgroup per (fit slot, sum slot,
// pass) combines that fit's rows of that sum -- its data rows (pass 0) or,
// on a streamed server, its nb_mc MC rows (pass 1) -- in a fixed order: each
// thread a fixed strided subset, then a binary tree of compensated pairs. The
// order depends on neither the other fits nor timing.
__global__ __launch_bounds__(BLOCK) void batch_reduce_kernel(BatchArgs a) {
  __shared__ Pair part[BLOCK];
  const int slot = blockIdx.x, sl = blockIdx.y, pass = blockIdx.z;
  if (slot % a.ngroups != a.group) return;  // another group's fit
  const FitView v = a.views[slot];
  if (!v.active) return;
  const double2* base;
  int n;
  if (pass == 0) {
    base = reinterpret_cast<const double2*>(a.rows) + static_cast<int64_t>(sl) * a.max_rows + v.row0;
    n = v.nrows;
  } else {
    base = reinterpret_cast<const double2*>(a.mc_rows) +
           (static_cast<int64_t>(sl) * a.max_slots + slot) * a.nb_mc;
    n = a.nb_mc;
  }
  Pair q = {0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += BLOCK) {
    const double2 x = base[r];
    q = padd(q, Pair{x.x, x.y});
  }
  part[threadIdx.x] = q;
  __syncthreads();
#pragma unroll
  for (int st = BLOCK / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) part[threadIdx.x] = padd(part[threadIdx.x], part[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.tot[(static_cast<int64_t>(slot) * 2 + pass) * 64 + sl] = part[0].s + part[0].e;
}

// End of a batched evaluation: the totals have reached host memory (the
// reduction writes them there); the flag the host cleared before the launch
// is set behind a system-scope release.
__global__ __launch_bounds__(64) void batch_publish_kernel(BatchArgs a) {
  if (threadIdx.x == 0) __hip_atomic_store(a.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ===========================================================================
// Gram matrix of the reduced chain amplitudes over MC events,
// G_kl = sum_j beta_k,j conj(beta_l,j): a dense events x components
// contraction, run on the matrix cores. Each event contributes the 16 reals
// b = (Re beta_1, Im beta_1, ..., Re beta_8, Im beta_8); the real Gram
// R = sum_j b_j b_j^T is accumulated by v_mfma_f64_16x16x4f64 with the same
// register as A and B operand (lane l holds b_{l mod 16} of event l / 16 of a
// 4-event step), in FP64.
// ===========================================================================
typedef double v4d __attribute__((ext_vector_type(4)));

// Each wave stages and contracts its own 64 events, so the waves synchronise
// only with themselves (LDS order within a wave), and the next event's cache
// values are loaded before the current one is computed and contracted; the
// running widths are formed from s (21 columns read, as in the passes).
template <class R, int MA, int MB>
__global__ __launch_bounds__(BLOCK) void gram_kernel(GramArgs a, EvalParams p) {
  constexpr int U = MA | MB;
  __shared__ double tile[BLOCK][17];
  __shared__ double wsum[BLOCK / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const LsConst<R>& L = ls_of<R>(p);
  const Cols<R> cols = columns<R>(static_cast<const R*>(a.cache), a.ld);
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * a.epb;
  const int64_t hi = lo + a.epb < a.n ? lo + a.epb : a.n;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  EventIn<R> nx;
  bool have_nx = lo + threadIdx.x < hi;
  if (have_nx) load_event<R, U, true>(cols, static_cast<uint32_t>(lo + threadIdx.x), nx);
  for (int64_t base = lo; base < hi; base += BLOCK) {  // the same trip count in every wave
    const EventIn<R> e = nx;
    const bool have = have_nx;
    const int64_t in = base + BLOCK + threadIdx.x;
    have_nx = in < hi;
    if (have_nx) load_event<R, U, true>(cols, static_cast<uint32_t>(in), nx);
    double b[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) b[j] = 0.0;
    if (have) {
      Amps<R> am;
      amplitudes<R, MA, MB, true>(L, e, am);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (U & (1 << k)) {
          b[2 * k] = am.B[k].re;
          b[2 * k + 1] = am.B[k].im;
        }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) tile[threadIdx.x][j] = b[j];
    // the wave reads back only the rows it wrote
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const double v = tile[wave * 64 + 4 * st + (lane >> 4)][lane & 15];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // the FP64 16x16x4 product leaves D[4 j + l / 16][l mod 16] in register j
  // of lane l (its four output registers are four rows apart)
#pragma unroll
  for (int j = 0; j < 4; ++j) wsum[wave][(4 * j + (lane >> 4)) * 16 + (lane & 15)] = acc[j];
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) v += wsum[w][threadIdx.x];
  a.rows[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = v;
}

// Combine the per-workgroup Gram rows in order (TwoSum) and convert the real
// 16 x 16 Gram into the complex 8 x 8 one:
// G_kl = R[2k][2l] + R[2k+1][2l+1] + i (R[2k+1][2l] - R[2k][2l+1]).
// The rows are loaded 32 at a time ahead of their (in-order) additions, so a
// thread waits for one memory latency per 32 rows, not per row.
__global__ __launch_bounds__(BLOCK) void gram_finalize_kernel(GramArgs a) {
  constexpr int AHEAD = 32;
  __shared__ double rg[256];
  Pair q = {0.0, 0.0};
  for (int r0 = 0; r0 < a.nb; r0 += AHEAD) {
    double v[AHEAD];
#pragma unroll
    for (int j = 0; j < AHEAD; ++j)
      v[j] = r0 + j < a.nb ? a.rows[static_cast<int64_t>(r0 + j) * 256 + threadIdx.x] : 0.0;
#pragma unroll
    for (int j = 0; j < AHEAD; ++j)
      if (r0 + j < a.nb) q = padd(q, Pair{v[j], 0.0});
  }
  rg[threadIdx.x] = q.s + q.e;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int k = threadIdx.x >> 3, l = threadIdx.x & 7;
    a.out[threadIdx.x * 2] = rg[(2 * k) * 16 + 2 * l] + rg[(2 * k + 1) * 16 + 2 * l + 1];
    a.out[threadIdx.x * 2 + 1] = rg[(2 * k + 1) * 16 + 2 * l] - rg[(2 * k) * 16 + 2 * l + 1];
  }
}

// ===========================================================================
// Pseudo-experiments (Sec. 3.1): candidates uniform in phase space by GENBOD
// (F. James, CERN 68-15), kept by accept-reject against Eq. (1). Random
// numbers: Philox4x32-10 (Salmon et al., SC11), so every candidate can be
// drawn by any thread, and the kept events come out in candidate order
// whatever the launch shape.
//
// A launch first flags its candidates (kept by GENBOD, kept, above the
// envelope) and counts the kept ones per workgroup; a one-workgroup scan turns
// the counts into output offsets; the write pass redraws the kept candidates
// (bitwise the same draw) and stores them at their rank.
// ===========================================================================
// Ten Philox rounds on (c0, c1, c2, c3) under key (k0, k1).
__device__ inline void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    c0 = hi1 ^ c1 ^ k0;
    c2 = hi0 ^ c3 ^ k1;
    c1 = lo1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}
// (k + 1/2) 2^-52, k = top 52 bits of the 64-bit word (hi, lo): in (0, 1)
__device__ inline double unit52(uint32_t hi, uint32_t lo) {
  const uint64_t k = (static_cast<uint64_t>(hi) << 20) | (lo >> 12);
  return (static_cast<double>(k) + 0.5) * 0x1p-52;
}
// uniforms 2j, 2j+1 of candidate i
__device__ inline void draw2(const GenConst& g, uint64_t i, uint32_t j, double& a, double& b) {
  uint32_t c0 = static_cast<uint32_t>(i), c1 = static_cast<uint32_t>(i >> 32), c2 = j, c3 = g.stream;
  philox10(c0, c1, c2, c3, g.key0, g.key1);
  a = unit52(c0, c1);
  b = unit52(c2, c3);
}

__device__ inline double breakup(double M, double ma, double mb) {
  const double v = (M * M - (ma + mb) * (ma + mb)) * (M * M - (ma - mb) * (ma - mb));
  return v > 0.0 ? sqrt(v) / (2.0 * M) : 0.0;
}
// daughters of a decay at rest with break-up momentum q along
// (cos theta = 2u - 1, phi = 2 pi v)
__device__ inline void split(double q, double ma, double mb, double u, double v, F4& a, F4& b) {
  const double ct = 2.0 * u - 1.0, st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
  double sp, cp;
  sincospi(2.0 * v, &sp, &cp);
  const double qx = q * st * cp, qy = q * st * sp, qz = q * ct;
  a = {sqrt(ma * ma + q * q), qx, qy, qz};
  b = {sqrt(mb * mb + q * q), -qx, -qy, -qz};
}
// p given in the rest frame of P (mass M), returned in P's frame:
// E' = (E_P E + P.p) / M, p' = p + P (E + E') / (E_P + M)
__device__ inline F4 boost_out(F4 p, F4 P, double M) {
  const double e = (P.e * p.e + P.x * p.x + P.y * p.y + P.z * p.z) / M;
  const double f = (p.e + e) / (P.e + M);
  return {e, p.x + f * P.x, p.y + f * P.y, p.z + f * P.z};
}

// GENBOD for the candidate: returns whether it is kept by the weight; if so
// p[4] and (data) t, u11 are filled.
template <bool DATA>
__device__ inline bool gen_candidate(const GenConst& g, uint64_t i, F4 p[4], double& t, double& u11) {
  double u0, u1, u2, u3;
  draw2(g, i, 0, u0, u1);
  draw2(g, i, 1, u2, u3);
  const double T = g.M - (g.m[0] + g.m[1] + g.m[2] + g.m[3]);
  const double rlo = fmin(u0, u1), rhi = fmax(u0, u1);
  const double M2 = g.m[0] + g.m[1] + rlo * T;
  const double M3 = g.m[0] + g.m[1] + g.m[2] + rhi * T;
  const double q2 = breakup(M2, g.m[0], g.m[1]);
  const double q3 = breakup(M3, M2, g.m[2]);
  const double q4 = breakup(g.M, M3, g.m[3]);
  if (!(u2 * g.wmax < q2 * q3 * q4)) return false;
  double u4, u5, u6, u7, u8, u9;
  draw2(g, i, 2, u4, u5);
  draw2(g, i, 3, u6, u7);
  draw2(g, i, 4, u8, u9);
  F4 P01, P012;
  split(q2, g.m[0], g.m[1], u3, u4, p[0], p[1]);
  split(q3, M2, g.m[2], u5, u6, P01, p[2]);
  p[0] = boost_out(p[0], P01, M2);
  p[1] = boost_out(p[1], P01, M2);
  split(q4, M3, g.m[3], u7, u8, P012, p[3]);
#pragma unroll
  for (int j = 0; j < 3; ++j) p[j] = boost_out(p[j], P012, M3);
  if (DATA) {
    double u10;
    draw2(g, i, 5, u10, u11);
    const double lam = u9 < 0.5 * (1.0 + g.y) ? g.gamma * (1.0 - g.y) : g.gamma * (1.0 + g.y);
    t = -log(u10) / lam;
  }
  return true;
}

template <int MA, int MB, bool DATA>
__global__ __launch_bounds__(BLOCK) void gen_flags_kernel(GenArgs a, EvalParams p) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;  // < a.g.n
  uint32_t f = 0;
  F4 q[4];
  double t = 0.0, u11 = 0.0;
  if (gen_candidate<DATA>(a.g, a.g.first + static_cast<uint64_t>(c), q, t, u11)) {
    f = 1;
    if (DATA) {
      double o[NCOL];
      tier0_event(a.g.t0, q, o);
      EventIn<double> e;
#pragma unroll
      for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int j = 0; j < CPS; ++j) e.v[sg][j] = o[CPS * sg + j];
      e.s3 = o[C_S3PI];
      Amps<double> am;
      amplitudes<double, MA, MB>(ls_of<double>(p), e, am);
      const TimeFns tf = time_fns(p.mix, t);
      const double B = rate_eq1(moments(am.A, am.Ab), tf);
      const double E = 2.0 * tf.ch * a.g.envelope;
      if (B > E) f |= 4;
      if (u11 * E < B) f |= 2;
    } else {
      f |= 2;
    }
  }
  a.flags[c] = static_cast<uint8_t>(f);
  const int kept = __syncthreads_count((f & 2) != 0);
  if (threadIdx.x == 0) a.bcount[blockIdx.x] = static_cast<uint32_t>(kept);
}

// exclusive prefix of the per-workgroup counts, in one workgroup
__global__ __launch_bounds__(FIN_BLOCK) void gen_scan_kernel(GenArgs a, int32_t nb) {
  __shared__ uint32_t part[FIN_BLOCK];
  const int per = (nb + FIN_BLOCK - 1) / FIN_BLOCK;
  const int lo = threadIdx.x * per, hi = min(lo + per, nb);
  uint32_t s = 0;
  for (int b = lo; b < hi; ++b) s += a.bcount[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < FIN_BLOCK; ++k) {
      const uint32_t v = part[k];
      part[k] = run;
      run += v;
    }
    *a.total = run;
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (int b = lo; b < hi; ++b) {
    a.boff[b] = run;
    run += a.bcount[b];
  }
}

template <bool DATA>
__global__ __launch_bounds__(BLOCK) void gen_write_kernel(GenArgs a) {
  __shared__ uint32_t wcount[BLOCK / 64];
  const int64_t c = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;  // < a.g.n
  const bool keep = (a.flags[c] & 2) != 0;
  const uint64_t mask = __ballot(keep);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t below = static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
  if (lane == 0) wcount[wave] = static_cast<uint32_t>(__popcll(mask));
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += wcount[w];
  if (!keep) return;
  const int64_t r = a.filled + a.boff[blockIdx.x] + woff + below;
  if (r >= a.n_out) return;
  F4 q[4];
  double t = 0.0, u11 = 0.0;
  gen_candidate<DATA>(a.g, a.g.first + static_cast<uint64_t>(c), q, t, u11);
  double* o = a.p4 + 16 * r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    o[4 * j] = q[j].e;
    o[4 * j + 1] = q[j].x;
    o[4 * j + 2] = q[j].y;
    o[4 * j + 3] = q[j].z;
  }
  if (DATA) a.t[r] = t;
  if (a.idx) a.idx[r] = static_cast<int64_t>(a.g.first + static_cast<uint64_t>(c));
  if (r == a.n_out - 1) *a.last = c;
}

// GENBOD and exceedance counts of the candidates below the cut: one packed
// word per workgroup (reusing the per-workgroup count array), then one
// workgroup adds them up.
__global__ __launch_bounds__(BLOCK) void gen_stats_kernel(GenArgs a, int64_t limit) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const uint32_t f = c < limit ? a.flags[c] : 0u;
  const int ps = __syncthreads_count(f & 1u);
  const int ex = __syncthreads_count((f >> 2) & 1u);
  if (threadIdx.x == 0) a.bcount[blockIdx.x] = static_cast<uint32_t>(ps) | (static_cast<uint32_t>(ex) << 16);
}

__global__ __launch_bounds__(FIN_BLOCK) void gen_sum_kernel(GenArgs a, int32_t nb) {
  __shared__ unsigned long long part[2][FIN_BLOCK];
  unsigned long long ps = 0, ex = 0;
  for (int b = threadIdx.x; b < nb; b += FIN_BLOCK) {
    const uint32_t w = a.bcount[b];
    ps += w & 0xFFFFu;
    ex += w >> 16;
  }
  part[0][threadIdx.x] = ps;
  part[1][threadIdx.x] = ex;
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long t = 0;
    for (int k = 0; k < FIN_BLOCK; ++k) t += part[threadIdx.x][k];
    a.counts[threadIdx.x] = t;
  }
}

// ===========================================================================
// Many parameter sets that share the lineshapes (for example the points of a
// numerical-gradient stencil): per data event the chain amplitudes B_k are
// computed once, and A_f, Abar_f of every set follow from the dense product
// [events x 16] . W[16 x 4 sets] (Eq. (2) with the coefficients of each set
// as columns), run on the matrix cores. The normalisation of each set comes
// from the MC Gram matrix.
//
// Workgroup (x, y): events [x epb, (x+1) epb) and sets 16 y .. 16 y + 15.
// Per 64-event tile of a wave: each lane writes its event's 16 reals to LDS;
// for each group of 16 events the wave forms the 16 x 64 block of (Re A,
// Im A, Re Abar, Im Abar) x 16 sets with 16 products 16x16x4, stores it in
// LDS, and every lane then finishes four (event, set) pairs: moments,
// Eq. (1) in FP64 at the set's x, y, and -ln B.
// ===========================================================================
template <class R> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in register r of lane l
  static __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int l, int r) { return 4 * r + (l >> 4); }
};

template <class R, int MA, int MB, bool RES = false>
__global__ __launch_bounds__(BLOCK) void multi_data_kernel(MultiArgs a, EvalParams p0) {
  constexpr int U = MA | MB, NW = BLOCK / 64;
  __shared__ R btile[NW][64][17];
  __shared__ R dtile[NW][16][65];
  __shared__ Pair red[NW][16][3];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sl = lane & 15, eg = lane >> 4;  // set within the chunk; event row class
  const int set = 16 * blockIdx.y + sl;
  const bool sv = set < a.n_sets;
  const EvalParams& ps = a.params[sv ? set : 0];
  const double xg = ps.mix.xg, yg = ps.mix.yg, gam = ps.mix.gamma;
  // this lane's contraction operands: W[4 kk + eg][64 y + 16 q + sl]
  const R* W = static_cast<const R*>(a.w);
  R w[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      w[q][kk] = W[(4 * kk + eg) * a.ldw + 64 * blockIdx.y + 16 * q + sl];
  const LsConst<R>& L = ls_of<R>(p0);
  const Cols<R> cols = columns<R>(static_cast<const R*>(a.cache), a.ld);
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * a.epb;
  const int64_t hi = lo + a.epb < a.n ? lo + a.epb : a.n;
  double s_l = 0.0, s_abs = 0.0, s_bad = 0.0;
  for (int64_t base = lo; base < hi; base += BLOCK) {  // same trip count in every wave
    const int64_t tile = base + 64 * wave;
    const int64_t i = tile + lane;
    R b[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) b[j] = R(0);
    if (i < hi) {
      EventIn<R> e;
      load_event<R, U>(cols, static_cast<uint32_t>(i), e);
      Amps<R> am;
      amplitudes<R, MA, MB>(L, e, am);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (U & (1 << k)) {
          b[2 * k] = am.B[k].re;
          b[2 * k + 1] = am.B[k].im;
        }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) btile[wave][lane][j] = b[j];
    __syncthreads();
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
      // A operand: lane l holds B of event 16 g + (l mod 16), component 4 kk + l / 16
      R av[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) av[kk] = btile[wave][16 * g + sl][4 * kk + eg];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        typename Mfma<R>::v4 c = {R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) c = Mfma<R>::mma(av[kk], w[q][kk], c);
#pragma unroll
        for (int r = 0; r < 4; ++r) dtile[wave][Mfma<R>::row(lane, r)][16 * q + sl] = c[r];
      }
      __syncthreads();
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int er = eg + 4 * jj;
        const int64_t ev = tile + 16 * g + er;
        if (sv && ev < hi) {
          const R* d = &dtile[wave][er][4 * sl];
          const Mom m = moments(Cp<R>{d[0], d[1]}, Cp<R>{d[2], d[3]});
          const double t = a.t[ev];
          TimeFns f;
          if constexpr (RES) {
            f = res_fns(ps.mix, t).f;  // B is then the resolved rate, e^{-Gamma t} inside
          } else {
            mix_cosh_sinh(yg * t, &f.ch, &f.sh);
            mix_sincos(xg * t, &f.sn, &f.cs);
          }
          const double B = rate_eq1(m, f);
          const bool ok = B > 0.0 && B < INFINITY;
          double l;
          if (ps.mix.g_bkg > 0.0) {
            // the mixture density with this set's 1 / Nhat and fraction
            double es, eb;
            if constexpr (RES) {
              Cd E, dE;
              conv_exp(ps.mix.g_bkg, 0.0, t, ps.mix.sigma_t, &E, &dE);
              es = ps.mix.inv_nhat;
              eb = ps.mix.g_bkg * E.re;
            } else {
              es = mix_exp(-gam * t) * ps.mix.inv_nhat;
              eb = ps.mix.g_bkg * mix_exp(-ps.mix.g_bkg * t);
            }
            l = ok ? -log((1.0 - ps.mix.f_bkg) * B * es + ps.mix.f_bkg * eb) : 0.0;
          } else {
            l = ok ? (RES ? -log(B) : gam * t - log(B)) : 0.0;
          }
          s_l += l;
          s_abs += fabs(l);
          s_bad += ok ? 0.0 : 1.0;
        }
      }
      __syncthreads();
    }
  }
  // lanes l, l + 16, l + 32, l + 48 hold the same set: combine them in a
  // fixed order, then the waves
  Pair q[3] = {{s_l, 0.0}, {s_abs, 0.0}, {s_bad, 0.0}};
#pragma unroll
  for (int off = 16; off < 64; off <<= 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const Pair o = {__shfl_xor(q[k].s, off), __shfl_xor(q[k].e, off)};
      q[k] = (lane & off) ? padd(o, q[k]) : padd(q[k], o);
    }
  if (lane < 16)
#pragma unroll
    for (int k = 0; k < 3; ++k) red[wave][lane][k] = q[k];
  __syncthreads();
  if (threadIdx.x < 48) {
    const int s = threadIdx.x / 3, k = threadIdx.x % 3;
    Pair r = red[0][s][k];
#pragma unroll
    for (int w2 = 1; w2 < NW; ++w2) r = padd(r, red[w2][s][k]);
    const int gs = 16 * blockIdx.y + s;
    if (gs < a.n_sets) {
      double* o = a.rows + ((static_cast<int64_t>(gs) * 3 + k) * a.nb + blockIdx.x) * 2;
      o[0] = r.s;
      o[1] = r.e;
    }
  }
}

// One workgroup per set: its rows in a fixed order, the MC normalisation
// from the Gram matrix, and the NLL.
template <int MA, int MB>
__global__ __launch_bounds__(64) void multi_finalize_kernel(MultiArgs a) {
  __shared__ Pair part[3][64];
  __shared__ double tot[3];
  const int set = blockIdx.x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double2* r = reinterpret_cast<const double2*>(a.rows) + (static_cast<int64_t>(set) * 3 + k) * a.nb;
    Pair q = {0.0, 0.0};
    for (int b = threadIdx.x; b < a.nb; b += 64) q = padd(q, Pair{r[b].x, r[b].y});
    part[k][threadIdx.x] = q;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    Pair q = {0.0, 0.0};
    for (int j = 0; j < 64; ++j) q = padd(q, part[threadIdx.x][j]);
    tot[threadIdx.x] = q.s + q.e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const EvalParams& p = a.params[set];
    double M[48];
    mc_from_gram<MA, MB>(p, a.gram, M);
    EvalArgs e = {};
    e.n_d = a.n;
    e.n_m = a.n_mc;
    e.result = a.results + static_cast<int64_t>(set) * RES_WORDS;
    finalize<MA, MB, 4>(e, p, tot, M, false);
  }
}

// Chain masks with dedicated instantiations: the four-component model
// (A_f = {1, 4}, Abar_f = {5, 2}) and the fourteen-component one
// (A_f = {1,2,3,4,7,8}, Abar_f = all). Any other model runs the general
// instantiation (all chains, absent ones with zero coefficients).
constexpr int SMALL_A = 0x09, SMALL_B = 0x12, FULL_A = 0xCF, FULL_B = 0xFF;

template <class R, int MA, int MB, bool GRAD>
hipError_t launch_eval_m(const EvalArgs& a, const EvalParams& p, hipStream_t s, hipEvent_t t0,
                         hipEvent_t t1) {
  const dim3 block(BLOCK);
  hipError_t e = hipSuccess;
  if (p.mix.g_bkg > 0.0) {
    // background component: the data pass needs Nhat, so the MC pass and its
    // reduction come first
    // (in Gram mode there is no MC pass: Nhat comes from the host)
    if (a.nb_m > 0) {
      if (t0 && (e = hipEventRecord(t0, s)) != hipSuccess) return e;
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, false>), dim3(a.nb_m), block, 0, s, a, p);
      if (t1 && (e = hipEventRecord(t1, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(Slots<GRAD, MA, MB>::NS, 1), block, 0, s, a, 1);
    if (a.nb_d > 0 && p.mix.sigma_t > 0.0)
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, true, true, true>), dim3(a.nb_d), block, 0, s, a, p);
    else if (a.nb_d > 0)
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, true, true>), dim3(a.nb_d), block, 0, s, a, p);
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(Slots<GRAD, MA, MB, true>::NT, 1), block, 0, s, a, 0);
  } else if (p.mix.sigma_t > 0.0) {
    // decay-time resolution: its own data pass, then the MC pass
    if (a.nb_d > 0)
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, true, false, true>), dim3(a.nb_d), block, 0, s, a, p);
    if (a.nb_m > 0) {
      if (t0 && (e = hipEventRecord(t0, s)) != hipSuccess) return e;
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, false>), dim3(a.nb_m), block, 0, s, a, p);
      if (t1 && (e = hipEventRecord(t1, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(Slots<GRAD, MA, MB>::NS, 2), block, 0, s, a, 0);
  } else if (a.nb_d > 0 && a.nb_m > 0) {
    // one launch for both passes (the timing events bracket it)
    if (t0 && (e = hipEventRecord(t0, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((eval_both_kernel<R, MA, MB, GRAD>), dim3(a.nb_d + a.nb_m), block, 0, s, a, p);
    if (t1 && (e = hipEventRecord(t1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(Slots<GRAD, MA, MB>::NS, 2), block, 0, s, a, 0);
  } else {
    if (a.nb_d > 0)
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, true>), dim3(a.nb_d), block, 0, s, a, p);
    if (a.nb_m > 0) {
      if (t0 && (e = hipEventRecord(t0, s)) != hipSuccess) return e;
      hipLaunchKernelGGL((eval_kernel<R, MA, MB, GRAD, false>), dim3(a.nb_m), block, 0, s, a, p);
      if (t1 && (e = hipEventRecord(t1, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(slot_reduce_kernel, dim3(Slots<GRAD, MA, MB>::NS, 2), block, 0, s, a, 0);
  }
  hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <class R, bool GRAD>
hipError_t launch_eval_r(int ma, int mb, const EvalArgs& a, const EvalParams& p, hipStream_t s,
                         hipEvent_t t0, hipEvent_t t1) {
  if (ma == SMALL_A && mb == SMALL_B) return launch_eval_m<R, SMALL_A, SMALL_B, GRAD>(a, p, s, t0, t1);
  if (ma == FULL_A && mb == FULL_B) return launch_eval_m<R, FULL_A, FULL_B, GRAD>(a, p, s, t0, t1);
  return launch_eval_m<R, 0xFF, 0xFF, GRAD>(a, p, s, t0, t1);
}

template <class R>
hipError_t launch_terms_r(int ma, int mb, const TermsArgs& a, const EvalParams& p, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.n + BLOCK - 1) / BLOCK)), block(BLOCK);
  if (ma == SMALL_A && mb == SMALL_B)
    hipLaunchKernelGGL((terms_kernel<R, SMALL_A, SMALL_B>), grid, block, 0, s, a, p);
  else if (ma == FULL_A && mb == FULL_B)
    hipLaunchKernelGGL((terms_kernel<R, FULL_A, FULL_B>), grid, block, 0, s, a, p);
  else
    hipLaunchKernelGGL((terms_kernel<R, 0xFF, 0xFF>), grid, block, 0, s, a, p);
  return hipGetLastError();
}

template <class R>
hipError_t launch_gram_r(int ma, int mb, const GramArgs& a, const EvalParams& p, hipStream_t s) {
  const dim3 grid(a.nb), block(BLOCK);
  if (ma == SMALL_A && mb == SMALL_B)
    hipLaunchKernelGGL((gram_kernel<R, SMALL_A, SMALL_B>), grid, block, 0, s, a, p);
  else if (ma == FULL_A && mb == FULL_B)
    hipLaunchKernelGGL((gram_kernel<R, FULL_A, FULL_B>), grid, block, 0, s, a, p);
  else
    hipLaunchKernelGGL((gram_kernel<R, 0xFF, 0xFF>), grid, block, 0, s, a, p);
  hipLaunchKernelGGL(gram_finalize_kernel, dim3(1), block, 0, s, a);
  return hipGetLastError();
}

template <class R, int MA, int MB>
hipError_t launch_batch_m(const BatchArgs& a, hipStream_t s) {
  constexpr int NS = Slots<true, MA, MB>::NS;
  const dim3 grid(BATCH_GRID), block(BLOCK);
  if (a.mc_cache) {
    // floating lineshapes: the fits' tier-0 records and the MC walk (no
    // model extensions: the host refuses them)
    if (a.mc_grid < 8 || a.mc_grid % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((batch_data_kernel<R, MA, MB>), grid, block, 0, s, a, a.params, a.rows);
    hipLaunchKernelGGL((batch_mc_kernel<R, MA, MB>), dim3(a.mc_grid), block, 0, s, a, a.params,
                       a.active, a.mc_rows);
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(a.max_slots, NS, 2), block, 0, s, a);
  } else {
    // fixed lineshapes: the fits' bases
    constexpr int NT = Slots<true, MA, MB, true>::NT;
    if (a.bkg && a.res)
      hipLaunchKernelGGL((batch_data_kernel<R, MA, MB, true, true, true>), grid, block, 0, s, a, a.params, a.rows);
    else if (a.bkg)
      hipLaunchKernelGGL((batch_data_kernel<R, MA, MB, true, false, true>), grid, block, 0, s, a, a.params, a.rows);
    else if (a.res)
      hipLaunchKernelGGL((batch_data_kernel<R, MA, MB, false, true, true>), grid, block, 0, s, a, a.params, a.rows);
    else
      hipLaunchKernelGGL((batch_data_kernel<R, MA, MB, false, false, true>), grid, block, 0, s, a, a.params,
                         a.rows);
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(a.max_slots, a.bkg ? NT : NS, 1), block, 0, s, a);
  }
  hipLaunchKernelGGL(batch_publish_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// Workgroups of the MC walk: as many as the device holds at once, rounded
// down to a multiple of the 8 XCDs.
template <class R, int MA, int MB>
int mc_grid_m(int device) {
  int per_cu = 0, n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_mc_kernel<R, MA, MB>, BLOCK, 0) != hipSuccess)
    return 0;
  return std::max(8, per_cu * n_cu / 8 * 8);
}

template <class R>
int mc_grid_r(int ma, int mb, int device) {
  if (ma == SMALL_A && mb == SMALL_B) return mc_grid_m<R, SMALL_A, SMALL_B>(device);
  if (ma == FULL_A && mb == FULL_B) return mc_grid_m<R, FULL_A, FULL_B>(device);
  return mc_grid_m<R, 0xFF, 0xFF>(device);
}

template <class R>
hipError_t launch_batch_r(int ma, int mb, const BatchArgs& a, hipStream_t s) {
  if (ma == SMALL_A && mb == SMALL_B) return launch_batch_m<R, SMALL_A, SMALL_B>(a, s);
  if (ma == FULL_A && mb == FULL_B) return launch_batch_m<R, FULL_A, FULL_B>(a, s);
  return launch_batch_m<R, 0xFF, 0xFF>(a, s);
}

template <bool DATA>
hipError_t launch_gen_m(int ma, int mb, const GenArgs& a, const EvalParams& p, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(a.g.n / BLOCK)), block(BLOCK);
  if (ma == SMALL_A && mb == SMALL_B)
    hipLaunchKernelGGL((gen_flags_kernel<SMALL_A, SMALL_B, DATA>), grid, block, 0, s, a, p);
  else if (ma == FULL_A && mb == FULL_B)
    hipLaunchKernelGGL((gen_flags_kernel<FULL_A, FULL_B, DATA>), grid, block, 0, s, a, p);
  else
    hipLaunchKernelGGL((gen_flags_kernel<0xFF, 0xFF, DATA>), grid, block, 0, s, a, p);
  hipLaunchKernelGGL(gen_scan_kernel, dim3(1), dim3(FIN_BLOCK), 0, s, a,
                     static_cast<int32_t>(a.g.n / BLOCK));
  hipLaunchKernelGGL((gen_write_kernel<DATA>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <class R>
hipError_t launch_multi_r(int ma, int mb, const MultiArgs& a, const EvalParams& p0, hipStream_t s) {
  const dim3 grid(a.nb, a.ldw / 64), block(BLOCK), fgrid(a.n_sets), fblock(64);
  const bool res = p0.mix.sigma_t > 0.0;
  if (ma == SMALL_A && mb == SMALL_B) {
    if (a.nb > 0 && res)
      hipLaunchKernelGGL((multi_data_kernel<R, SMALL_A, SMALL_B, true>), grid, block, 0, s, a, p0);
    else if (a.nb > 0)
      hipLaunchKernelGGL((multi_data_kernel<R, SMALL_A, SMALL_B>), grid, block, 0, s, a, p0);
    hipLaunchKernelGGL((multi_finalize_kernel<SMALL_A, SMALL_B>), fgrid, fblock, 0, s, a);
  } else if (ma == FULL_A && mb == FULL_B) {
    if (a.nb > 0 && res)
      hipLaunchKernelGGL((multi_data_kernel<R, FULL_A, FULL_B, true>), grid, block, 0, s, a, p0);
    else if (a.nb > 0)
      hipLaunchKernelGGL((multi_data_kernel<R, FULL_A, FULL_B>), grid, block, 0, s, a, p0);
    hipLaunchKernelGGL((multi_finalize_kernel<FULL_A, FULL_B>), fgrid, fblock, 0, s, a);
  } else {
    if (a.nb > 0 && res)
      hipLaunchKernelGGL((multi_data_kernel<R, 0xFF, 0xFF, true>), grid, block, 0, s, a, p0);
    else if (a.nb > 0)
      hipLaunchKernelGGL((multi_data_kernel<R, 0xFF, 0xFF>), grid, block, 0, s, a, p0);
    hipLaunchKernelGGL((multi_finalize_kernel<0xFF, 0xFF>), fgrid, fblock, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gen_chunk(bool data, int ma, int mb, const GenArgs& a, const EvalParams& p,
                            hipStream_t s) {
  if (a.g.n <= 0 || a.g.n % BLOCK != 0 || a.g.n / BLOCK > (int64_t(1) << 20))
    return hipErrorInvalidValue;
  return data ? launch_gen_m<true>(ma, mb, a, p, s) : launch_gen_m<false>(ma, mb, a, p, s);
}

hipError_t launch_gen_stats(const GenArgs& a, int64_t limit, hipStream_t s) {
  if (limit <= 0) return hipSuccess;
  if (limit > a.g.n) return hipErrorInvalidValue;
  const int32_t nb = static_cast<int32_t>((limit + BLOCK - 1) / BLOCK);
  hipLaunchKernelGGL(gen_stats_kernel, dim3(nb), dim3(BLOCK), 0, s, a, limit);
  hipLaunchKernelGGL(gen_sum_kernel, dim3(1), dim3(FIN_BLOCK), 0, s, a, nb);
  return hipGetLastError();
}

bool specialised(int ma, int mb) {
  return (ma == SMALL_A && mb == SMALL_B) || (ma == FULL_A && mb == FULL_B);
}

int slots_for(bool grad, int ma, int mb) {
  if (!specialised(ma, mb)) ma = mb = 0xFF;
  return grad ? 11 + 2 * (popc(ma) + popc(mb)) : 4;
}

namespace {
template <int MA, int MB>
void finalize_host_m(bool grad, const EvalArgs& a, const EvalParams& p, const double* D, double* M,
                     const double* G) {
  if (G) mc_from_gram<MA, MB>(p, G, M);
  if (grad)
    finalize<MA, MB, Slots<true, MA, MB>::NS>(a, p, D, M, true);
  else
    finalize<MA, MB, Slots<false, MA, MB>::NS>(a, p, D, M, false);
}
}  // namespace

double gram_sum_t(int ma, int mb, const EvalParams& p, const double* G) {
  double M[64];
  if (ma == SMALL_A && mb == SMALL_B)
    mc_from_gram<SMALL_A, SMALL_B>(p, G, M);
  else if (ma == FULL_A && mb == FULL_B)
    mc_from_gram<FULL_A, FULL_B>(p, G, M);
  else
    mc_from_gram<0xFF, 0xFF>(p, G, M);
  const MixConst& x = p.mix;
  return x.h_sum * (M[0] + M[1]) + x.h_diff * (M[0] - M[1]) - x.h_re * M[2] - x.h_im * M[3];
}

void finalize_host(int ma, int mb, bool grad, const EvalArgs& a, const EvalParams& p, const double* D,
                   double* M, const double* G) {
  if (ma == SMALL_A && mb == SMALL_B)
    finalize_host_m<SMALL_A, SMALL_B>(grad, a, p, D, M, G);
  else if (ma == FULL_A && mb == FULL_B)
    finalize_host_m<FULL_A, FULL_B>(grad, a, p, D, M, G);
  else
    finalize_host_m<0xFF, 0xFF>(grad, a, p, D, M, G);
}

template <class R>
hipError_t launch_basis_r(int ma, int mb, const R* cache, int64_t ld, int64_t n, const EvalParams& p, R* basis,
                          int64_t bld, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((n + BLOCK - 1) / BLOCK)), block(BLOCK);
  if (ma == SMALL_A && mb == SMALL_B)
    hipLaunchKernelGGL((basis_kernel<R, SMALL_A, SMALL_B>), grid, block, 0, s, cache, ld, n, p, basis, bld);
  else if (ma == FULL_A && mb == FULL_B)
    hipLaunchKernelGGL((basis_kernel<R, FULL_A, FULL_B>), grid, block, 0, s, cache, ld, n, p, basis, bld);
  else
    hipLaunchKernelGGL((basis_kernel<R, 0xFF, 0xFF>), grid, block, 0, s, cache, ld, n, p, basis, bld);
  return hipGetLastError();
}

int basis_columns(int ma, int mb) {
  if (ma == SMALL_A && mb == SMALL_B) return 2 * popc(SMALL_A | SMALL_B);
  if (ma == FULL_A && mb == FULL_B) return 2 * popc(FULL_A | FULL_B);
  return 16;
}

hipError_t launch_basis(int precision, int ma, int mb, const void* cache, int64_t ld, int64_t n,
                        const EvalParams& p, void* basis, int64_t bld, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > INT32_MAX / 8 || bld < n || ld < n) return hipErrorInvalidValue;
  return precision == 0 ? launch_basis_r<double>(ma, mb, static_cast<const double*>(cache), ld, n, p,
                                                 static_cast<double*>(basis), bld, s)
                        : launch_basis_r<float>(ma, mb, static_cast<const float*>(cache), ld, n, p,
                                                static_cast<float*>(basis), bld, s);
}

hipError_t launch_tier0(const Tier0Const& k, const double* p4, const double* t, int64_t n, int64_t ld,
                        double* c64, float* c32, double* t64, unsigned* n_bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n + BLOCK - 1) / BLOCK)), block(BLOCK);
  hipLaunchKernelGGL(tier0_kernel, grid, block, 0, s, k, p4, t, n, ld, c64, c32, t64, n_bad);
  return hipGetLastError();
}

hipError_t launch_eval(int precision, bool grad, int ma, int mb, const EvalArgs& a,
                       const EvalParams& p, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (precision == 0)
    return grad ? launch_eval_r<double, true>(ma, mb, a, p, s, t0, t1)
                : launch_eval_r<double, false>(ma, mb, a, p, s, t0, t1);
  return grad ? launch_eval_r<float, true>(ma, mb, a, p, s, t0, t1)
              : launch_eval_r<float, false>(ma, mb, a, p, s, t0, t1);
}

int batch_mc_grid(int precision, int ma, int mb, int device) {
  return precision == 0 ? mc_grid_r<double>(ma, mb, device) : mc_grid_r<float>(ma, mb, device);
}

hipError_t launch_batch(int precision, int ma, int mb, const BatchArgs& a, hipStream_t s) {
  return precision == 0 ? launch_batch_r<double>(ma, mb, a, s) : launch_batch_r<float>(ma, mb, a, s);
}

hipError_t launch_gram(int precision, int ma, int mb, const GramArgs& a, const EvalParams& p,
                       hipStream_t s) {
  if (a.n <= 0 || a.nb <= 0) return hipErrorInvalidValue;
  return precision == 0 ? launch_gram_r<double>(ma, mb, a, p, s)
                        : launch_gram_r<float>(ma, mb, a, p, s);
}

hipError_t launch_terms(int precision, int ma, int mb, const TermsArgs& a, const EvalParams& p,
                        hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  return precision == 0 ? launch_terms_r<double>(ma, mb, a, p, s)
                        : launch_terms_r<float>(ma, mb, a, p, s);
}

hipError_t launch_multi(int precision, int ma, int mb, const MultiArgs& a, const EvalParams& p0,
                        hipStream_t s) {
  if (a.n_sets < 1 || a.n_sets > MAX_SETS || a.ldw < 64 || a.ldw % 64 != 0 ||
      a.n_sets > 16 * (a.ldw / 64) || a.nb < 0 || (a.nb > 0 && a.epb % BLOCK != 0))
    return hipErrorInvalidValue;
  return precision == 0 ? launch_multi_r<double>(ma, mb, a, p0, s)
                        : launch_multi_r<float>(ma, mb, a, p0, s);
}

}  // namespace mxa
