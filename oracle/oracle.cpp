// Oracle: a plain, slow FP64 CPU definition of the likelihood of the
// time-dependent amplitude model for D0 -> K+ pi- pi+ pi- (Hasse et al.,
// "Amplitude analysis of four-body decays using a massively-parallel fitting
// framework", arXiv:1702.06735).
//
// TEST INFRASTRUCTURE ONLY. The GPU library is checked against this file; the
// two share no code. Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark load it.
//
// Everything is recomputed per event from the raw four-momenta, with no
// caching and no reordering beyond what the definitions state:
//   Sec. 3 and Fig. 2: quasi-two-body decay chains, each the product of a spin
//       factor, form (barrier) factors and resonance lineshapes, Bose
//       symmetrised over the two identical pi-;
//   Eq. (2): A_f = sum_i c_i A_i and Abar_f = sum_i cbar_i A_i;
//   Eq. (1): the time-dependent rate B(Phi, t) without CP violation;
//   Sec. 3.1: normalisation by a Monte Carlo average over uniform phase space,
//       here of B integrated over t in [0, inf) in closed form;
//   NLL = sum_data (Gamma t_i - ln B_i) + n_data ln(Nhat);
//   the NLL gradient by forward-mode dual numbers.
// The paper does not fix the lineshape, barrier, spin-factor or component
// definitions; the reading used for each is stated where it is defined.
//
// Units: GeV, ps. Metric (+,-,-,-). Event record: 4 four-momenta (E,px,py,pz)
// in the order K+, pi-(a), pi+, pi-(b); 16 doubles per event.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Scalars: double, or a dual number carrying the derivatives with respect to
// up to NG real parameters (forward-mode automatic differentiation).
// ---------------------------------------------------------------------------
constexpr int NG = 40;

struct Dual {
  double v;
  double d[NG];
};

Dual dconst(double v) {
  Dual r;
  r.v = v;
  std::memset(r.d, 0, sizeof r.d);
  return r;
}
Dual operator+(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v + b.v;
  for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
Dual operator-(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v - b.v;
  for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
Dual operator-(const Dual& a) {
  Dual r; r.v = -a.v;
  for (int i = 0; i < NG; ++i) r.d[i] = -a.d[i];
  return r;
}
Dual operator*(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v * b.v;
  for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
Dual operator/(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v / b.v;
  for (int i = 0; i < NG; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
Dual operator+(double a, const Dual& b) { return b + a; }
Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
Dual operator-(double a, const Dual& b) { return -b + a; }
Dual operator*(const Dual& a, double b) {
  Dual r; r.v = a.v * b;
  for (int i = 0; i < NG; ++i) r.d[i] = a.d[i] * b;
  return r;
}
Dual operator*(double a, const Dual& b) { return b * a; }
Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
Dual operator/(double a, const Dual& b) { return dconst(a) / b; }

// chain rule for a function f with value fv and derivative fp at a.v
Dual chain(const Dual& a, double fv, double fp) {
  Dual r; r.v = fv;
  for (int i = 0; i < NG; ++i) r.d[i] = fp * a.d[i];
  return r;
}
Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
Dual log(const Dual& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
Dual cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
Dual sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
Dual cosh(const Dual& a) { return chain(a, std::cosh(a.v), std::sinh(a.v)); }
Dual sinh(const Dual& a) { return chain(a, std::sinh(a.v), std::cosh(a.v)); }

double val(double a) { return a; }
double val(const Dual& a) { return a.v; }
using std::sqrt; using std::log; using std::cos; using std::sin; using std::cosh; using std::sinh;

template <class T> T lift(double v);
template <> double lift<double>(double v) { return v; }
template <> Dual lift<Dual>(double v) { return dconst(v); }

// ---------------------------------------------------------------------------
// Complex numbers over either scalar type.
// ---------------------------------------------------------------------------
template <class T> struct Cx { T re, im; };

template <class T> Cx<T> cx(T re, T im) { return Cx<T>{re, im}; }
template <class T> Cx<T> operator+(const Cx<T>& a, const Cx<T>& b) { return {a.re + b.re, a.im + b.im}; }
template <class T> Cx<T> operator*(const Cx<T>& a, const Cx<T>& b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> Cx<T> operator*(const Cx<T>& a, const T& b) { return {a.re * b, a.im * b}; }
template <class T> Cx<T> scale(const Cx<T>& a, double b) { return {a.re * b, a.im * b}; }
template <class T> T norm2(const Cx<T>& a) { return a.re * a.re + a.im * a.im; }
// b / a for real b and complex a
template <class T> Cx<T> real_over(const T& b, const Cx<T>& a) {
  T den = norm2(a);
  return {b * a.re / den, -(b * a.im) / den};
}

// ---------------------------------------------------------------------------
// Four-vector kinematics.
// ---------------------------------------------------------------------------
struct V4 { double t, x, y, z; };

V4 operator+(const V4& a, const V4& b) { return {a.t + b.t, a.x + b.x, a.y + b.y, a.z + b.z}; }
V4 operator-(const V4& a, const V4& b) { return {a.t - b.t, a.x - b.x, a.y - b.y, a.z - b.z}; }
V4 operator*(double s, const V4& a) { return {s * a.t, s * a.x, s * a.y, s * a.z}; }
double dot(const V4& a, const V4& b) { return a.t * b.t - a.x * b.x - a.y * b.y - a.z * b.z; }

// Two-body break-up momentum squared of a system of invariant mass squared s
// into masses ma, mb (Kallen function / 4s), clamped at zero below threshold.
template <class T> T q2_of(const T& s, double ma, double mb) {
  T r = (s - (ma + mb) * (ma + mb)) * (s - (ma - mb) * (ma - mb)) / (4.0 * s);
  if (val(r) < 0.0) return lift<T>(0.0);
  return r;
}

// Blatt-Weisskopf barrier factors without the q^L factor (the q^L dependence
// is carried by the covariant spin tensors), z = (r q)^2:
//   F_0 = 1, F_1 = (1+z)^(-1/2), F_2 = (9+3z+z^2)^(-1/2).
template <class T> T barrier(int L, const T& z) {
  if (L == 0) return lift<T>(1.0);
  if (L == 1) return 1.0 / sqrt(1.0 + z);
  return 1.0 / sqrt(9.0 + 3.0 * z + z * z);
}

// Relative momentum of u and v projected orthogonal to P: the rank-1 orbital
// tensor of the vertex P -> u v.
V4 orbital1(const V4& P, const V4& u, const V4& v) {
  V4 w = u - v;
  return w - (dot(w, P) / dot(P, P)) * P;
}
// a.b restricted to the space orthogonal to P (the spin-1 projector contracted
// with a and b).
double proj(const V4& P, const V4& a, const V4& b) {
  return dot(a, b) - dot(a, P) * dot(b, P) / dot(P, P);
}
// Rank-2 orbital tensor of ell in the rest frame of P, contracted with a, b:
//   (a.l)(b.l) - (1/3)(l.l) proj(P; a, b).
double orbital2(const V4& P, const V4& l, const V4& a, const V4& b) {
  return dot(a, l) * dot(b, l) - dot(l, l) * proj(P, a, b) / 3.0;
}
// Totally antisymmetric tensor contracted with four vectors: the determinant of
// the matrix whose rows are the contravariant components, i.e. eps_{0123} = +1.
double levi(const V4& a, const V4& b, const V4& c, const V4& d) {
  const double m[4][4] = {{a.t, a.x, a.y, a.z}, {b.t, b.x, b.y, b.z},
                          {c.t, c.x, c.y, c.z}, {d.t, d.x, d.y, d.z}};
  double det = 0.0;
  for (int j = 0; j < 4; ++j) {
    // 3x3 minor without row 0 and column j
    int cols[3], k = 0;
    for (int c2 = 0; c2 < 4; ++c2) if (c2 != j) cols[k++] = c2;
    double minor = m[1][cols[0]] * (m[2][cols[1]] * m[3][cols[2]] - m[2][cols[2]] * m[3][cols[1]])
                 - m[1][cols[1]] * (m[2][cols[0]] * m[3][cols[2]] - m[2][cols[2]] * m[3][cols[0]])
                 + m[1][cols[2]] * (m[2][cols[0]] * m[3][cols[1]] - m[2][cols[1]] * m[3][cols[0]]);
    det += ((j % 2 == 0) ? 1.0 : -1.0) * m[0][j] * minor;
  }
  return det;
}

// ---------------------------------------------------------------------------
// Model description and parameters.
// ---------------------------------------------------------------------------
}  // namespace

extern "C" {
// Fixed model constants and the membership of A_f and Abar_f. Basis index k
// (1..8): 1 K*0 rho0 S-wave, 2 K*0 rho0 P-wave, 3 K*0 rho0 D-wave,
// 4 (K+pi-)_S rho0, 5 a1 -> rho pi S-wave, 6 a1 -> rho pi D-wave,
// 7 K1(1270) -> K*0 pi+, 8 K1(1400) -> K*0 pi+.
struct orc_model {
  double m_D, m_K, m_pi;     // parent and final-state masses [GeV]
  double gamma;              // D0 width Gamma = 1/tau [1/ps]
  double r;                  // barrier radius [1/GeV], every vertex
  double m_ks_ref, m_rho_ref;  // nominal K*0, rho0 masses in the three-body q0
  double m_k1a, g_k1a;       // K1(1270)+ (fixed)
  double m_k1b, g_k1b;       // K1(1400)+ (fixed)
  int32_t n_a, n_ab;         // number of components in A_f, Abar_f
  int32_t comp_a[8];         // basis indices of A_f components
  int32_t comp_ab[8];        // basis indices of Abar_f components
  double g_bkg;              // background decay rate [1/ps]; 0: no background component
  int32_t cpv;               // 1: CP violation in mixing, q/p free (flavour-tagged data)
  double sigma_t;            // Gaussian decay-time resolution [ps]; 0: none
};
}

namespace {

// Parameter vector theta: (Re, Im) of the A_f coefficients in member order,
// then of the Abar_f coefficients, then x, y, then mass and width of K*0,
// rho0 and a1(1260), then (models with CP violation in mixing) |q/p| and
// arg(q/p), or (models with a background component) the background fraction f.
template <class T> struct Params {
  Cx<T> c[8];   // A_f coefficient of basis k (index k-1); zero if absent
  Cx<T> cb[8];  // Abar_f coefficient
  T x, y;
  T m_ks, g_ks, m_rho, g_rho, m_a1, g_a1;
  T qp_abs, qp_arg;  // q/p = |q/p| e^{i arg}; 1 and 0 without CP violation
  T f_bkg;      // zero without a background component
};

bool has_bkg(const orc_model& m) { return m.g_bkg > 0.0; }
int n_theta_of(const orc_model& m) {
  return 2 * (m.n_a + m.n_ab) + 8 + (m.cpv ? 2 : 0) + (has_bkg(m) ? 1 : 0);
}

template <class T> Params<T> unpack(const orc_model& m, const double* th, bool seed_duals);

template <> Params<double> unpack<double>(const orc_model& m, const double* th, bool) {
  Params<double> p;
  for (int k = 0; k < 8; ++k) p.c[k] = p.cb[k] = {0.0, 0.0};
  int i = 0;
  for (int j = 0; j < m.n_a; ++j, i += 2) p.c[m.comp_a[j] - 1] = {th[i], th[i + 1]};
  for (int j = 0; j < m.n_ab; ++j, i += 2) p.cb[m.comp_ab[j] - 1] = {th[i], th[i + 1]};
  p.x = th[i++]; p.y = th[i++];
  p.m_ks = th[i++]; p.g_ks = th[i++];
  p.m_rho = th[i++]; p.g_rho = th[i++];
  p.m_a1 = th[i++]; p.g_a1 = th[i++];
  p.qp_abs = 1.0; p.qp_arg = 0.0;
  if (m.cpv) { p.qp_abs = th[i++]; p.qp_arg = th[i++]; }
  p.f_bkg = has_bkg(m) ? th[i++] : 0.0;
  return p;
}

template <> Params<Dual> unpack<Dual>(const orc_model& m, const double* th, bool) {
  // parameter number i carries the unit derivative direction i
  auto var = [&](int i) { Dual d = dconst(th[i]); d.d[i] = 1.0; return d; };
  Params<Dual> p;
  for (int k = 0; k < 8; ++k) p.c[k] = p.cb[k] = {dconst(0.0), dconst(0.0)};
  int i = 0;
  for (int j = 0; j < m.n_a; ++j, i += 2) p.c[m.comp_a[j] - 1] = {var(i), var(i + 1)};
  for (int j = 0; j < m.n_ab; ++j, i += 2) p.cb[m.comp_ab[j] - 1] = {var(i), var(i + 1)};
  p.x = var(i); ++i; p.y = var(i); ++i;
  p.m_ks = var(i); ++i; p.g_ks = var(i); ++i;
  p.m_rho = var(i); ++i; p.g_rho = var(i); ++i;
  p.m_a1 = var(i); ++i; p.g_a1 = var(i); ++i;
  p.qp_abs = dconst(1.0); p.qp_arg = dconst(0.0);
  if (m.cpv) { p.qp_abs = var(i); ++i; p.qp_arg = var(i); ++i; }
  p.f_bkg = dconst(0.0);
  if (has_bkg(m)) { p.f_bkg = var(i); ++i; }
  return p;
}

// ---------------------------------------------------------------------------
// Lineshapes (Sec. 3 names "resonance lineshapes" without fixing them; the
// reading here is the relativistic Breit-Wigner with Blatt-Weisskopf barriers).
// ---------------------------------------------------------------------------

// Two-body resonance of spin 1 (K*0 -> K+ pi-, rho0 -> pi+ pi-) with a
// mass-dependent width:
//   Gamma(s) = Gamma0 (q/q0)^3 (m0/sqrt s) B'_1(q,q0)^2,
//   LS = B'_1(q,q0) / (m0^2 - s - i m0 Gamma(s)),
// where q0 is the break-up momentum at s = m0^2 and B'_L = F_L(q)/F_L(q0).
template <class T>
Cx<T> ls_two_body(double s, const T& m0, const T& g0, double ma, double mb, double r) {
  double q2 = q2_of(s, ma, mb);
  T q02 = q2_of(m0 * m0, ma, mb);
  double q = std::sqrt(q2);
  T q0 = sqrt(q02);
  T bprime = barrier(1, lift<T>(r * r * q2)) / barrier(1, r * r * q02);
  T ratio = q / q0;
  T width = g0 * ratio * ratio * ratio * (m0 / std::sqrt(s)) * bprime * bprime;
  Cx<T> den = {m0 * m0 - s, -(m0 * width)};
  return real_over(bprime, den);
}

// Resonance decaying to another resonance (mass sqrt(s_r2) in this event) and a
// pion, with constant width and orbital momentum L at its decay vertex:
//   LS_L = B'_L(q,q0) / (m0^2 - s - i m0 Gamma0),
// q from the event's sub-system mass, q0 at s = m0^2 with the sub-resonance at
// its nominal mass m_r2_ref; B'_0 = 1.
template <class T>
Cx<T> ls_three_body(int L, double s, double s_r2, double mc, const T& m0, const T& g0,
                    double m_r2_ref, double r) {
  T bprime = lift<T>(1.0);
  if (L > 0) {
    double q2 = q2_of(s, std::sqrt(s_r2), mc);
    T q02 = q2_of(m0 * m0, m_r2_ref, mc);
    bprime = barrier(L, lift<T>(r * r * q2)) / barrier(L, r * r * q02);
  }
  Cx<T> den = {m0 * m0 - s, -(m0 * g0)};
  return real_over(bprime, den);
}

// ---------------------------------------------------------------------------
// Spin factors of one Bose configuration (Sec. 3, Fig. 2), in covariant tensor
// form (the paper leaves the formalism open). sigma = 0 takes pi_s = pi-(a),
// pi_o = pi-(b); sigma = 1 swaps them.
// ---------------------------------------------------------------------------
struct Kin {
  double s_kpi;    // (K+ pi_s)^2
  double s_pipi;   // (pi+ pi_o)^2
  double s_kpipi;  // (K+ pi_s pi+)^2
  double s_3pi;    // (pi- pi+ pi-)^2, the same in both configurations
  double sf[7];    // VV S, VV P, VV D, SV, a1 S, a1 D, K1 (raw tensors)
  double qd_vv;    // D-vertex break-up momentum for D -> (K pi_s)(pi+ pi_o)
  double qd_a1;    // ... for D -> (3 pi) K+
  double qd_k1;    // ... for D -> (K pi_s pi+) pi_o
};

Kin kinematics(const V4 p[4], int sigma, double m_D, double m_K, double m_pi) {
  const V4& k = p[0];
  const V4& pip = p[2];
  const V4& ps = sigma == 0 ? p[1] : p[3];
  const V4& po = sigma == 0 ? p[3] : p[1];
  // sums that involve both pi- are formed as (p1 + p3) so that they do not
  // depend on which pi- is labelled a
  const V4 pim_pair = p[1] + p[3];
  const V4 pD = (k + pip) + pim_pair;
  const V4 three_pi = pip + pim_pair;

  Kin o;
  const V4 P1 = k + ps;     // K*0 or (K pi)_S
  const V4 P2 = pip + po;   // rho0
  const V4 PK1 = P1 + pip;  // K1+
  o.s_kpi = dot(P1, P1);
  o.s_pipi = dot(P2, P2);
  o.s_kpipi = dot(PK1, PK1);
  o.s_3pi = dot(three_pi, three_pi);

  // D -> V1 V2 and D -> S V2
  const V4 t1 = orbital1(P1, k, ps);
  const V4 t2 = orbital1(P2, pip, po);
  const V4 lD = orbital1(pD, P1, P2);
  o.sf[0] = dot(t1, t2);
  o.sf[1] = levi(lD, pD, t1, t2);
  o.sf[2] = orbital2(pD, lD, t1, t2);
  o.sf[3] = dot(lD, t2);

  // D -> a1- K+, a1- -> rho0 pi_s, rho0 -> pi+ pi_o
  {
    const V4& PA = three_pi;
    const V4 tV = orbital1(P2, pip, po);
    const V4 lDa = orbital1(pD, PA, k);
    const V4 lA = orbital1(PA, P2, ps);
    o.sf[4] = proj(PA, lDa, tV);
    o.sf[5] = orbital2(PA, lA, lDa, tV);
  }
  // D -> K1+ pi_o, K1+ -> K*0 pi+, K*0 -> K+ pi_s
  {
    const V4 tV = orbital1(P1, k, ps);
    const V4 lDk = orbital1(pD, PK1, po);
    o.sf[6] = proj(PK1, lDk, tV);
  }
  const double mD2 = m_D * m_D;
  o.qd_vv = std::sqrt(q2_of(mD2, std::sqrt(o.s_kpi), std::sqrt(o.s_pipi)));
  o.qd_a1 = std::sqrt(q2_of(mD2, std::sqrt(o.s_3pi), m_K));
  o.qd_k1 = std::sqrt(q2_of(mD2, std::sqrt(o.s_kpipi), m_pi));
  return o;
}

void read_event(const double* ev, V4 p[4]) {
  for (int i = 0; i < 4; ++i) p[i] = {ev[4 * i], ev[4 * i + 1], ev[4 * i + 2], ev[4 * i + 3]};
}

// Basis amplitudes of one Bose configuration: spin factor x D-vertex barrier x
// lineshapes of the chain.
template <class T>
void basis_sigma(const orc_model& m, const Params<T>& P, const Kin& K, Cx<T> b[8]) {
  const double r = m.r, r2 = r * r;
  const Cx<T> ks = ls_two_body(K.s_kpi, P.m_ks, P.g_ks, m.m_K, m.m_pi, r);
  const Cx<T> rho = ls_two_body(K.s_pipi, P.m_rho, P.g_rho, m.m_pi, m.m_pi, r);
  const Cx<T> a1s = ls_three_body(0, K.s_3pi, K.s_pipi, m.m_pi, P.m_a1, P.g_a1, m.m_rho_ref, r);
  const Cx<T> a1d = ls_three_body(2, K.s_3pi, K.s_pipi, m.m_pi, P.m_a1, P.g_a1, m.m_rho_ref, r);
  const Cx<T> k1a = ls_three_body(0, K.s_kpipi, K.s_kpi, m.m_pi, lift<T>(m.m_k1a),
                                  lift<T>(m.g_k1a), m.m_ks_ref, r);
  const Cx<T> k1b = ls_three_body(0, K.s_kpipi, K.s_kpi, m.m_pi, lift<T>(m.m_k1b),
                                  lift<T>(m.g_k1b), m.m_ks_ref, r);
  const double f1vv = barrier(1, r2 * K.qd_vv * K.qd_vv);
  const double f2vv = barrier(2, r2 * K.qd_vv * K.qd_vv);
  const double f1a1 = barrier(1, r2 * K.qd_a1 * K.qd_a1);
  const double f1k1 = barrier(1, r2 * K.qd_k1 * K.qd_k1);
  const Cx<T> ks_rho = ks * rho;
  b[0] = scale(ks_rho, K.sf[0]);
  b[1] = scale(ks_rho, K.sf[1] * f1vv);
  b[2] = scale(ks_rho, K.sf[2] * f2vv);
  b[3] = scale(rho, K.sf[3] * f1vv);
  b[4] = scale(a1s * rho, K.sf[4] * f1a1);
  b[5] = scale(a1d * rho, K.sf[5] * f1a1);
  b[6] = scale(k1a * ks, K.sf[6] * f1k1);
  b[7] = scale(k1b * ks, K.sf[6] * f1k1);
}

// Bose-symmetrised basis amplitudes B_k = b_k(sigma=a) + b_k(sigma=b).
template <class T>
void basis(const orc_model& m, const Params<T>& P, const double* ev, Cx<T> B[8]) {
  V4 p[4];
  read_event(ev, p);
  const Kin ka = kinematics(p, 0, m.m_D, m.m_K, m.m_pi);
  const Kin kb = kinematics(p, 1, m.m_D, m.m_K, m.m_pi);
  Cx<T> ba[8], bb[8];
  basis_sigma(m, P, ka, ba);
  basis_sigma(m, P, kb, bb);
  for (int k = 0; k < 8; ++k) B[k] = ba[k] + bb[k];
}

// Eq. (2): coherent sums over the decay chains of each amplitude.
template <class T>
void amplitudes(const orc_model& m, const Params<T>& P, const double* ev, Cx<T>& A, Cx<T>& Ab) {
  Cx<T> B[8];
  basis(m, P, ev, B);
  A = {lift<T>(0.0), lift<T>(0.0)};
  Ab = A;
  for (int j = 0; j < m.n_a; ++j) A = A + P.c[m.comp_a[j] - 1] * B[m.comp_a[j] - 1];
  for (int j = 0; j < m.n_ab; ++j) Ab = Ab + P.cb[m.comp_ab[j] - 1] * B[m.comp_ab[j] - 1];
}

// Amplitude moments entering Eq. (1): |A|^2 + |Abar|^2, |A|^2 - |Abar|^2 and
// A Abar^*.
template <class T> struct Moments { T sum, diff, re_x, im_x; };
template <class T> Moments<T> moments(const Cx<T>& A, const Cx<T>& Ab) {
  const T a2 = norm2(A), b2 = norm2(Ab);
  // A conj(Ab)
  const T re = A.re * Ab.re + A.im * Ab.im;
  const T im = A.im * Ab.re - A.re * Ab.im;
  return {a2 + b2, a2 - b2, re, im};
}

// Eq. (1): the rate divided by exp(-Gamma t) N_f, taken literally (no overall
// factor 1/2; N_f cancels in the normalisation).
template <class T>
T rate(const Moments<T>& M, const T& x, const T& y, double gamma, double t) {
  const T yt = y * (gamma * t), xt = x * (gamma * t);
  return M.sum * cosh(yt) + M.diff * cos(xt) - 2.0 * M.re_x * sinh(yt) - 2.0 * M.im_x * sin(xt);
}

// Integral over t in [0, inf) of exp(-Gamma t) times Eq. (1); the paper does
// not describe the time part of its normalisation. Uses
//   int e^{-G t} cosh(yGt) dt = 1/(G(1-y^2)),   int e^{-G t} sinh(yGt) dt = y/(G(1-y^2)),
//   int e^{-G t} cos(xGt) dt  = 1/(G(1+x^2)),   int e^{-G t} sin(xGt) dt  = x/(G(1+x^2)).
template <class T>
T rate_time_integrated(const Moments<T>& M, const T& x, const T& y, double gamma) {
  const T hy = 1.0 / (gamma * (1.0 - y * y));
  const T hx = 1.0 / (gamma * (1.0 + x * x));
  return M.sum * hy + M.diff * hx - 2.0 * M.re_x * (y * hy) - 2.0 * M.im_x * (x * hx);
}

// Eq. (1) with a Gaussian decay-time resolution of width sigma (an
// extension): the density of the measured time t is the rate e^{-Gamma t'}
// B(t') at the true time t' >= 0 convolved with the Gaussian,
//   R(t) = int_0^inf e^{-Gamma t'} B(t') exp(-(t - t')^2 / (2 sigma^2)) / (sqrt(2 pi) sigma) dt',
// integrated here by adaptive Gauss-Kronrod (7-15) quadrature over the range
// where the Gaussian exceeds e^{-98} of its peak. Over all measured times it
// integrates to the time-integrated rate, so the normalisation is unchanged.
constexpr double GK_X[8] = {0.991455371120812639, 0.949107912342758525, 0.864864423359769073,
                            0.741531185599394440, 0.586087235467691130, 0.405845151377397167,
                            0.207784955007898468, 0.0};
constexpr double GK_WK[8] = {0.022935322010529225, 0.063092092629978553, 0.104790010322250184,
                             0.140653259715525919, 0.169004726639267903, 0.190350578064785410,
                             0.204432940075298892, 0.209482141084727828};
constexpr double GK_WG[4] = {0.129484966168869693, 0.279705391489276668, 0.381830050505118945,
                             0.417959183673469388};

template <class T>
T resolved_integrand(const Moments<T>& M, const T& x, const T& y, double gamma, double sigma,
                     double t, double tp) {
  const double d = (t - tp) / sigma;
  const double gw = std::exp(-0.5 * d * d) / (2.5066282746310002 * sigma) * std::exp(-gamma * tp);
  return rate(M, x, y, gamma, tp) * gw;
}

template <class T>
void gk15(const Moments<T>& M, const T& x, const T& y, double gamma, double sigma, double t,
          double a, double b, T& kron, double& err) {
  const double c = 0.5 * (a + b), h = 0.5 * (b - a);
  T k = resolved_integrand(M, x, y, gamma, sigma, t, c) * GK_WK[7];
  double g = val(resolved_integrand(M, x, y, gamma, sigma, t, c)) * GK_WG[3];
  for (int j = 0; j < 7; ++j) {
    const T f1 = resolved_integrand(M, x, y, gamma, sigma, t, c - h * GK_X[j]);
    const T f2 = resolved_integrand(M, x, y, gamma, sigma, t, c + h * GK_X[j]);
    k = k + (f1 + f2) * GK_WK[j];
    if (j & 1) g += (val(f1) + val(f2)) * GK_WG[j / 2];
  }
  kron = k * h;
  err = std::fabs(val(kron) - g * h);
}

template <class T>
T rate_resolved(const Moments<T>& M, const T& x, const T& y, double gamma, double sigma, double t) {
  const double lo = std::max(0.0, t - 14.0 * sigma), hi = std::max(t, 0.0) + 14.0 * sigma;
  // a stack of intervals; refine until each meets its share of the tolerance
  struct Iv { double a, b; int depth; };
  std::vector<Iv> todo;
  const int n0 = 16;
  for (int i = 0; i < n0; ++i) todo.push_back({lo + (hi - lo) * i / n0, lo + (hi - lo) * (i + 1) / n0, 0});
  // total from a first pass, for the relative tolerance
  double total = 0.0;
  for (const Iv& v : todo) {
    T k;
    double e;
    gk15(M, x, y, gamma, sigma, t, v.a, v.b, k, e);
    total += std::fabs(val(k));
  }
  T sum = lift<T>(0.0);
  while (!todo.empty()) {
    const Iv v = todo.back();
    todo.pop_back();
    T k;
    double e;
    gk15(M, x, y, gamma, sigma, t, v.a, v.b, k, e);
    // |K15 - G7| bounds the 7-point rule's error; the 15-point result is
    // many orders more accurate than that on these smooth integrands
    if (e <= 1e-11 * total * (v.b - v.a) / (hi - lo) || v.depth >= 30) {
      sum = sum + k;
    } else {
      const double c = 0.5 * (v.a + v.b);
      todo.push_back({v.a, c, v.depth + 1});
      todo.push_back({c, v.b, v.depth + 1});
    }
  }
  return sum;
}

// The background's decay-time density g e^{-g t'} (t' >= 0) convolved with the
// same Gaussian, divided by g: the convolution above with the rate replaced by
// 1 (x = y = 0 and |A|^2 = 1/2 = |Abar|^2 make Eq. (1) equal to 1) and Gamma
// by g, so the same quadrature serves both.
double bkg_time_resolved(double g, double sigma, double t) {
  const Moments<double> one = {1.0, 0.0, 0.0, 0.0};
  return rate_resolved(one, 0.0, 0.0, g, sigma, t);
}

// ---------------------------------------------------------------------------
// Compensated (Neumaier) summation.
// ---------------------------------------------------------------------------
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};
template <class T> struct Acc;
template <> struct Acc<double> {
  Neumaier n;
  void add(double x) { n.add(x); }
  void add_acc(const Acc& o) { n.add(o.value()); }
  double value() const { return n.value(); }
};
template <> struct Acc<Dual> {
  Neumaier v, d[NG];
  void add(const Dual& x) { v.add(x.v); for (int i = 0; i < NG; ++i) d[i].add(x.d[i]); }
  void add_acc(const Acc& o) { add(o.value()); }
  Dual value() const {
    Dual r; r.v = v.value();
    for (int i = 0; i < NG; ++i) r.d[i] = d[i].value();
    return r;
  }
};

// Event loops run over fixed chunks so that the result does not depend on the
// number of threads.
constexpr int64_t CHUNK = 2048;

int check_params(const orc_model& m, const double* th, int n_theta) {
  if (n_theta != n_theta_of(m)) return -1;
  const Params<double> p = unpack<double>(m, th, false);
  if (!(std::fabs(p.y) < 1.0)) return -4;
  if (!(p.g_ks > 0 && p.g_rho > 0 && p.g_a1 > 0)) return -4;
  if (!(p.m_ks > m.m_K + m.m_pi)) return -4;
  if (!(p.m_rho > 2.0 * m.m_pi)) return -4;
  if (!(p.m_a1 > m.m_rho_ref + m.m_pi)) return -4;
  if (!(p.f_bkg >= 0.0 && p.f_bkg < 1.0)) return -4;
  if (!(p.qp_abs > 0.0)) return -4;
  for (int i = 0; i < n_theta; ++i) if (!std::isfinite(th[i])) return -4;
  return 0;
}

int check_model(const orc_model* m) {
  if (!m) return -1;
  if (m->n_a < 0 || m->n_a > 8 || m->n_ab < 0 || m->n_ab > 8) return -1;
  if (!(m->g_bkg >= 0.0) || !std::isfinite(m->g_bkg)) return -1;
  if (m->cpv != 0 && m->cpv != 1) return -1;
  if (!(m->sigma_t >= 0.0) || !std::isfinite(m->sigma_t)) return -1;
  if (n_theta_of(*m) > NG) return -1;
  for (int j = 0; j < m->n_a; ++j) if (m->comp_a[j] < 1 || m->comp_a[j] > 8) return -1;
  for (int j = 0; j < m->n_ab; ++j) if (m->comp_ab[j] < 1 || m->comp_ab[j] > 8) return -1;
  return 0;
}

// NLL = sum_data (Gamma t_i - ln B_i) + n_data ln(Nhat),
// Nhat = (1/n_mc) sum_mc T_j, the Monte Carlo estimate of the phase-space
// integral of the time-integrated rate (Sec. 3.1; up to the constant
// phase-space volume, which the NLL does not need).
//
// With CP violation in mixing (an extension: Eq. (1) assumes none) a D0 at
// t = 0 reaches f through g+ A_f + (q/p) g- Abar_f and a D0bar reaches the
// CP-conjugate state through g+ Abar_fbar + (p/q) g- A_fbar; with CP
// conserved in the decay amplitudes, the D0bar event taken to its CP
// conjugate has Eq. (1) with Abar_f replaced by (p/q) Abar_f. So a data event
// with flavour tag tau = +1 (D0) or -1 (D0bar, given as its CP conjugate) has
// Eq. (1) with Abar_f -> (q/p)^tau Abar_f, each flavour has its own
// normalisation Nhat_tau (the same replacement in the MC sum), and
// NLL = sum (Gamma t_i - ln B_i) + n_+ ln Nhat_+ + n_- ln Nhat_-.
//
// With a background component (an extension: the paper's study has none,
// Sec. 4) each data event's density is the mixture
//   p_i = (1 - f) B_i e^{-Gamma t_i} / Nhat + f Gamma_b e^{-Gamma_b t_i},
// the signal normalised over phase space and decay time by Nhat, the
// background uniform in phase space and exponential in time, and
// NLL = -sum_data ln p_i. With f = 0 this is the NLL above. With CP violation
// as well, each flavour's signal takes its own Nhat_tau; the background, the
// same for both flavours, has one fraction.
// (q/p)^tau for tau = +1, -1
template <class T> Cx<T> qp_power(const Params<T>& P, int tau) {
  const T r = tau > 0 ? P.qp_abs : 1.0 / P.qp_abs;
  const T a = tau > 0 ? P.qp_arg : -P.qp_arg;
  return {r * cos(a), r * sin(a)};
}

template <class T>
int nll_generic(const orc_model& m, const double* th, const double* p4d, const double* td,
                const int8_t* tag, int64_t nd, const double* p4m, int64_t nm, int nthreads, T& nll,
                double diag[4]) {
  const Params<T> P = unpack<T>(m, th, true);
  const bool cpv = m.cpv != 0;
  const Cx<T> mu_p = qp_power(P, +1), mu_m = qp_power(P, -1);
  const double G = m.gamma;
  const int64_t nchd = (nd + CHUNK - 1) / CHUNK, nchm = (nm + CHUNK - 1) / CHUNK;
  std::vector<Acc<T>> acc_d(nchd), acc_m(nchm), acc_mb(cpv ? nchm : 0);
  std::vector<double> absd(nchd, 0.0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  // normalisation: the MC estimate of the integral of the time-integrated rate
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t c = 0; c < nchm; ++c) {
    const int64_t lo = c * CHUNK, hi = std::min(nm, lo + CHUNK);
    for (int64_t i = lo; i < hi; ++i) {
      Cx<T> A, Ab;
      amplitudes(m, P, p4m + 16 * i, A, Ab);
      if (cpv) {
        acc_m[c].add(rate_time_integrated(moments(A, mu_p * Ab), P.x, P.y, G));
        acc_mb[c].add(rate_time_integrated(moments(A, mu_m * Ab), P.x, P.y, G));
      } else {
        acc_m[c].add(rate_time_integrated(moments(A, Ab), P.x, P.y, G));
      }
    }
  }
  Acc<T> sm, smb;
  for (int64_t c = 0; c < nchm; ++c) sm.add_acc(acc_m[c]);
  const T nhat = sm.value() / static_cast<double>(nm);
  if (!(val(nhat) > 0.0) || !std::isfinite(val(nhat))) return -4;
  T nhat_b = nhat;
  if (cpv) {
    for (int64_t c = 0; c < nchm; ++c) smb.add_acc(acc_mb[c]);
    nhat_b = smb.value() / static_cast<double>(nm);
    if (!(val(nhat_b) > 0.0) || !std::isfinite(val(nhat_b))) return -4;
  }
  int64_t n_minus = 0;
  if (cpv && tag)
    for (int64_t i = 0; i < nd; ++i) n_minus += tag[i] < 0 ? 1 : 0;
  const bool bkg = has_bkg(m);
  int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
#endif
  for (int64_t c = 0; c < nchd; ++c) {
    const int64_t lo = c * CHUNK, hi = std::min(nd, lo + CHUNK);
    for (int64_t i = lo; i < hi; ++i) {
      Cx<T> A, Ab;
      amplitudes(m, P, p4d + 16 * i, A, Ab);
      const bool minus = cpv && tag && tag[i] < 0;
      if (cpv) Ab = (minus ? mu_m : mu_p) * Ab;
      const T& nh = minus ? nhat_b : nhat;  // this flavour's normalisation
      const T B = m.sigma_t > 0.0 ? rate_resolved(moments(A, Ab), P.x, P.y, G, m.sigma_t, td[i])
                                  : rate(moments(A, Ab), P.x, P.y, G, td[i]);
      if (!(val(B) > 0.0) || !std::isfinite(val(B))) { ++bad; continue; }
      T l;
      if (bkg && m.sigma_t > 0.0) {
        // both extensions: B is the resolved signal density R(t) (the
        // exponential inside), the background's exponential is convolved too
        const T dens = (1.0 - P.f_bkg) * (B / nh) +
                       P.f_bkg * (m.g_bkg * bkg_time_resolved(m.g_bkg, m.sigma_t, td[i]));
        l = -log(dens);
      } else if (m.sigma_t > 0.0) {
        l = -log(B);  // B is the resolved density R(t) here
      } else if (bkg) {
        const T dens = (1.0 - P.f_bkg) * B * (std::exp(-G * td[i]) / nh) +
                       P.f_bkg * (m.g_bkg * std::exp(-m.g_bkg * td[i]));
        l = -log(dens);
      } else {
        l = G * td[i] - log(B);
      }
      acc_d[c].add(l);
      absd[c] += std::fabs(val(l));
    }
  }
  if (bad) return -4;
  Acc<T> sd;
  Neumaier sabs;
  for (int64_t c = 0; c < nchd; ++c) { sd.add_acc(acc_d[c]); sabs.add(absd[c]); }
  const T sum_l = sd.value();
  if (bkg) {
    nll = sum_l;
  } else if (cpv) {
    nll = sum_l + static_cast<double>(nd - n_minus) * log(nhat);
    if (n_minus > 0) nll = nll + static_cast<double>(n_minus) * log(nhat_b);
  } else {
    nll = sum_l + static_cast<double>(nd) * log(nhat);
  }
  diag[0] = val(nhat);
  diag[1] = val(sum_l);
  // scale of the NLL: sum of |terms|, used to judge relative agreement
  diag[2] = sabs.value() + (bkg ? 0.0
                                 : static_cast<double>(nd - n_minus) * std::fabs(std::log(val(nhat))) +
                                       static_cast<double>(n_minus) * std::fabs(std::log(val(nhat_b))));
  diag[3] = 0.0;
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Pseudo-experiments (Sec. 3.1, and the generation timing of Table 2):
// candidates uniform in four-body phase space by GENBOD (F. James, "Monte
// Carlo phase space", CERN 68-15, 1968), kept with probability proportional
// to the rate by accept-reject.
//
// Random numbers: Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror and
// D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC11), a
// counter-based generator, so that candidate i can be produced on its own.
// Candidate i of a sample with seed s takes twelve uniforms: u[2j], u[2j+1]
// from the block for counter (i mod 2^32, i div 2^32, j, stream), j = 0..5,
// key (s mod 2^32, s div 2^32); stream 0 for phase-space samples, 1 for data.
// A uniform is (k + 1/2) 2^-52 with k the top 52 bits of a 64-bit word made
// of two output words (first word high), so it lies strictly inside (0, 1).
// Use of the uniforms:
//   u0, u1   the two GENBOD intermediate masses (sorted);
//   u2       GENBOD acceptance: keep if u2 wmax < weight;
//   u3..u8   three isotropic directions (cos theta = 2u - 1, phi = 2 pi u');
//   u9, u10  decay time from exp(-G t) cosh(y G t): the rate G(1-y) when
//            u9 < (1+y)/2, else G(1+y); t = -ln(u10) / rate;
//   u11      data acceptance: keep if u11 E < B(Phi, t), E = 2 cosh(yGt) M_Phi,
//            which bounds Eq. (1) whenever M_Phi >= |A|^2 + |Abar|^2.
// ---------------------------------------------------------------------------
namespace {

// Ten rounds; each multiplies words 0 and 2 by the two Philox constants and
// mixes the high halves with words 1, 3 and the key, which advances by the
// two Weyl constants between rounds.
void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c[0];
    const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
    const uint32_t w0 = static_cast<uint32_t>(b >> 32) ^ c[1] ^ k0;
    const uint32_t w2 = static_cast<uint32_t>(a >> 32) ^ c[3] ^ k1;
    c[0] = w0;
    c[1] = static_cast<uint32_t>(b);
    c[2] = w2;
    c[3] = static_cast<uint32_t>(a);
  }
}

double uniform_of(uint32_t hi, uint32_t lo) {
  const uint64_t k = (static_cast<uint64_t>(hi) << 32 | lo) >> 12;
  return (static_cast<double>(k) + 0.5) * std::ldexp(1.0, -52);
}

void candidate_uniforms(uint64_t seed, uint64_t i, uint32_t stream, double u[12]) {
  for (uint32_t j = 0; j < 6; ++j) {
    uint32_t c[4] = {static_cast<uint32_t>(i), static_cast<uint32_t>(i >> 32), j, stream};
    philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    u[2 * j] = uniform_of(c[0], c[1]);
    u[2 * j + 1] = uniform_of(c[2], c[3]);
  }
}

// momentum of either daughter in the rest frame of a parent of mass M
double breakup(double M, double ma, double mb) {
  const double v = (M * M - (ma + mb) * (ma + mb)) * (M * M - (ma - mb) * (ma - mb));
  return v > 0.0 ? std::sqrt(v) / (2.0 * M) : 0.0;
}

// Lorentz transformation of p from the rest frame of P to the frame in which
// P has its given momentum: beta = P/E_P, gamma = E_P/M.
V4 boost_from_rest(const V4& p, const V4& P, double M) {
  const double gam = P.t / M;
  const double bx = P.x / P.t, by = P.y / P.t, bz = P.z / P.t;
  const double bp = bx * p.x + by * p.y + bz * p.z;
  const double f = gam * gam / (1.0 + gam) * bp + gam * p.t;  // (gamma-1)/beta^2 = gamma^2/(1+gamma)
  return {gam * (p.t + bp), p.x + f * bx, p.y + f * by, p.z + f * bz};
}

// the two back-to-back daughters of a decay at rest with break-up momentum q
// along the direction (cos theta = 2u - 1, phi = 2 pi v)
void split(double q, double ma, double mb, double u, double v, V4& a, V4& b) {
  const double ct = 2.0 * u - 1.0, st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  const double ph = 6.283185307179586 * v;  // 2 pi
  const double nx = st * std::cos(ph), ny = st * std::sin(ph), nz = ct;
  a = {std::sqrt(ma * ma + q * q), q * nx, q * ny, q * nz};
  b = {std::sqrt(mb * mb + q * q), -q * nx, -q * ny, -q * nz};
}

// GENBOD for M -> m0 m1 m2 m3: intermediate masses M2 (of 0 1) and M3 (of
// 0 1 2) from the sorted uniforms; weight = product of the three break-up
// momenta. If kept, the decays M -> M3 m3, M3 -> M2 m2 and M2 -> m0 m1 are
// made at rest and boosted outwards. Returns whether the candidate is kept.
bool genbod(const double u[12], double M, const double m[4], double wmax, V4 p[4]) {
  const double T = M - (m[0] + m[1] + m[2] + m[3]);
  const double rlo = std::min(u[0], u[1]), rhi = std::max(u[0], u[1]);
  const double M2 = m[0] + m[1] + rlo * T;
  const double M3 = m[0] + m[1] + m[2] + rhi * T;
  const double q2 = breakup(M2, m[0], m[1]);
  const double q3 = breakup(M3, M2, m[2]);
  const double q4 = breakup(M, M3, m[3]);
  if (!(u[2] * wmax < q2 * q3 * q4)) return false;
  V4 P01, P012;
  split(q2, m[0], m[1], u[3], u[4], p[0], p[1]);
  split(q3, M2, m[2], u[5], u[6], P01, p[2]);
  p[0] = boost_from_rest(p[0], P01, M2);
  p[1] = boost_from_rest(p[1], P01, M2);
  split(q4, M3, m[3], u[7], u[8], P012, p[3]);
  for (int j = 0; j < 3; ++j) p[j] = boost_from_rest(p[j], P012, M3);
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface (ctypes).
// Return codes: 0 ok, -1 invalid argument, -4 outside the model's domain
// (|y| >= 1, width <= 0, mass at or below threshold, B_i <= 0 or non-finite).
// ---------------------------------------------------------------------------
extern "C" {

int orc_n_theta(const orc_model* m) { return check_model(m) ? -1 : n_theta_of(*m); }

double orc_q2(double s, double ma, double mb) { return q2_of(s, ma, mb); }
double orc_barrier(int L, double z) { return barrier(L, z); }

void orc_ls_two_body(double s, double m0, double g0, double ma, double mb, double r, double* out) {
  const Cx<double> v = ls_two_body(s, m0, g0, ma, mb, r);
  out[0] = v.re; out[1] = v.im;
}
void orc_ls_three_body(int L, double s, double s_r2, double mc, double m0, double g0,
                       double m_r2_ref, double r, double* out) {
  const Cx<double> v = ls_three_body(L, s, s_r2, mc, m0, g0, m_r2_ref, r);
  out[0] = v.re; out[1] = v.im;
}

// Per configuration sigma (0, 1): out[14*sigma + 0..6] raw spin factors
// (VV S, VV P, VV D, SV, a1 S, a1 D, K1), out[14*sigma + 7..9] the D-vertex
// break-up momenta (VV, a1, K1), out[14*sigma + 10..13] the invariant masses
// squared s(K+ pi_s), s(pi+ pi_o), s(K+ pi_s pi+), s(pi- pi+ pi-).
void orc_spin_factors(const double* ev, double m_D, double m_K, double m_pi, double* out) {
  V4 p[4];
  read_event(ev, p);
  for (int sg = 0; sg < 2; ++sg) {
    const Kin k = kinematics(p, sg, m_D, m_K, m_pi);
    double* o = out + 14 * sg;
    for (int i = 0; i < 7; ++i) o[i] = k.sf[i];
    o[7] = k.qd_vv;
    o[8] = k.qd_a1;
    o[9] = k.qd_k1;
    o[10] = k.s_kpi;
    o[11] = k.s_pipi;
    o[12] = k.s_kpipi;
    o[13] = k.s_3pi;
  }
}

// Bose-symmetrised basis amplitudes B_k of one event: out[2k], out[2k+1].
int orc_basis(const orc_model* m, const double* th, int n_theta, const double* ev, double* out) {
  if (check_model(m) || n_theta != n_theta_of(*m)) return -1;
  const Params<double> P = unpack<double>(*m, th, false);
  Cx<double> B[8];
  basis(*m, P, ev, B);
  for (int k = 0; k < 8; ++k) { out[2 * k] = B[k].re; out[2 * k + 1] = B[k].im; }
  return 0;
}

// Eq. (1) and its time integral from given amplitude values.
double orc_rate(double are, double aim, double bre, double bim, double x, double y,
                double gamma, double t) {
  const Moments<double> M = moments(Cx<double>{are, aim}, Cx<double>{bre, bim});
  return rate(M, x, y, gamma, t);
}
double orc_rate_integrated(double are, double aim, double bre, double bim, double x, double y,
                           double gamma) {
  const Moments<double> M = moments(Cx<double>{are, aim}, Cx<double>{bre, bim});
  return rate_time_integrated(M, x, y, gamma);
}

// Per-event terms: out[5*i + 0..4] = |A|^2, |Abar|^2, Re(A Abar^*),
// Im(A Abar^*), and the rate: Eq. (1) at t[i] if t is given, else its time
// integral.
int orc_event_terms(const orc_model* m, const double* th, int n_theta, const double* p4,
                    const double* t, int64_t n, int nthreads, double* out) {
  if (check_model(m) || n < 0 || (n > 0 && (!p4 || !out))) return -1;
  const int rc = check_params(*m, th, n_theta);
  if (rc) return rc;
  const Params<double> P = unpack<double>(*m, th, false);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) {
    Cx<double> A, Ab;
    amplitudes(*m, P, p4 + 16 * i, A, Ab);
    const Moments<double> M = moments(A, Ab);
    out[5 * i + 0] = norm2(A);
    out[5 * i + 1] = norm2(Ab);
    out[5 * i + 2] = M.re_x;
    out[5 * i + 3] = M.im_x;
    out[5 * i + 4] = !t ? rate_time_integrated(M, P.x, P.y, m->gamma)
                     : m->sigma_t > 0.0 ? rate_resolved(M, P.x, P.y, m->gamma, m->sigma_t, t[i])
                                        : rate(M, P.x, P.y, m->gamma, t[i]);
  }
  return 0;
}

// out[0] = NLL, out[1] = Nhat, out[2] = sum over data of (Gamma t - ln B),
// out[3] = scale S = sum |Gamma t - ln B| + n_data |ln Nhat|.
int orc_nll(const orc_model* m, const double* th, int n_theta, const double* p4d,
            const double* td, int64_t nd, const double* p4m, int64_t nm, int nthreads,
            double* out) {
  if (check_model(m) || nd < 0 || nm <= 0 || !p4m || (nd > 0 && (!p4d || !td)) || !out)
    return -1;
  int rc = check_params(*m, th, n_theta);
  if (rc) { out[0] = INFINITY; return rc; }
  double nll, diag[4];
  rc = nll_generic<double>(*m, th, p4d, td, nullptr, nd, p4m, nm, nthreads, nll, diag);
  if (rc) { out[0] = INFINITY; return rc; }
  out[0] = nll; out[1] = diag[0]; out[2] = diag[1]; out[3] = diag[2];
  return 0;
}

// As orc_nll, plus grad[0..n_theta-1] = dNLL/dtheta by dual numbers.
int orc_nll_grad(const orc_model* m, const double* th, int n_theta, const double* p4d,
                 const double* td, int64_t nd, const double* p4m, int64_t nm, int nthreads,
                 double* out, double* grad) {
  if (check_model(m) || nd < 0 || nm <= 0 || !p4m || (nd > 0 && (!p4d || !td)) || !out || !grad)
    return -1;
  int rc = check_params(*m, th, n_theta);
  if (rc) { out[0] = INFINITY; return rc; }
  Dual nll;
  double diag[4];
  rc = nll_generic<Dual>(*m, th, p4d, td, nullptr, nd, p4m, nm, nthreads, nll, diag);
  if (rc) { out[0] = INFINITY; return rc; }
  out[0] = nll.v; out[1] = diag[0]; out[2] = diag[1]; out[3] = diag[2];
  for (int i = 0; i < n_theta; ++i) grad[i] = nll.d[i];
  return 0;
}

// As orc_nll / orc_nll_grad with flavour tags tag[nd] (+1 D0, -1 D0bar given
// as its CP conjugate) for models with CP violation in mixing; grad may be
// NULL.
int orc_nll_tagged(const orc_model* m, const double* th, int n_theta, const double* p4d,
                   const double* td, const int8_t* tag, int64_t nd, const double* p4m, int64_t nm,
                   int nthreads, double* out, double* grad) {
  if (check_model(m) || nd < 0 || nm <= 0 || !p4m || (nd > 0 && (!p4d || !td || !tag)) || !out)
    return -1;
  for (int64_t i = 0; i < nd; ++i) if (tag[i] != 1 && tag[i] != -1) return -1;
  int rc = check_params(*m, th, n_theta);
  if (rc) { out[0] = INFINITY; return rc; }
  double diag[4];
  if (grad) {
    Dual nll;
    rc = nll_generic<Dual>(*m, th, p4d, td, tag, nd, p4m, nm, nthreads, nll, diag);
    if (rc) { out[0] = INFINITY; return rc; }
    out[0] = nll.v;
    for (int i = 0; i < n_theta; ++i) grad[i] = nll.d[i];
  } else {
    double nll;
    rc = nll_generic<double>(*m, th, p4d, td, tag, nd, p4m, nm, nthreads, nll, diag);
    if (rc) { out[0] = INFINITY; return rc; }
    out[0] = nll;
  }
  out[1] = diag[0]; out[2] = diag[1]; out[3] = diag[2];
  return 0;
}

// One Philox4x32-10 block: ctr[4] is replaced by the output.
void orc_philox(uint32_t* ctr, uint32_t k0, uint32_t k1) { philox4x32_10(ctr, k0, k1); }

// The twelve uniforms of candidate i (see above).
void orc_candidate_uniforms(uint64_t seed, uint64_t i, uint32_t stream, double* u) {
  candidate_uniforms(seed, i, stream, u);
}

// Candidates first .. first + n_cand - 1 of a sample. kind 1: uniform phase
// space (stream 0); kind 0: data (stream 1) at theta, kept by Eq. (1) with
// the envelope M_Phi = envelope. The kept ones, in candidate order, fill
// idx/p4 [16 each]/t (t for data only) up to max_out. stats[0] = kept,
// stats[1] = kept by GENBOD, stats[2] = candidates whose rate exceeded the
// envelope (only counted for data). Returns 0, or -1 / -4 as the others.
int orc_generate(const orc_model* m, const double* th, int n_theta, int kind, uint64_t seed,
                 uint64_t first, int64_t n_cand, double wmax, double envelope, int64_t max_out,
                 int nthreads, int64_t* idx, double* p4, double* t, int64_t* stats) {
  if (check_model(m) || (kind != 0 && kind != 1) || n_cand < 0 || max_out < 0 || !stats ||
      !(wmax > 0.0) || (max_out > 0 && (!idx || !p4 || (kind == 0 && !t))))
    return -1;
  // pseudo-data follow Eq. (1) as printed: models with CP violation or a
  // background component are generated per component by the caller
  if (kind == 0 && (m->cpv || has_bkg(*m) || m->sigma_t > 0.0)) return -1;
  const bool data = kind == 0;
  Params<double> P{};
  if (data) {
    if (!(envelope > 0.0)) return -1;
    const int rc = check_params(*m, th, n_theta);
    if (rc) return rc;
    P = unpack<double>(*m, th, false);
  }
  const double mass[4] = {m->m_K, m->m_pi, m->m_pi, m->m_pi};
  const double G = m->gamma;
  std::vector<signed char> flag(static_cast<size_t>(n_cand));
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t c = 0; c < n_cand; ++c) {
    double u[12];
    V4 p[4];
    candidate_uniforms(seed, first + static_cast<uint64_t>(c), data ? 1u : 0u, u);
    signed char f = 0;
    if (genbod(u, m->m_D, mass, wmax, p)) {
      f = 1;
      if (data) {
        const double lam = u[9] < 0.5 * (1.0 + P.y) ? G * (1.0 - P.y) : G * (1.0 + P.y);
        const double tt = -std::log(u[10]) / lam;
        double ev[16];
        for (int j = 0; j < 4; ++j) {
          ev[4 * j] = p[j].t; ev[4 * j + 1] = p[j].x; ev[4 * j + 2] = p[j].y; ev[4 * j + 3] = p[j].z;
        }
        Cx<double> A, Ab;
        amplitudes(*m, P, ev, A, Ab);
        const double B = rate(moments(A, Ab), P.x, P.y, G, tt);
        const double E = 2.0 * std::cosh(P.y * G * tt) * envelope;
        if (B > E) f |= 4;
        if (u[11] * E < B) f |= 2;
      } else {
        f |= 2;
      }
    }
    flag[c] = f;
  }
  // output rank of every kept candidate, then the kept events in parallel
  std::vector<int64_t> rank(static_cast<size_t>(n_cand));
  int64_t kept = 0, ps = 0, ex = 0;
  for (int64_t c = 0; c < n_cand; ++c) {
    ps += flag[c] & 1;
    ex += (flag[c] >> 2) & 1;
    rank[c] = kept;
    kept += (flag[c] >> 1) & 1;
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t c = 0; c < n_cand; ++c) {
    if (!(flag[c] & 2) || rank[c] >= max_out) continue;
    const int64_t r = rank[c];
    double u[12];
    V4 p[4];
    const uint64_t i = first + static_cast<uint64_t>(c);
    candidate_uniforms(seed, i, data ? 1u : 0u, u);
    genbod(u, m->m_D, mass, wmax, p);
    idx[r] = static_cast<int64_t>(i);
    for (int j = 0; j < 4; ++j) {
      double* o = p4 + 16 * r + 4 * j;
      o[0] = p[j].t; o[1] = p[j].x; o[2] = p[j].y; o[3] = p[j].z;
    }
    if (data) {
      const double lam = u[9] < 0.5 * (1.0 + P.y) ? G * (1.0 - P.y) : G * (1.0 + P.y);
      t[r] = -std::log(u[10]) / lam;
    }
  }
  stats[0] = kept;
  stats[1] = ps;
  stats[2] = ex;
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
