// Host side of the mixamp C-ABI (include/mixamp.h): contexts, sample
// loading, parameter preparation, and the evaluation launches.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mixamp.h"
#include "bfgs.h"
#include "internal.h"

using namespace mxa;

namespace {

thread_local std::string g_err;

#define fail mxa::set_error

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                 \
  } while (0)

struct Sample {
  int64_t n = 0, ld = 0;
  double* c64 = nullptr;  // [NCOL][ld]
  float* c32 = nullptr;   // [NCOL][ld]
  double* t = nullptr;    // [ld], data only
};

// Events per sample are limited so that a lane's byte offset into an FP64
// column fits in 32 bits.
constexpr int64_t MAX_EVENTS = int64_t(1) << 28;
// Fixed workgroup budget of one evaluation; a function of the sample sizes
// only, so results are bitwise reproducible on any device.
constexpr int64_t TARGET_BLOCKS = 1024;
constexpr int64_t MIN_EVENTS_PER_BLOCK = 4 * BLOCK;
// Scratch of mxa_nll_grad_noalloc (an evaluation for callers that cannot
// allocate): the workgroup rows [slots][workgroups][2] and the slot totals
// [2][64] of one evaluation, sized for the largest launch -- 2 TARGET_BLOCKS
// workgroups and 45 sums (43 of the general model's adjoint plus two of a
// background component). Each device holds its own copy for the life of the
// process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (scratch_setup).
constexpr int64_t SCRATCH_ROW_WORDS = 2 * TARGET_BLOCKS * 45 * 2;
constexpr int64_t SCRATCH_WORDS = SCRATCH_ROW_WORDS + 128;
constexpr int MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) double scratch[SCRATCH_WORDS];

namespace {

std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Record the current device's address of the scratch array (once per device;
// mxa_create calls it with the context's device current).
int32_t scratch_setup(int device) {
  if (device >= MAX_DEVICES) return MXA_OK;  // mxa_nll_grad_noalloc then refuses
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return MXA_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess)
    return mxa::set_error(MXA_EDEVICE, "scratch address on device %d: %s", device, hipGetErrorString(e));
  g_scratch[device] = static_cast<double*>(ptr);
  return MXA_OK;
}

double* scratch_of(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

// Candidates per generator launch.
constexpr int64_t GEN_CHUNK_MIN = int64_t(1) << 16;
constexpr int64_t GEN_CHUNK_MAX = int64_t(1) << 24;

// Bound of the GENBOD weight q(M2; m0, m1) q(M3; M2, m2) q(M; M3, m3) for
// M -> m0 m1 m2 m3: 1.01 x its maximum over a 1001 x 1001 grid of the sorted
// uniforms (the weight is smooth, so the grid maximum is within ~1e-6 of the
// true one).
double genbod_bound(double M, const double m[4]) {
  auto q = [](double P, double a, double b) {
    const double v = (P * P - (a + b) * (a + b)) * (P * P - (a - b) * (a - b));
    return v > 0.0 ? sqrt(v) / (2.0 * P) : 0.0;
  };
  const double T = M - (m[0] + m[1] + m[2] + m[3]);
  double best = 0.0;
  for (int i = 0; i <= 1000; ++i)
    for (int j = i; j <= 1000; ++j) {
      const double M2 = m[0] + m[1] + T * (i / 1000.0), M3 = m[0] + m[1] + m[2] + T * (j / 1000.0);
      best = std::max(best, q(M2, m[0], m[1]) * q(M3, M2, m[2]) * q(M, M3, m[3]));
    }
  return 1.01 * best;
}

}  // namespace

int32_t mxa::set_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

struct mxa_ctx {
  mxa_model_desc model;
  int device = 0;
  hipStream_t stream = nullptr;
  int ma = 0, mb = 0;  // chain masks of A_f and Abar_f (bit k-1 for chain k)
  Sample s[3];  // MXA_DATA, MXA_MC, MXA_DATA_BAR
  bool have_params = false;
  int n_theta = 0;
  double theta[MAX_THETA];
  EvalParams params;      // models with CP violation: those of the D0-tagged data
  EvalParams params_bar;  // models with CP violation: those of the D0bar-tagged data
  // reduction buffers
  double* rows = nullptr;
  int64_t rows_cap = 0;
  double* d_result = nullptr;  // device address of h_result
  double* h_totals = nullptr;  // mapped, coherent pinned host memory [2][64]:
                               // the slot totals the host finalises
  double* d_host_totals = nullptr;  // device address of h_totals
  double h_gram[128] = {};     // host copy of the reduced Gram matrix
  double* h_result = nullptr;  // mapped, coherent pinned host memory
  unsigned* d_bad = nullptr;
  double* d_totals = nullptr;  // [2][64] slot totals of an evaluation
  // MC Gram matrix of the reduced chain amplitudes (MXA_MC_GRAM mode)
  int mc_mode = MXA_MC_DIRECT;
  double* d_gram = nullptr;       // [8][8][2]
  double* d_gram_rows = nullptr;  // [nb][256]
  int64_t gram_rows_cap = 0;
  bool gram_valid = false;
  int gram_precision = -1;
  double gram_shape[6];           // masses and widths the Gram was built with
  // the MC pass alternates its workgroup order between evaluations
  int32_t rev = 0;
  // sequence number of the last evaluation, written by its last kernel into
  // the result record after the slot totals
  double seq = 0.0;
  // timing
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double time_ms = 0.0;
  int64_t timed = 0;
  // pseudo-experiment scratch: per-candidate flags, per-workgroup counts and
  // offsets, and {total, last, counts[2]}
  // many-set evaluation: per-set constants, contraction matrix, rows, results
  EvalParams* d_multi_params = nullptr;  // [MAX_SETS]
  EvalParams* h_multi_params = nullptr;  // pinned staging
  void* d_multi_w = nullptr;             // [16][64 * 4] in FP64 (or FP32)
  double* h_multi_w = nullptr;           // pinned staging
  double* d_multi_rows = nullptr;
  int64_t multi_rows_cap = 0;
  double* h_multi_res = nullptr;         // mapped, [MAX_SETS][RES_WORDS]
  double* d_multi_res = nullptr;
  uint8_t* gen_flags = nullptr;
  uint32_t* gen_blocks = nullptr;
  unsigned long long* gen_misc = nullptr;
};

namespace {

int32_t check_model(const mxa_model_desc* m);

}  // namespace

int32_t mxa::check_model_desc(const mxa_model_desc* m) { return check_model(m); }

namespace {

int32_t check_model(const mxa_model_desc* m) {
  if (!m) return fail(MXA_EINVAL, "model is NULL");
  if (m->n_a < 0 || m->n_a > 8 || m->n_ab < 0 || m->n_ab > 8)
    return fail(MXA_EINVAL, "n_a and n_ab must be in 0..8");
  if (!(m->g_bkg >= 0.0) || !isfinite(m->g_bkg)) return fail(MXA_EINVAL, "g_bkg must be >= 0");
  if (m->cpv != 0 && m->cpv != 1) return fail(MXA_EINVAL, "cpv must be 0 or 1");
  if (!(m->sigma_t >= 0.0) || !isfinite(m->sigma_t)) return fail(MXA_EINVAL, "sigma_t must be >= 0");
  if (theta_count(*m) > MAX_THETA) return fail(MXA_EINVAL, "too many parameters");
  int seen_a = 0, seen_b = 0;
  for (int j = 0; j < m->n_a; ++j) {
    const int k = m->comp_a[j];
    if (k < 1 || k > 8 || (seen_a & (1 << (k - 1))))
      return fail(MXA_EINVAL, "comp_a[%d] = %d is not a distinct chain index 1..8", j, k);
    seen_a |= 1 << (k - 1);
  }
  for (int j = 0; j < m->n_ab; ++j) {
    const int k = m->comp_ab[j];
    if (k < 1 || k > 8 || (seen_b & (1 << (k - 1))))
      return fail(MXA_EINVAL, "comp_ab[%d] = %d is not a distinct chain index 1..8", j, k);
    seen_b |= 1 << (k - 1);
  }
  const double v[] = {m->m_D, m->m_K, m->m_pi, m->gamma, m->r, m->m_ks_ref, m->m_rho_ref,
                      m->m_k1a, m->g_k1a, m->m_k1b, m->g_k1b};
  for (double x : v)
    if (!(x > 0.0) || !isfinite(x)) return fail(MXA_EINVAL, "model constants must be positive");
  if (!(m->m_D > m->m_K + 3.0 * m->m_pi)) return fail(MXA_EINVAL, "m_D below the final state");
  return MXA_OK;
}

int32_t ensure(double** p, int64_t* cap, int64_t need) {
  if (*cap >= need) return MXA_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  HIP_TRY(hipMalloc(p, need * sizeof(double)));
  *cap = need;
  return MXA_OK;
}

void free_sample(Sample& s) {
  if (s.c64) (void)hipFree(s.c64);
  if (s.c32) (void)hipFree(s.c32);
  if (s.t) (void)hipFree(s.t);
  s = Sample();
}

// Two-body break-up momentum squared at s = m^2 and its derivative d/ds.
double q2_at(double s, double ma, double mb) {
  const double a = (ma + mb) * (ma + mb), b = (ma - mb) * (ma - mb);
  return (s - a) * (s - b) / (4.0 * s);
}
double dq2_ds(double s, double ma, double mb) {
  const double a = (ma + mb) * (ma + mb), b = (ma - mb) * (ma - mb);
  return (s * s - a * b) / (4.0 * s * s);
}

// Per-launch constants of a spin-1 two-body resonance with mass-dependent
// width: D = (m0^2 - s) - i K g(s), K = Gamma0 m0^2 (1 + z0) / q0^3; the
// factor sqrt(1 + z0) of B'_1 multiplies every chain containing it.
struct TwoBody {
  double m2, K, kappa;
  double dK_dm, dK_dg, dlnkappa_dm;
};
TwoBody two_body(double m0, double g0, double ma, double mb, double r) {
  TwoBody t;
  const double s0 = m0 * m0;
  const double q02 = q2_at(s0, ma, mb);
  const double z0 = r * r * q02;
  t.m2 = s0;
  t.K = g0 * s0 * (1.0 + z0) / (q02 * sqrt(q02));
  t.kappa = sqrt(1.0 + z0);
  const double dq02_dm = 2.0 * m0 * dq2_ds(s0, ma, mb);
  // d ln K / d m0 = 2/m0 + (r^2/(1+z0) - 3/(2 q0^2)) dq0^2/dm0
  t.dK_dm = t.K * (2.0 / m0 + (r * r / (1.0 + z0) - 1.5 / q02) * dq02_dm);
  t.dK_dg = t.K / g0;
  t.dlnkappa_dm = 0.5 * r * r / (1.0 + z0) * dq02_dm;
  return t;
}

}  // namespace

int mxa::theta_count(const mxa_model_desc& m) {
  return 2 * (m.n_a + m.n_ab) + 8 + (m.g_bkg > 0.0 ? 1 : 0) + (m.cpv ? 2 : 0);
}

int mxa::shape_offset(const mxa_model_desc& m) { return 2 * (m.n_a + m.n_ab) + 2; }

int32_t mxa::make_params(const mxa_model_desc& m, const double* th, EvalParams& P) {
  if (m.cpv) return fail(MXA_EINVAL, "parameters of a model with CP violation come in two sets");
  const int nc = m.n_a + m.n_ab;
  const int nt = theta_count(m);
  const double f_bkg = nt > 2 * nc + 8 ? th[2 * nc + 8] : 0.0;
  const double* coef = th;
  const double x = th[2 * nc], y = th[2 * nc + 1];
  const double m_ks = th[2 * nc + 2], g_ks = th[2 * nc + 3];
  const double m_rho = th[2 * nc + 4], g_rho = th[2 * nc + 5];
  const double m_a1 = th[2 * nc + 6], g_a1 = th[2 * nc + 7];
  for (int i = 0; i < nt; ++i)
    if (!isfinite(th[i])) return fail(MXA_EDOMAIN, "theta[%d] is not finite", i);
  if (!(f_bkg >= 0.0 && f_bkg < 1.0)) return fail(MXA_EDOMAIN, "background fraction must be in [0, 1)");
  if (!(fabs(y) < 1.0)) return fail(MXA_EDOMAIN, "|y| must be < 1 (y = %g)", y);
  if (!(g_ks > 0.0 && g_rho > 0.0 && g_a1 > 0.0)) return fail(MXA_EDOMAIN, "widths must be > 0");
  if (!(m_ks > m.m_K + m.m_pi)) return fail(MXA_EDOMAIN, "K*0 mass at or below K pi threshold");
  if (!(m_rho > 2.0 * m.m_pi)) return fail(MXA_EDOMAIN, "rho0 mass at or below pi pi threshold");
  if (!(m_a1 > m.m_rho_ref + m.m_pi)) return fail(MXA_EDOMAIN, "a1 mass at or below rho pi threshold");

  const double r = m.r;
  const TwoBody ks = two_body(m_ks, g_ks, m.m_K, m.m_pi, r);
  const TwoBody rho = two_body(m_rho, g_rho, m.m_pi, m.m_pi, r);
  // a1 D-wave: B'_2 = F_2(q) sqrt(9 + 3 z0 + z0^2), q0 at the nominal rho0 mass
  const double a1_s0 = m_a1 * m_a1;
  const double a1_q02 = q2_at(a1_s0, m.m_rho_ref, m.m_pi);
  const double a1_z0 = r * r * a1_q02;
  const double a1_f2 = sqrt(9.0 + 3.0 * a1_z0 + a1_z0 * a1_z0);
  const double a1_dz0_dm = r * r * 2.0 * m_a1 * dq2_ds(a1_s0, m.m_rho_ref, m.m_pi);
  const double a1_dlnf2_dm = 0.5 * (3.0 + 2.0 * a1_z0) / (a1_f2 * a1_f2) * a1_dz0_dm;

  // kappa_k: parameter-only factors of chain k
  double kappa[8];
  kappa[0] = kappa[1] = kappa[2] = ks.kappa * rho.kappa;
  kappa[3] = rho.kappa;
  kappa[4] = rho.kappa;
  kappa[5] = rho.kappa * a1_f2;
  kappa[6] = kappa[7] = ks.kappa;

  memset(&P, 0, sizeof P);
  FinConst& F = P.fin;
  for (int k = 0; k < 8; ++k) F.kappa[k] = kappa[k];
  F.na = m.n_a;
  F.nb = m.n_ab;
  for (int j = 0; j < m.n_a; ++j) {
    const int k = m.comp_a[j] - 1;
    F.ka[j] = k;
    F.ca[k][0] = coef[2 * j] * kappa[k];
    F.ca[k][1] = coef[2 * j + 1] * kappa[k];
  }
  for (int j = 0; j < m.n_ab; ++j) {
    const int k = m.comp_ab[j] - 1;
    F.kb[j] = k;
    F.cb[k][0] = coef[2 * (m.n_a + j)] * kappa[k];
    F.cb[k][1] = coef[2 * (m.n_a + j) + 1] * kappa[k];
  }
  F.lam_ks = ks.dlnkappa_dm;
  F.lam_rho = rho.dlnkappa_dm;
  F.lam_a1d = a1_dlnf2_dm;
  F.ks_alpha_m = 2.0 * m_ks;
  F.ks_beta_m = ks.dK_dm;
  F.ks_beta_g = ks.dK_dg;
  F.rho_alpha_m = 2.0 * m_rho;
  F.rho_beta_m = rho.dK_dm;
  F.rho_beta_g = rho.dK_dg;
  F.a1_m0 = m_a1;
  F.a1_g0 = g_a1;
  const double G = m.gamma;
  const double oy = 1.0 - y * y, ox = 1.0 + x * x;
  F.dhsum_dy = 2.0 * y / (G * oy * oy);
  F.dhre_dy = 2.0 * (1.0 + y * y) / (G * oy * oy);
  F.dhdiff_dx = -2.0 * x / (G * ox * ox);
  F.dhim_dx = 2.0 * (1.0 - x * x) / (G * ox * ox);
  F.n_theta = nt;

  LsConst<double>& L = P.ld;
  L.ks_m2 = ks.m2;
  L.ks_k = ks.K;
  L.rho_m2 = rho.m2;
  L.rho_k = rho.K;
  L.a1_m2 = a1_s0;
  L.a1_mg = m_a1 * g_a1;
  L.k1a_m2 = m.m_k1a * m.m_k1a;
  L.k1a_mg = m.m_k1a * m.g_k1a;
  L.k1b_m2 = m.m_k1b * m.m_k1b;
  L.k1b_mg = m.m_k1b * m.g_k1b;
  {
    const double ta = (m.m_K + m.m_pi) * (m.m_K + m.m_pi);
    const double tb = (m.m_K - m.m_pi) * (m.m_K - m.m_pi);
    L.ks_tsum = ta + tb;
    L.ks_tprod = ta * tb;
  }
  L.rho_tsum = 4.0 * m.m_pi * m.m_pi;
  L.rho_tprod = 0.0;
  L.r2x2 = 2.0 * r * r;
  for (int k = 0; k < 8; ++k)
    for (int q = 0; q < 2; ++q) {
      L.ca[k][q] = F.ca[k][q];
      L.cb[k][q] = F.cb[k][q];
    }
  LsConst<float>& Lf = P.lf;
  Lf.ks_m2 = static_cast<float>(L.ks_m2);
  Lf.ks_k = static_cast<float>(L.ks_k);
  Lf.rho_m2 = static_cast<float>(L.rho_m2);
  Lf.rho_k = static_cast<float>(L.rho_k);
  Lf.a1_m2 = static_cast<float>(L.a1_m2);
  Lf.a1_mg = static_cast<float>(L.a1_mg);
  Lf.k1a_m2 = static_cast<float>(L.k1a_m2);
  Lf.k1a_mg = static_cast<float>(L.k1a_mg);
  Lf.k1b_m2 = static_cast<float>(L.k1b_m2);
  Lf.k1b_mg = static_cast<float>(L.k1b_mg);
  Lf.ks_tsum = static_cast<float>(L.ks_tsum);
  Lf.ks_tprod = static_cast<float>(L.ks_tprod);
  Lf.rho_tsum = static_cast<float>(L.rho_tsum);
  Lf.rho_tprod = static_cast<float>(L.rho_tprod);
  Lf.r2x2 = static_cast<float>(L.r2x2);
  for (int k = 0; k < 8; ++k)
    for (int q = 0; q < 2; ++q) {
      Lf.ca[k][q] = static_cast<float>(L.ca[k][q]);
      Lf.cb[k][q] = static_cast<float>(L.cb[k][q]);
    }
  MixConst& X = P.mix;
  X.gamma = G;
  X.xg = x * G;
  X.yg = y * G;
  X.h_sum = 1.0 / (G * oy);
  X.h_diff = 1.0 / (G * ox);
  X.h_re = 2.0 * y / (G * oy);
  X.h_im = 2.0 * x / (G * ox);
  X.f_bkg = f_bkg;
  X.g_bkg = m.g_bkg;
  X.sigma_t = m.sigma_t;
  X.inv_nhat = 0.0;
  L.mc_hp = X.h_sum + X.h_diff;
  L.mc_hm = X.h_sum - X.h_diff;
  L.mc_hr = 0.5 * X.h_re;
  L.mc_hi = 0.5 * X.h_im;
  Lf.mc_hp = static_cast<float>(L.mc_hp);
  Lf.mc_hm = static_cast<float>(L.mc_hm);
  Lf.mc_hr = static_cast<float>(L.mc_hr);
  Lf.mc_hi = static_cast<float>(L.mc_hi);
  return MXA_OK;
}

namespace {

int32_t load_common(mxa_ctx* c, int32_t kind, const double* p4, const double* t, int64_t n,
                    bool device_src) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  if (kind != MXA_DATA && kind != MXA_MC && !(kind == MXA_DATA_BAR && c->model.cpv))
    return fail(MXA_EINVAL, "kind must be MXA_DATA or MXA_MC (or MXA_DATA_BAR for a model with CP "
                "violation)");
  const bool data = kind != MXA_MC;
  if (n < 0 || n > MAX_EVENTS) return fail(MXA_EINVAL, "n = %lld outside 0..2^28", (long long)n);
  if (n > 0 && !p4) return fail(MXA_EINVAL, "p4 is NULL");
  if (n > 0 && data && !t) return fail(MXA_EINVAL, "data events need decay times");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  Sample& s = c->s[kind];
  free_sample(s);
  if (kind == MXA_MC) c->gram_valid = false;
  if (n == 0) return MXA_OK;
  const int64_t ld = (n + 63) / 64 * 64;
  HIP_TRY(hipMalloc(&s.c64, NCOL * ld * sizeof(double)));
  HIP_TRY(hipMalloc(&s.c32, NCOL * ld * sizeof(float)));
  if (data) HIP_TRY(hipMalloc(&s.t, ld * sizeof(double)));
  s.ld = ld;
  const double* dp = p4;
  const double* dt = t;
  double* stage_p = nullptr;
  double* stage_t = nullptr;
  int32_t rc = MXA_OK;
  if (!device_src) {
    hipError_t e = hipMalloc(&stage_p, n * 16 * sizeof(double));
    if (e == hipSuccess && data) e = hipMalloc(&stage_t, n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(stage_p, p4, n * 16 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && data)
      e = hipMemcpyAsync(stage_t, t, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) rc = fail(e == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "staging: %s", hipGetErrorString(e));
    dp = stage_p;
    dt = stage_t;
  }
  unsigned h_bad = 0;
  if (rc == MXA_OK) {
    Tier0Const k;
    k.m_D = c->model.m_D;
    k.m_K = c->model.m_K;
    k.m_pi = c->model.m_pi;
    k.r = c->model.r;
    k.tol_p = 1e-6;
    k.tol_m2 = 1e-6;
    k.parity = kind == MXA_DATA_BAR ? 1 : 0;
    k.allow_neg_t = c->model.sigma_t > 0.0 ? 1 : 0;
    hipError_t e = hipMemsetAsync(c->d_bad, 0, sizeof(unsigned), c->stream);
    if (e == hipSuccess)
      e = launch_tier0(k, dp, data ? dt : nullptr, n, ld, s.c64, s.c32, s.t, c->d_bad, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, c->d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(MXA_EDEVICE, "tier-0 precompute: %s", hipGetErrorString(e));
  }
  if (stage_p) (void)hipFree(stage_p);
  if (stage_t) (void)hipFree(stage_t);
  if (rc == MXA_OK && h_bad > 0)
    rc = fail(MXA_EINVAL, "%u of %lld events fail validation (non-finite, four-momentum not "
              "conserved, off mass shell, or decay time outside [0, inf))", h_bad, (long long)n);
  if (rc != MXA_OK) free_sample(s);
  else s.n = n;
  return rc;
}

struct Shape {
  int64_t epb_d = 0, epb_m = 0;
  int32_t nb_d = 0, nb_m = 0;
};

// Waiting for an evaluation: the host watches the result record's sequence
// word (written last by the publishing kernel, after a system-scope release)
// for up to SPIN_NS, then falls back to a stream synchronisation, which also
// reports any launch error. Measured on the 50k + 4M-event evaluation: 3-4 us
// less per call than synchronising the stream at once (FP32 NLL+gradient
// 85.0 -> 81.9 us, FP32 NLL 77.2 -> 73.3 us).
constexpr int64_t SPIN_NS = 2000000;
bool wait_record(const double* rec, double seq) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    for (int i = 0; i < 256; ++i) {
      double v;
      __atomic_load(rec + 7, &v, __ATOMIC_ACQUIRE);
      if (v == seq) return true;
    }
    if (std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count() >
        SPIN_NS)
      return false;
  }
}

// Each pass is its own launch, so each fills the device on its own: up to
// TARGET_BLOCKS workgroups of at least MIN_EVENTS_PER_BLOCK (MC) or BLOCK
// (data, whose events cost about twice as much) events, equal shares.
Shape shape_for(int64_t nd, int64_t nm) {
  Shape sh;
  if (nd > 0) {
    const int64_t bd = std::min<int64_t>(TARGET_BLOCKS, (nd + BLOCK - 1) / BLOCK);
    sh.epb_d = (nd + bd - 1) / bd;
    sh.nb_d = static_cast<int32_t>((nd + sh.epb_d - 1) / sh.epb_d);
  }
  if (nm > 0) {
    const int64_t bm = std::min<int64_t>(TARGET_BLOCKS, (nm + MIN_EVENTS_PER_BLOCK - 1) / MIN_EVENTS_PER_BLOCK);
    sh.epb_m = (nm + bm - 1) / bm;
    sh.nb_m = static_cast<int32_t>((nm + sh.epb_m - 1) / sh.epb_m);
  }
  return sh;
}

const double* shape_params(const mxa_ctx* c) { return c->theta + 2 * (c->model.n_a + c->model.n_ab) + 2; }

// Build the Gram matrix of the reduced chain amplitudes over the MC sample
// for the current masses and widths.
int32_t build_gram(mxa_ctx* c, int32_t precision) {
  const Sample& M = c->s[MXA_MC];
  if (M.n == 0) return fail(MXA_EINVAL, "no MC sample loaded");
  if (!c->have_params) return fail(MXA_EINVAL, "no parameters set");
  HIP_TRY(hipSetDevice(c->device));
  GramArgs g;
  g.cache = precision == MXA_FP64 ? static_cast<const void*>(M.c64) : static_cast<const void*>(M.c32);
  g.ld = M.ld;
  g.n = M.n;
  const int64_t nb = std::min<int64_t>(256, (M.n + 4 * BLOCK - 1) / (4 * BLOCK));
  g.epb = (M.n + nb - 1) / nb;
  g.nb = static_cast<int32_t>((M.n + g.epb - 1) / g.epb);
  int32_t rc = ensure(&c->d_gram_rows, &c->gram_rows_cap, static_cast<int64_t>(g.nb) * 256);
  if (rc) return rc;
  if (!c->d_gram) HIP_TRY(hipMalloc(&c->d_gram, 128 * sizeof(double)));
  g.rows = c->d_gram_rows;
  g.out = c->d_gram;
  HIP_TRY(launch_gram(precision, c->ma, c->mb, g, c->params, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->h_gram, c->d_gram, sizeof c->h_gram, hipMemcpyDeviceToHost));
  c->gram_valid = true;
  c->gram_precision = precision;
  memcpy(c->gram_shape, shape_params(c), sizeof c->gram_shape);
  return MXA_OK;
}

// CP violation in mixing: the D0-tagged data have Eq. (1) with Abar_f ->
// (q/p) Abar_f and the D0bar-tagged data (their CP conjugates) with Abar_f ->
// (p/q) Abar_f. Abar_f enters only through its coefficients, so each flavour
// is the model without CP violation at coefficients cbar_k mu (mu = q/p or
// p/q), with its own normalisation. theta_of_mu writes that theta.
void theta_of_mu(const mxa_model_desc& m, const double* th, double mr, double mi, double* out) {
  const int nstd = 2 * (m.n_a + m.n_ab) + 8;
  memcpy(out, th, nstd * sizeof(double));
  if (m.g_bkg > 0.0) out[nstd] = th[nstd + 2];  // the background fraction follows |q/p|, arg(q/p)
  for (int j = m.n_a; j < m.n_a + m.n_ab; ++j) {
    const double a = th[2 * j], b = th[2 * j + 1];
    out[2 * j] = mr * a - mi * b;
    out[2 * j + 1] = mi * a + mr * b;
  }
}

// the two parameter sets of a model with CP violation (|q/p| = th[nstd],
// arg(q/p) = th[nstd + 1])
int32_t cpv_params(const mxa_model_desc& m, const double* th, EvalParams& Pp, EvalParams& Pm) {
  const int nstd = 2 * (m.n_a + m.n_ab) + 8;
  const double r = th[nstd], phi = th[nstd + 1];
  if (!(r > 0.0) || !isfinite(r) || !isfinite(phi))
    return fail(MXA_EDOMAIN, "|q/p| must be finite and > 0 and arg(q/p) finite");
  mxa_model_desc ms = m;
  ms.cpv = 0;
  double tp[MAX_THETA], tm[MAX_THETA];
  theta_of_mu(m, th, r * cos(phi), r * sin(phi), tp);
  theta_of_mu(m, th, cos(phi) / r, -sin(phi) / r, tm);
  const int32_t rc = make_params(ms, tp, Pp);
  return rc ? rc : make_params(ms, tm, Pm);
}

// parameters of either kind of model
int32_t params_of(const mxa_model_desc& m, const double* th, EvalParams& P, EvalParams& Pbar) {
  return m.cpv ? cpv_params(m, th, P, Pbar) : make_params(m, th, P);
}

int32_t eval_sample(mxa_ctx* c, int32_t precision, bool grad, const Sample& D, const EvalParams& P,
                    double* nll_out, double* grad_out, double* diag, bool noalloc);

// noalloc: the reduction buffers are the device's scratch array, not the
// context's (mxa_nll_grad_noalloc)
int32_t evaluate(mxa_ctx* c, int32_t precision, bool grad, double* nll_out, double* grad_out,
                 double* diag, bool noalloc = false) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  if (!c->model.cpv)
    return eval_sample(c, precision, grad, c->s[MXA_DATA], c->params, nll_out, grad_out, diag, noalloc);
  if (!nll_out || (grad && !grad_out)) return fail(MXA_EINVAL, "output pointer is NULL");
  if (!c->have_params) return fail(MXA_EINVAL, "no parameters set");
  // the two flavours, each the model without CP violation (a flavour without
  // events adds nothing); the gradient by the chain rule
  const mxa_model_desc& m = c->model;
  const int nstd = 2 * (m.n_a + m.n_ab) + 8;
  const double r = c->theta[nstd], phi = c->theta[nstd + 1];
  const Sample* S[2] = {&c->s[MXA_DATA], &c->s[MXA_DATA_BAR]};
  const EvalParams* PP[2] = {&c->params, &c->params_bar};
  const double mu[2][2] = {{r * cos(phi), r * sin(phi)}, {cos(phi) / r, -sin(phi) / r}};
  double total = 0.0, dg[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < c->n_theta && grad; ++i) grad_out[i] = 0.0;
  for (int f = 0; f < 2; ++f) {
    if (S[f]->n == 0 && !(f == 0 && S[1]->n == 0)) continue;
    double v = 0.0, g[MAX_THETA], d[4] = {0.0, 0.0, 0.0, 0.0};
    const int32_t rc = eval_sample(c, precision, grad, *S[f], *PP[f], &v, grad ? g : nullptr, d, noalloc);
    if (rc) {
      *nll_out = v;
      return rc;
    }
    total += v;
    if (f == 0) dg[0] = d[0];
    for (int q = 1; q < 4; ++q) dg[q] += d[q];
    if (!grad) continue;
    const double mr = mu[f][0], mi = mu[f][1], sg = f == 0 ? 1.0 : -1.0;
    for (int i = 0; i < nstd; ++i) {
      const int j = i / 2;
      if (j >= m.n_a && j < m.n_a + m.n_ab) continue;
      grad_out[i] += g[i];
    }
    for (int j = m.n_a; j < m.n_a + m.n_ab; ++j) {
      const double ga = g[2 * j], gb = g[2 * j + 1];
      const double a = c->theta[2 * j], b = c->theta[2 * j + 1];
      const double ap = mr * a - mi * b, bp = mi * a + mr * b;  // mu cbar
      grad_out[2 * j] += ga * mr + gb * mi;
      grad_out[2 * j + 1] += -ga * mi + gb * mr;
      // d(mu cbar)/d|q/p| = +-(mu cbar)/|q/p|, d(mu cbar)/d arg = +-i (mu cbar)
      grad_out[nstd] += sg * (ga * ap + gb * bp) / r;
      grad_out[nstd + 1] += sg * (-ga * bp + gb * ap);
    }
    if (m.g_bkg > 0.0) grad_out[nstd + 2] += g[nstd];  // one fraction for both flavours
  }
  *nll_out = total;
  if (diag)
    for (int q = 0; q < 4; ++q) diag[q] = dg[q];
  return MXA_OK;
}

// One evaluation of a model without CP violation (or one flavour of one with
// it) on the data sample D with parameters P.
int32_t eval_sample(mxa_ctx* c, int32_t precision, bool grad, const Sample& D, const EvalParams& P,
                    double* nll_out, double* grad_out, double* diag, bool noalloc) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  if (precision != MXA_FP64 && precision != MXA_FP32AMP)
    return fail(MXA_EINVAL, "precision must be MXA_FP64 or MXA_FP32AMP");
  if (!nll_out || (grad && !grad_out)) return fail(MXA_EINVAL, "output pointer is NULL");
  if (!c->have_params) return fail(MXA_EINVAL, "no parameters set");
  const Sample& M = c->s[MXA_MC];
  if (M.n == 0) return fail(MXA_EINVAL, "no MC sample loaded");
  HIP_TRY(hipSetDevice(c->device));
  const bool use_gram = c->mc_mode == MXA_MC_GRAM;
  const bool bkg = c->model.g_bkg > 0.0;
  if (noalloc && use_gram)
    return fail(MXA_EINVAL, "the evaluation without allocation needs the direct MC mode");
  if (use_gram && (!c->gram_valid || c->gram_precision != precision ||
                   memcmp(c->gram_shape, shape_params(c), sizeof c->gram_shape) != 0)) {
    const int32_t rc = build_gram(c, precision);
    if (rc) return rc;
  }
  const Shape sh = shape_for(D.n, use_gram ? 0 : M.n);
  const int ns = slots_for(grad, c->ma, c->mb) + (bkg && grad ? 2 : 0);
  const int64_t nrows = static_cast<int64_t>(sh.nb_d) + sh.nb_m;
  double* rows = nullptr;
  double* totals = nullptr;
  if (noalloc) {
    double* base = scratch_of(c->device);
    if (!base) return fail(MXA_EDEVICE, "no scratch array on device %d", c->device);
    if (nrows * ns * 2 > SCRATCH_ROW_WORDS)
      return fail(MXA_EINVAL, "evaluation needs %lld scratch words, the maximum is %lld",
                  static_cast<long long>(nrows * ns * 2), static_cast<long long>(SCRATCH_ROW_WORDS));
    rows = base;
    totals = base + SCRATCH_ROW_WORDS;
  } else {
    const int32_t rc = ensure(&c->rows, &c->rows_cap, nrows * ns * 2);
    if (rc) return rc;
    rows = c->rows;
    totals = c->d_totals;
  }
  EvalArgs a;
  memset(&a, 0, sizeof a);
  const bool f64 = precision == MXA_FP64;
  a.cache_d = f64 ? static_cast<const void*>(D.c64) : static_cast<const void*>(D.c32);
  a.t_d = D.t;
  a.cache_m = f64 ? static_cast<const void*>(M.c64) : static_cast<const void*>(M.c32);
  a.ld_d = D.ld;
  a.ld_m = M.ld;
  a.n_d = D.n;
  a.n_m = M.n;
  a.epb_d = sh.epb_d;
  a.epb_m = sh.epb_m;
  a.nb_d = sh.nb_d;
  a.nb_m = sh.nb_m;
  a.rows = rows;
  a.totals = totals;
  a.result = c->d_result;
  a.host_totals = c->d_host_totals;
  a.rev = c->rev;
  c->rev ^= 1;
  if (bkg && use_gram) {
    // the data pass needs Nhat before it runs: from the Gram matrix, here
    const double sum_t = gram_sum_t(c->ma, c->mb, P, c->h_gram);
    if (!(sum_t > 0.0) || !isfinite(sum_t)) {
      *nll_out = INFINITY;
      return fail(MXA_EDOMAIN, "Nhat = %g from the Gram matrix", sum_t / static_cast<double>(M.n));
    }
    a.inv_nhat = static_cast<double>(M.n) / sum_t;
  }
  const bool watch = SPIN_NS > 0 && !c->timing;
  if (watch) {
    c->seq += 1.0;
    a.seq = c->seq;
  }
  HIP_TRY(launch_eval(precision, grad, c->ma, c->mb, a, P, c->stream,
                      c->timing ? c->ev0 : nullptr, c->timing ? c->ev1 : nullptr));
  if (!watch || !wait_record(c->h_result, c->seq)) HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->timing) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->time_ms += ms;
    c->timed += 1;
  }
  {
    // the NLL and gradient from the published totals, into the record
    double Dt[64], Mt[64];
    memcpy(Dt, c->h_totals, sizeof Dt);
    memcpy(Mt, c->h_totals + 64, sizeof Mt);
    EvalArgs h = a;
    h.result = c->h_result;
    finalize_host(c->ma, c->mb, grad, h, P, Dt, Mt, use_gram ? c->h_gram : nullptr);
  }
  const double* r = c->h_result;
  *nll_out = r[0];
  if (diag) {
    diag[0] = r[1];
    diag[1] = r[2];
    diag[2] = r[3];
    diag[3] = r[4];
  }
  if (grad)
    for (int i = 0; i < P.fin.n_theta; ++i) grad_out[i] = r[8 + i];
  if (r[6] != 0.0) {
    *nll_out = INFINITY;
    return fail(MXA_EDOMAIN, "rate not positive: %g data events with B <= 0 or non-finite, Nhat = %g",
                r[4], r[1]);
  }
  return MXA_OK;
}

}  // namespace

extern "C" {

int32_t mxa_n_theta(const mxa_model_desc* model) {
  const int32_t rc = check_model(model);
  return rc ? rc : theta_count(*model);
}

int32_t mxa_create(const mxa_model_desc* model, int32_t device, void* stream, mxa_ctx** out) {
  if (!out) return fail(MXA_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t rc = check_model(model);
  if (rc) return rc;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(MXA_EDEVICE, "no HIP device available");
  if (device < 0 || device >= count) return fail(MXA_EDEVICE, "device %d not in 0..%d", device, count - 1);
  HIP_TRY(hipSetDevice(device));
  rc = scratch_setup(device);
  if (rc) return rc;
  mxa_ctx* c = new (std::nothrow) mxa_ctx();
  if (!c) return fail(MXA_ENOMEM, "host allocation failed");
  c->model = *model;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  for (int j = 0; j < model->n_a; ++j) c->ma |= 1 << (model->comp_a[j] - 1);
  for (int j = 0; j < model->n_ab; ++j) c->mb |= 1 << (model->comp_ab[j] - 1);
  c->n_theta = theta_count(*model);
  // the last kernel writes the slot totals and the sequence word straight
  // into mapped, coherent pinned host memory: no device-to-host copy per
  // evaluation
  hipError_t e = hipHostMalloc(&c->h_result, RES_WORDS * sizeof(double),
                               hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&c->d_result), c->h_result, 0);
  if (e == hipSuccess) memset(c->h_result, 0, RES_WORDS * sizeof(double));
  if (e == hipSuccess)
    e = hipHostMalloc(&c->h_totals, 128 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&c->d_host_totals), c->h_totals, 0);
  if (e == hipSuccess) e = hipMalloc(&c->d_bad, sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(&c->d_totals, 128 * sizeof(double));
  if (e == hipSuccess) e = hipEventCreate(&c->ev0);
  if (e == hipSuccess) e = hipEventCreate(&c->ev1);
  if (e != hipSuccess) {
    mxa_destroy(c);
    return fail(e == hipErrorOutOfMemory ? MXA_ENOMEM : MXA_EDEVICE, "context setup: %s", hipGetErrorString(e));
  }
  *out = c;
  return MXA_OK;
}

int32_t mxa_destroy(mxa_ctx* c) {
  if (!c) return MXA_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_sample(c->s[0]);
  free_sample(c->s[1]);
  free_sample(c->s[2]);
  if (c->rows) (void)hipFree(c->rows);
  if (c->d_gram) (void)hipFree(c->d_gram);
  if (c->d_gram_rows) (void)hipFree(c->d_gram_rows);
  if (c->h_result) (void)hipHostFree(c->h_result);
  if (c->h_totals) (void)hipHostFree(c->h_totals);
  if (c->d_bad) (void)hipFree(c->d_bad);
  if (c->d_totals) (void)hipFree(c->d_totals);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->d_multi_params) (void)hipFree(c->d_multi_params);
  if (c->h_multi_params) (void)hipHostFree(c->h_multi_params);
  if (c->d_multi_w) (void)hipFree(c->d_multi_w);
  if (c->h_multi_w) (void)hipHostFree(c->h_multi_w);
  if (c->d_multi_rows) (void)hipFree(c->d_multi_rows);
  if (c->h_multi_res) (void)hipHostFree(c->h_multi_res);
  if (c->gen_flags) (void)hipFree(c->gen_flags);
  if (c->gen_blocks) (void)hipFree(c->gen_blocks);
  if (c->gen_misc) (void)hipFree(c->gen_misc);
  delete c;
  return MXA_OK;
}

int32_t mxa_load_events(mxa_ctx* c, int32_t kind, const double* p4, const double* t, int64_t n) {
  return load_common(c, kind, p4, t, n, false);
}

int32_t mxa_load_events_device(mxa_ctx* c, int32_t kind, const double* d_p4, const double* d_t,
                               int64_t n) {
  return load_common(c, kind, d_p4, d_t, n, true);
}

int32_t mxa_sample_size(mxa_ctx* c, int32_t kind, int64_t* n) {
  if (!c || !n) return fail(MXA_EINVAL, "NULL argument");
  if (kind != MXA_DATA && kind != MXA_MC && kind != MXA_DATA_BAR) return fail(MXA_EINVAL, "bad kind");
  *n = c->s[kind].n;
  return MXA_OK;
}

int32_t mxa_set_params(mxa_ctx* c, const double* theta, int32_t n_theta) {
  if (!c || !theta) return fail(MXA_EINVAL, "NULL argument");
  if (n_theta != c->n_theta) return fail(MXA_EINVAL, "n_theta = %d, model needs %d", n_theta, c->n_theta);
  c->have_params = false;
  const int32_t rc = params_of(c->model, theta, c->params, c->params_bar);
  if (rc) return rc;
  memcpy(c->theta, theta, n_theta * sizeof(double));
  c->have_params = true;
  return MXA_OK;
}

int32_t mxa_nll(mxa_ctx* c, int32_t precision, double* nll_out, double* diag) {
  return evaluate(c, precision, false, nll_out, nullptr, diag);
}

int32_t mxa_nll_grad(mxa_ctx* c, int32_t precision, double* nll_out, double* grad_out, double* diag) {
  return evaluate(c, precision, true, nll_out, grad_out, diag);
}

int32_t mxa_nll_grad_noalloc(mxa_ctx* c, int32_t precision, double* nll_out, double* grad_out,
                             double* diag) {
  return evaluate(c, precision, true, nll_out, grad_out, diag, true);
}

}  // extern "C"

namespace {

// NLL and the gradient of the free parameters idx by central differences with
// steps h (the rest of g left 0) at th: in Gram mode, with no free mass or
// width and 2 n + 1 <= MXA_MAX_SETS, one many-set call; otherwise one
// evaluation per point. A point outside the model's domain gives +inf.
int32_t central_grad(mxa_ctx* c, int32_t precision, const double* th, const std::vector<int>& idx,
                     const std::vector<double>& h, double* f, double* g) {
  const int nt = c->n_theta, nf = static_cast<int>(idx.size()), np = 2 * nf + 1;
  const int nstd = 2 * (c->model.n_a + c->model.n_ab) + 2;  // coefficients, x, y
  bool shapes_fixed = true;
  for (int i : idx) shapes_fixed = shapes_fixed && i < nstd;
  std::vector<double> pts(static_cast<size_t>(np) * nt), v(np, INFINITY);
  for (int p = 0; p < np; ++p) {
    double* q = pts.data() + static_cast<size_t>(p) * nt;
    memcpy(q, th, nt * sizeof(double));
    if (p > 0) q[idx[(p - 1) / 2]] += ((p - 1) % 2 == 0 ? 1.0 : -1.0) * h[(p - 1) / 2];
  }
  int32_t rc = MXA_OK;
  if (c->mc_mode == MXA_MC_GRAM && shapes_fixed && np <= MAX_SETS && !c->model.cpv &&
      !(c->model.g_bkg > 0.0)) {
    rc = mxa_nll_multi(c, precision, pts.data(), np, v.data());
    if (rc == MXA_EDOMAIN) rc = MXA_OK;  // every point outside: all +inf
  } else {
    for (int p = 0; p < np && rc == MXA_OK; ++p) {
      rc = mxa_set_params(c, pts.data() + static_cast<size_t>(p) * nt, nt);
      if (rc == MXA_OK) rc = evaluate(c, precision, false, &v[p], nullptr, nullptr);
      if (rc == MXA_EDOMAIN) {
        v[p] = INFINITY;
        rc = MXA_OK;
      }
    }
  }
  if (rc) return rc;
  *f = v[0];
  for (int a = 0; a < nf; ++a) g[idx[a]] = (v[1 + 2 * a] - v[2 + 2 * a]) / (2.0 * h[a]);
  return MXA_OK;
}

}  // namespace

extern "C" {

int32_t mxa_fit(mxa_ctx* c, int32_t precision, const mxa_fit_request* req, mxa_fit_result* out) {
  if (!c || !req || !out || !req->theta0 || !req->scale) return fail(MXA_EINVAL, "NULL argument");
  const bool central = req->gradient == MXA_GRAD_CENTRAL;
  if (req->gradient != MXA_GRAD_ADJOINT && !central)
    return fail(MXA_EINVAL, "gradient must be MXA_GRAD_ADJOINT or MXA_GRAD_CENTRAL");
  if (central && precision != MXA_FP64)
    return fail(MXA_EINVAL, "central differences need MXA_FP64 (FP32 amplitude rounding is "
                "larger than the NLL's change over a step)");
  const auto clock_ns = [] {
    return static_cast<int64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                    std::chrono::steady_clock::now().time_since_epoch())
                                    .count());
  };
  const int64_t t0 = clock_ns();
  const int nt = c->n_theta;
  std::vector<int> idx;
  std::vector<double> sc;
  for (int i = 0; i < nt; ++i) {
    const double v = req->scale[i];
    if (!(v >= 0.0) || !isfinite(v)) return fail(MXA_EINVAL, "scale[%d] = %g", i, v);
    if (v > 0.0) {
      idx.push_back(i);
      sc.push_back(v);
    }
  }
  if (idx.empty()) return fail(MXA_EINVAL, "no free parameter (all scales are 0)");
  EvalParams probe, probe_bar;
  int32_t rc = params_of(c->model, req->theta0, probe, probe_bar);
  if (rc) return rc;
  Bfgs b;
  b.init(req->theta0, nt, idx.data(), sc.data(), static_cast<int>(idx.size()),
         req->max_evals > 0 ? req->max_evals : 150, req->gtol > 0 ? req->gtol : 1e-3, req->ftol,
         req->edm_tol > 0 ? req->edm_tol : 0.0, req->errors != 0);
  std::vector<double> g(nt, 0.0), h(sc.size());
  for (size_t a = 0; a < sc.size(); ++a) h[a] = 1e-4 * sc[a];
  int64_t points = 0;
  while (b.status() == Bfgs::RUNNING) {
    // a trial point outside the model's domain, or with a non-positive rate,
    // is reported to the minimiser as +inf (its line search then shortens
    // the step)
    double f = INFINITY;
    rc = mxa_set_params(c, b.point(), nt);
    if (rc == MXA_OK && central) {
      rc = central_grad(c, precision, b.point(), idx, h, &f, g.data());
      points += 2 * static_cast<int64_t>(idx.size()) + 1;
    } else if (rc == MXA_OK) {
      rc = evaluate(c, precision, true, &f, g.data(), nullptr);
      points += 1;
    }
    if (rc == MXA_EDOMAIN) {
      f = INFINITY;
    } else if (rc != MXA_OK) {
      return rc;
    }
    b.tell(f, g.data());
  }
  memset(out, 0, sizeof *out);
  b.best(out->theta);
  out->nll = b.best_f();
  out->grad_norm = b.grad_norm();
  out->n_evals = b.evals();
  out->status = b.status() == Bfgs::CONVERGED   ? MXA_FIT_CONVERGED
                : b.status() == Bfgs::MAX_EVALS ? MXA_FIT_MAX_EVALS
                                                : MXA_FIT_FAILED;
  out->n = c->s[MXA_DATA].n;
  out->t_submit_ns = out->t_start_ns = t0;
  if (b.errors_ok()) {
    out->errors_ok = 1;
    for (int i = 0; i < b.n_free(); ++i) out->err[b.free_index(i)] = b.errors()[i];
  }
  for (int i = 0; i < nt; ++i) out->grad[i] = b.best_grad()[i];
  out->n_points = points;
  rc = mxa_set_params(c, out->theta, nt);
  out->t_done_ns = clock_ns();
  return rc;
}

int32_t mxa_event_terms(mxa_ctx* c, int32_t kind, int32_t precision, double* out) {
  if (!c || !out) return fail(MXA_EINVAL, "NULL argument");
  if (kind != MXA_DATA && kind != MXA_MC && !(kind == MXA_DATA_BAR && c->model.cpv))
    return fail(MXA_EINVAL, "bad kind");
  if (precision != MXA_FP64 && precision != MXA_FP32AMP) return fail(MXA_EINVAL, "bad precision");
  if (!c->have_params) return fail(MXA_EINVAL, "no parameters set");
  const Sample& s = c->s[kind];
  if (s.n == 0) return MXA_OK;
  HIP_TRY(hipSetDevice(c->device));
  double* d_out = nullptr;
  HIP_TRY(hipMalloc(&d_out, s.n * 5 * sizeof(double)));
  TermsArgs a;
  a.cache = precision == MXA_FP64 ? static_cast<const void*>(s.c64) : static_cast<const void*>(s.c32);
  a.t = kind != MXA_MC ? s.t : nullptr;
  a.ld = s.ld;
  a.n = s.n;
  a.out = d_out;
  hipError_t e = launch_terms(precision, c->ma, c->mb, a,
                              kind == MXA_DATA_BAR ? c->params_bar : c->params, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, s.n * 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d_out);
  if (e != hipSuccess) return fail(MXA_EDEVICE, "event terms: %s", hipGetErrorString(e));
  return MXA_OK;
}

int32_t mxa_gram(mxa_ctx* c, int32_t precision, double* out) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  if (precision != MXA_FP64 && precision != MXA_FP32AMP) return fail(MXA_EINVAL, "bad precision");
  int32_t rc = build_gram(c, precision);
  if (rc || !out) return rc;
  double g[128];
  HIP_TRY(hipMemcpy(g, c->d_gram, sizeof g, hipMemcpyDeviceToHost));
  // chain amplitudes B_k = kappa_k beta_k
  const double* kap = c->params.fin.kappa;
  for (int k = 0; k < 8; ++k)
    for (int l = 0; l < 8; ++l)
      for (int q = 0; q < 2; ++q) out[(k * 8 + l) * 2 + q] = g[(k * 8 + l) * 2 + q] * kap[k] * kap[l];
  return MXA_OK;
}

int32_t mxa_generate(mxa_ctx* c, int32_t kind, uint64_t seed, uint64_t first, int64_t n,
                     double wmax, double envelope, double* d_p4, double* d_t, int64_t* d_idx,
                     mxa_gen_stats* stats) {
  if (!c || !stats) return fail(MXA_EINVAL, "NULL argument");
  memset(stats, 0, sizeof *stats);
  stats->next = first;
  if (kind != MXA_DATA && kind != MXA_MC) return fail(MXA_EINVAL, "kind must be MXA_DATA or MXA_MC");
  const bool data = kind == MXA_DATA;
  if (data && (c->model.cpv || c->model.g_bkg > 0.0 || c->model.sigma_t > 0.0))
    return fail(MXA_EINVAL, "pseudo-data follow Eq. (1): generate each component with the model "
                "without CP violation, background or resolution (and smear the times)");
  if (n < 0 || n > MAX_EVENTS) return fail(MXA_EINVAL, "n = %lld out of range", (long long)n);
  if (!(wmax >= 0.0) || !isfinite(wmax)) return fail(MXA_EINVAL, "wmax must be finite and >= 0");
  if (data && (!(envelope > 0.0) || !isfinite(envelope)))
    return fail(MXA_EINVAL, "the envelope must be finite and positive");
  if (data && !c->have_params) return fail(MXA_EINVAL, "no parameters set");
  if (n > 0 && (!d_p4 || (data && !d_t))) return fail(MXA_EINVAL, "output pointer is NULL");
  if (n == 0) return MXA_OK;
  const mxa_model_desc& md = c->model;
  const double mass[4] = {md.m_K, md.m_pi, md.m_pi, md.m_pi};
  if (wmax == 0.0) wmax = genbod_bound(md.m_D, mass);
  HIP_TRY(hipSetDevice(c->device));
  if (!c->gen_flags) HIP_TRY(hipMalloc(&c->gen_flags, GEN_CHUNK_MAX));
  if (!c->gen_blocks) HIP_TRY(hipMalloc(&c->gen_blocks, 2 * (GEN_CHUNK_MAX / BLOCK) * sizeof(uint32_t)));
  if (!c->gen_misc) HIP_TRY(hipMalloc(&c->gen_misc, 8 * sizeof(unsigned long long)));
  GenArgs a;
  memset(&a, 0, sizeof a);
  a.g.key0 = static_cast<uint32_t>(seed);
  a.g.key1 = static_cast<uint32_t>(seed >> 32);
  a.g.stream = data ? 1u : 0u;
  a.g.M = md.m_D;
  for (int j = 0; j < 4; ++j) a.g.m[j] = mass[j];
  a.g.wmax = wmax;
  a.g.envelope = envelope;
  a.g.gamma = md.gamma;
  a.g.y = data ? c->theta[2 * (md.n_a + md.n_ab) + 1] : 0.0;
  a.g.t0.m_D = md.m_D;
  a.g.t0.m_K = md.m_K;
  a.g.t0.m_pi = md.m_pi;
  a.g.t0.r = md.r;
  a.flags = c->gen_flags;
  a.bcount = c->gen_blocks;
  a.boff = c->gen_blocks + GEN_CHUNK_MAX / BLOCK;
  unsigned long long* misc = c->gen_misc;
  a.total = reinterpret_cast<uint32_t*>(misc);
  a.last = reinterpret_cast<int64_t*>(misc + 1);
  a.counts = misc + 2;
  a.p4 = d_p4;
  a.t = data ? d_t : nullptr;
  a.idx = d_idx;
  a.n_out = n;
  const int64_t max_cand = GEN_CHUNK_MAX + (int64_t(1) << 17) * n;
  int64_t filled = 0, n_cand = 0, n_ps = 0, n_ex = 0;
  uint64_t cand = first;
  while (filled < n) {
    const int64_t need = n - filled;
    // chunk from the acceptance so far (a first guess before any)
    const double rate = n_cand > 0 ? std::max(1e-6, double(filled) / double(n_cand)) : (data ? 0.01 : 0.5);
    int64_t ch = static_cast<int64_t>(std::min(1.1 * double(need) / rate, double(GEN_CHUNK_MAX))) + BLOCK;
    ch = std::min<int64_t>(std::max<int64_t>(ch, GEN_CHUNK_MIN), GEN_CHUNK_MAX) / BLOCK * BLOCK;
    if (n_cand >= max_cand)
      return fail(MXA_EDOMAIN, "%lld of %lld candidates kept: acceptance too low", (long long)filled,
                  (long long)n_cand);
    if (cand + static_cast<uint64_t>(ch) < cand) return fail(MXA_EINVAL, "candidate index overflow");
    a.g.first = cand;
    a.g.n = ch;
    a.filled = filled;
    unsigned long long h[4];
    HIP_TRY(hipMemsetAsync(misc, 0, 4 * sizeof(unsigned long long), c->stream));
    HIP_TRY(launch_gen_chunk(data, c->ma, c->mb, a, c->params, c->stream));
    HIP_TRY(hipMemcpyAsync(h, misc, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int64_t total = static_cast<int64_t>(static_cast<uint32_t>(h[0]));
    const int64_t last = static_cast<int64_t>(h[1]);
    const int64_t take = std::min(total, need);
    const int64_t limit = total >= need ? last + 1 : ch;
    HIP_TRY(launch_gen_stats(a, limit, c->stream));
    HIP_TRY(hipMemcpyAsync(h + 2, misc + 2, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    n_ps += static_cast<int64_t>(h[2]);
    n_ex += static_cast<int64_t>(h[3]);
    filled += take;
    n_cand += limit;
    cand += static_cast<uint64_t>(limit);
  }
  stats->n_candidates = n_cand;
  stats->n_phase_space = n_ps;
  stats->n_exceed = n_ex;
  stats->next = cand;
  return MXA_OK;
}

int32_t mxa_nll_multi(mxa_ctx* c, int32_t precision, const double* thetas, int32_t n_sets,
                      double* nll_out) {
  if (!c || !thetas || !nll_out) return fail(MXA_EINVAL, "NULL argument");
  if (precision != MXA_FP64 && precision != MXA_FP32AMP) return fail(MXA_EINVAL, "bad precision");
  if (n_sets < 1 || n_sets > MXA_MAX_SETS)
    return fail(MXA_EINVAL, "n_sets must be in 1..%d", MXA_MAX_SETS);
  if (c->model.cpv) return fail(MXA_EINVAL, "many parameter sets: models with CP violation are not supported");
  const Sample& D = c->s[MXA_DATA];
  const Sample& M = c->s[MXA_MC];
  if (M.n == 0) return fail(MXA_EINVAL, "no MC sample loaded");
  const int nt = c->n_theta;
  const int sh0 = shape_offset(c->model);
  for (int s = 1; s < n_sets; ++s)
    if (memcmp(thetas + static_cast<int64_t>(s) * nt + sh0, thetas + sh0, 6 * sizeof(double)))
      return fail(MXA_EINVAL, "set %d has other masses or widths than set 0", s);
  HIP_TRY(hipSetDevice(c->device));
  if (!c->d_multi_params) {
    HIP_TRY(hipMalloc(&c->d_multi_params, MXA_MAX_SETS * sizeof(EvalParams)));
    HIP_TRY(hipHostMalloc(&c->h_multi_params, MXA_MAX_SETS * sizeof(EvalParams), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&c->d_multi_w, 16 * 4 * 64 * sizeof(double)));
    HIP_TRY(hipHostMalloc(&c->h_multi_w, 16 * 4 * 64 * sizeof(double), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&c->h_multi_res, MXA_MAX_SETS * RES_WORDS * sizeof(double),
                          hipHostMallocMapped | hipHostMallocCoherent));
    HIP_TRY(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->d_multi_res), c->h_multi_res, 0));
  }
  // per-set constants; a set outside the model's domain takes a valid set's
  // constants (its result is replaced by +inf)
  EvalParams* P = c->h_multi_params;
  std::vector<char> ok(n_sets, 0);
  int first = -1;
  for (int s = 0; s < n_sets; ++s) {
    ok[s] = make_params(c->model, thetas + static_cast<int64_t>(s) * nt, P[s]) == MXA_OK;
    if (ok[s] && first < 0) first = s;
  }
  if (first < 0) return fail(MXA_EDOMAIN, "no parameter set inside the model's domain");
  for (int s = 0; s < n_sets; ++s)
    if (!ok[s]) P[s] = P[first];
  // the Gram matrix is taken at the first valid set's lineshapes
  memcpy(c->theta, thetas + static_cast<int64_t>(first) * nt, nt * sizeof(double));
  c->params = P[first];
  c->have_params = true;
  if (!c->gram_valid || c->gram_precision != precision ||
      memcmp(c->gram_shape, shape_params(c), sizeof c->gram_shape) != 0) {
    const int32_t rc = build_gram(c, precision);
    if (rc) return rc;
  }
  // with a background component each set's data term needs its Nhat: from
  // the Gram matrix, here (a set whose Nhat is not positive counts as outside
  // the domain)
  if (c->model.g_bkg > 0.0)
    for (int s = 0; s < n_sets; ++s) {
      if (!ok[s]) continue;
      const double sum_t = gram_sum_t(c->ma, c->mb, P[s], c->h_gram);
      if (sum_t > 0.0 && isfinite(sum_t)) {
        P[s].mix.inv_nhat = static_cast<double>(M.n) / sum_t;
      } else {
        ok[s] = 0;
        P[s] = P[first];
      }
    }
  // contraction matrix W[16][ldw]: column 64 (s / 16) + 4 (s mod 16) + {0, 1,
  // 2, 3} gives Re A, Im A, Re Abar, Im Abar of set s from the 16 reals
  // (Re B_k, Im B_k), with the precision's own coefficient values
  const bool f64 = precision == MXA_FP64;
  const int n_chunks = (n_sets + 15) / 16;
  const int ldw = 64 * n_chunks;
  double* w64 = c->h_multi_w;
  float* w32 = reinterpret_cast<float*>(c->h_multi_w);
  for (int i = 0; i < 16 * ldw; ++i) {
    if (f64) w64[i] = 0.0;
    else w32[i] = 0.0f;
  }
  for (int s = 0; s < n_sets; ++s) {
    if (!ok[s]) continue;
    const int col = 64 * (s / 16) + 4 * (s % 16);
    for (int k = 0; k < 8; ++k) {
      const double ar = f64 ? P[s].ld.ca[k][0] : P[s].lf.ca[k][0];
      const double ai = f64 ? P[s].ld.ca[k][1] : P[s].lf.ca[k][1];
      const double br = f64 ? P[s].ld.cb[k][0] : P[s].lf.cb[k][0];
      const double bi = f64 ? P[s].ld.cb[k][1] : P[s].lf.cb[k][1];
      const double v0[4] = {ar, ai, br, bi}, v1[4] = {-ai, ar, -bi, br};
      for (int q = 0; q < 4; ++q) {
        const int i0 = (2 * k) * ldw + col + q, i1 = (2 * k + 1) * ldw + col + q;
        if (f64) {
          w64[i0] = v0[q];
          w64[i1] = v1[q];
        } else {
          w32[i0] = static_cast<float>(v0[q]);
          w32[i1] = static_cast<float>(v1[q]);
        }
      }
    }
  }
  MultiArgs a;
  memset(&a, 0, sizeof a);
  a.cache = f64 ? static_cast<const void*>(D.c64) : static_cast<const void*>(D.c32);
  a.t = D.t;
  a.ld = D.ld;
  a.n = D.n;
  a.nb = static_cast<int32_t>(std::min<int64_t>(TARGET_BLOCKS, (D.n + BLOCK - 1) / BLOCK));
  a.epb = a.nb > 0 ? ((D.n + a.nb - 1) / a.nb + BLOCK - 1) / BLOCK * BLOCK : BLOCK;
  if (a.nb > 0) a.nb = static_cast<int32_t>((D.n + a.epb - 1) / a.epb);
  a.n_sets = n_sets;
  a.ldw = ldw;
  a.w = c->d_multi_w;
  a.params = c->d_multi_params;
  a.gram = c->d_gram;
  a.n_mc = M.n;
  a.results = c->d_multi_res;
  const int64_t need = static_cast<int64_t>(n_sets) * 3 * std::max(a.nb, 1) * 2;
  if (c->multi_rows_cap < need) {
    if (c->d_multi_rows) (void)hipFree(c->d_multi_rows);
    c->d_multi_rows = nullptr;
    c->multi_rows_cap = 0;
    HIP_TRY(hipMalloc(&c->d_multi_rows, need * sizeof(double)));
    c->multi_rows_cap = need;
  }
  a.rows = c->d_multi_rows;
  HIP_TRY(hipMemcpyAsync(c->d_multi_params, P, n_sets * sizeof(EvalParams), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_multi_w, c->h_multi_w, 16 * ldw * (f64 ? sizeof(double) : sizeof(float)),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(launch_multi(precision, c->ma, c->mb, a, P[first], c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int s = 0; s < n_sets; ++s) {
    const double* r = c->h_multi_res + static_cast<int64_t>(s) * RES_WORDS;
    nll_out[s] = ok[s] ? r[0] : INFINITY;
  }
  return MXA_OK;
}

int32_t mxa_set_mc_mode(mxa_ctx* c, int32_t mode) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  if (mode != MXA_MC_DIRECT && mode != MXA_MC_GRAM) return fail(MXA_EINVAL, "bad MC mode");
  c->mc_mode = mode;
  return MXA_OK;
}

int32_t mxa_set_stream(mxa_ctx* c, void* stream) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  HIP_TRY(hipSetDevice(c->device));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (s) {
    hipDevice_t dev = -1;
    HIP_TRY(hipStreamGetDevice(s, &dev));
    if (dev != c->device) return fail(MXA_EINVAL, "stream of device %d, context on device %d", dev, c->device);
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->stream = s;
  return MXA_OK;
}

int32_t mxa_set_timing(mxa_ctx* c, int32_t on) {
  if (!c) return fail(MXA_EINVAL, "context is NULL");
  c->timing = on != 0;
  return MXA_OK;
}

int32_t mxa_kernel_time(mxa_ctx* c, double* ms_total, int64_t* launches, int32_t reset) {
  if (!c || !ms_total || !launches) return fail(MXA_EINVAL, "NULL argument");
  *ms_total = c->time_ms;
  *launches = c->timed;
  if (reset) {
    c->time_ms = 0.0;
    c->timed = 0;
  }
  return MXA_OK;
}

int32_t mxa_launch_shape(mxa_ctx* c, int32_t grad, int64_t* out4) {
  if (!c || !out4) return fail(MXA_EINVAL, "NULL argument");
  (void)grad;
  const Shape sh = shape_for(c->s[MXA_DATA].n, c->s[MXA_MC].n);
  out4[0] = sh.nb_d;
  out4[1] = sh.epb_d;
  out4[2] = sh.nb_m;
  out4[3] = sh.epb_m;
  return MXA_OK;
}

const char* mxa_last_error(void) { return g_err.c_str(); }

}  // extern "C"
