// Internal definitions shared by the HIP kernels (kernels.hip) and the host
// side of the C-ABI (api.hip). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mxa {

// ---------------------------------------------------------------------------
// Tier-0 per-event cache: parameter-independent values computed once per
// sample from the four-momenta (Sec. 3: form factors, spin factors and the
// kinematic parts of the lineshapes are shared by every evaluation).
// Column-major (structure of arrays): value c of event i is at [c * ld + i].
// Per Bose configuration sigma (columns 12 sigma + 0..11):
//   0 s(K+ pi_s)            1 g_K*  = q^3 F_1(q)^2 / sqrt(s) of K*0 -> K pi
//   2 s(pi+ pi_o)           3 g_rho = q^3 F_1(q)^2 / sqrt(s) of rho0 -> pi pi
//   4 s(K+ pi_s pi+)
//   5 VV S-wave spin factor x F_1(q_K*) F_1(q_rho)
//   6 VV P-wave x F_1(q_D) F_1(q_K*) F_1(q_rho)
//   7 VV D-wave x F_2(q_D) F_1(q_K*) F_1(q_rho)
//   8 SV spin factor x F_1(q_D) F_1(q_rho)
//   9 a1 S-wave x F_1(q_D,a1) F_1(q_rho)
//  10 a1 D-wave x F_1(q_D,a1) F_1(q_rho) F_2(q_a1)
//  11 K1 S-wave x F_1(q_D,K1) F_1(q_K*)
// Shared: column 24 s(pi- pi+ pi-).
// pi_s is pi-(a) for sigma = 0 and pi-(b) for sigma = 1; pi_o is the other.
// ---------------------------------------------------------------------------
constexpr int NCOL = 25;
constexpr int CPS = 12;  // columns per Bose configuration
enum : int {
  C_SKPI = 0, C_GKS = 1, C_SPIPI = 2, C_GRHO = 3, C_SKPIPI = 4,
  C_SF1 = 5, C_SF2 = 6, C_SF3 = 7, C_SF4 = 8, C_SF5 = 9, C_SF6 = 10, C_SF7 = 11,
  C_S3PI = 24,
};

constexpr int BLOCK = 256;      // threads per workgroup of every kernel
constexpr int FIN_BLOCK = 1024; // threads of the generator's one-workgroup scan and sum
constexpr int MAX_THETA = 40;
constexpr int RES_WORDS = 8 + MAX_THETA;  // result record (doubles)

// Model constants needed on the device to build the tier-0 cache.
struct Tier0Const {
  double m_D, m_K, m_pi, r;
  double tol_p, tol_m2;  // validation tolerances
  int32_t parity = 0;    // 1: negate the 3-momenta on input (CP conjugate of a D0bar event)
  int32_t allow_neg_t = 0;  // 1: measured decay times may be negative (resolution)
};

// Per-launch lineshape and coefficient constants in the amplitude precision R.
// The reduced lineshape of a resonance is 1/D with
//   K*0, rho0: D = (m0^2 - s) - i K g(s),  K = Gamma0 m0^2 (1 + z0) / q0^3,
//   a1, K1:    D = (m0^2 - s) - i m0 Gamma0;
// every factor that depends only on the parameters (sqrt(1+z0) of the F_1
// ratio, sqrt(9+3z0+z0^2) of the F_2 ratio) is folded into the effective
// coefficient c'_k = c_k kappa_k.
// The running width enters through g(s) = q^3 F_1(q)^2 / sqrt(s), which a
// pass either reads from the cache or forms from s alone: with
// P = (s - (m_a + m_b)^2)(s - (m_a - m_b)^2) = 4 s q^2,
//   g = P sqrt(P) / (s (8 s + 2 r^2 P)).
template <class R> struct LsConst {
  R ks_m2, ks_k;
  R rho_m2, rho_k;
  R a1_m2, a1_mg;
  R k1a_m2, k1a_mg;
  R k1b_m2, k1b_mg;
  // P = s (s - t_sum) + t_prod with t_sum, t_prod the sum and product of
  // the two thresholds (m_a + m_b)^2, (m_a - m_b)^2
  R ks_tsum, ks_tprod;
  R rho_tsum, rho_tprod;  // (2 m_pi)^2, 0
  R r2x2;                 // 2 r^2
  // MC adjoint weights (Eq. (1) integrated over t): h_sum + h_diff,
  // h_sum - h_diff, h_re / 2, h_im / 2
  R mc_hp, mc_hm, mc_hr, mc_hi;
  R ca[8][2];  // c'_k of A_f (zero for chains not in A_f)
  R cb[8][2];  // c'_k of Abar_f
};

// Eq. (1) constants. Data: B = (|A|^2+|Ab|^2) cosh(yG t) + (|A|^2-|Ab|^2) cos(xG t)
//   - 2 Re(A Ab*) sinh(yG t) - 2 Im(A Ab*) sin(xG t).
// MC (time-integrated): T = h_sum (|A|^2+|Ab|^2) + h_diff (|A|^2-|Ab|^2)
//   - h_re Re(A Ab*) - h_im Im(A Ab*).
//
// Background component (models with g_bkg > 0): fraction f_bkg of the data,
// uniform in phase space with decay times from g_bkg exp(-g_bkg t).
struct MixConst {
  double gamma, xg, yg;
  double h_sum, h_diff, h_re, h_im;
  double f_bkg, g_bkg;  // g_bkg = 0: no background component
  double sigma_t;       // Gaussian decay-time resolution [ps]; 0: none
  double inv_nhat;      // many-set evaluation with a background component:
                        // 1 / Nhat of this set (from the Gram matrix); else 0
};

// Constants of the step from slot totals to the NLL and gradient
// (finalize(): on the host after a context's evaluation or a server tick, on
// the device in the many-set finalisation).
struct FinConst {
  double kappa[8];
  double ca[8][2], cb[8][2];
  double lam_ks, lam_rho, lam_a1d;  // d ln kappa / d m0 of K*0, rho0, a1 D-wave
  double ks_alpha_m, ks_beta_m, ks_beta_g;     // dD/dm0 = alpha - i g beta ...
  double rho_alpha_m, rho_beta_m, rho_beta_g;
  double a1_m0, a1_g0;
  double dhsum_dy, dhre_dy, dhdiff_dx, dhim_dx;
  int32_t na, nb;
  int32_t ka[8], kb[8];  // chain index (0..7) of theta's A_f / Abar_f entries
  int32_t n_theta;
};

struct EvalParams {
  LsConst<double> ld;
  LsConst<float> lf;
  MixConst mix;
  FinConst fin;
};

// Device buffers and launch geometry of one evaluation.
struct EvalArgs {
  const void* cache_d;  // data tier-0 cache (R), [NCOL][ld_d]
  const double* t_d;    // data decay times, [ld_d]
  const void* cache_m;  // MC tier-0 cache (R), [NCOL][ld_m]
  int64_t ld_d, ld_m;
  int64_t n_d, n_m;
  int64_t epb_d, epb_m;  // events per workgroup
  int32_t nb_d, nb_m;    // workgroups on data, on MC
  double* rows;          // [NS][nb_d + nb_m][2] workgroup partials (sum, error)
  double* totals;        // [2][64] slot totals of the data and the MC pass
  double* result;        // RES_WORDS doubles
  double* host_totals;   // mapped host memory [2][64] (or NULL): the
                         // reduction writes the slot totals here as well, for
                         // the host's finalisation (context evaluations)
  double inv_nhat;       // > 0: 1 / Nhat for a background data pass (Gram
                         // mode, formed on the host); 0: from the MC totals
  int32_t rev;           // 1: MC workgroups take the ranges in reverse order
  double seq;            // > 0: the last kernel writes it to result[7]
                         // after the totals, so that the host can wait for
                         // them by watching that word
};

// Gram matrix G_kl = sum_j beta_k,j conj(beta_l,j) of the reduced chain
// amplitudes over a sample (MFMA, FP64 accumulation).
struct GramArgs {
  const void* cache;
  int64_t ld, n, epb;
  int32_t nb;
  double* rows;  // [nb][256] per-workgroup real Gram (16 x 16)
  double* out;   // [8][8][2] complex Gram
};

// Batched evaluation of many fits (the fit server). A persistent launch walks
// a table of items (fit slot, event range of fit_chunk(n) events, by the fit's size); each item
// writes one row of partial sums. Then one workgroup per (fit, sum) combines
// that fit's rows in a fixed order into host memory, where the host forms
// each fit's NLL and gradient (with the shared MC Gram matrix).
// A fit's rows, and so its result, depend only on its own events and
// parameters, not on which other fits share the launch.
constexpr int MAX_FIT_EVENTS = 524288;  // events of one fit
// Events per item of a fit of n events: about n / 128, in whole workgroups
// of BLOCK events, at least one and at most 16 per thread (at most 128 items
// per fit). An item ends in a workgroup reduction of all the fit's sums, so
// longer items spread that cost over more events, while shorter ones give a
// fit running alone more workgroups (measured on 256 toy fits: n / 32 lost
// 20% on one fit at a time, n / 128 matched one-event items). A function of n
// alone, so that a fit's rows (and result) do not depend on the fits beside
// it.
constexpr int64_t fit_chunk(int64_t n) {
  const int64_t c = ((n + 127) / 128 + BLOCK - 1) / BLOCK * BLOCK;
  return c < BLOCK ? BLOCK : (c > 16 * BLOCK ? 16 * BLOCK : c);
}
constexpr int64_t MAX_FIT_ITEMS = MAX_FIT_EVENTS / (16 * BLOCK) + 32;  // items of one fit
constexpr int BATCH_GRID = 1024;  // workgroups of the persistent launch
// Servers with floating lineshapes also walk (MC range, active fit) items in
// a persistent launch of mc_grid workgroups (a multiple of the 8 XCDs, as
// many as are resident at once) over nb_mc ranges (a multiple of 8) of the
// shared MC sample, writing rows [NS][max_slots][nb_mc]; the reduction
// combines a fit's MC rows like its data rows, and the host uses those totals
// in place of the Gram matrix.

struct FitView {
  const void* cache;  // the fit's tier-0 cache (amplitude precision)
  const double* t;    // decay times
  int64_t ld, n;
  int32_t row0, nrows;
  int32_t active;
  int32_t pad;
};
struct FitItem {
  int32_t slot, row;
  int64_t lo, hi;
};
struct BatchArgs {
  const FitItem* items;
  const int32_t* n_items;
  const FitView* views;      // [max_slots]
  const EvalParams* params;  // [max_slots]
  double* rows;              // [NS (+ 2 with a background)][max_rows][2]
  int32_t max_rows;
  int32_t max_slots;
  int64_t n_mc;
  // floating lineshapes only (mc_cache null otherwise)
  const void* mc_cache;      // shared MC tier-0 cache (amplitude precision)
  int64_t mc_ld, epb_mc;
  int32_t nb_mc;             // MC ranges, a multiple of 8
  int32_t mc_grid;           // workgroups of the MC walk (batch_mc_grid)
  const int32_t* active;     // [max_slots] slots of the active fits
  const int32_t* n_active;
  double* mc_rows;           // [NS][max_slots][nb_mc][2]
  double* tot;               // [max_slots][2][64] data and MC totals, in mapped host
                             // memory: the host forms each fit's NLL and gradient
  unsigned* done;            // mapped host word: set last, behind a system-scope release
  // the group of slots this call evaluates (slot mod ngroups == group): its
  // work table (items), parameters and flag; the reduction skips the others
  int32_t group, ngroups;
  // model extensions (Gram servers): a background component (each fit's
  // 1 / Nhat for the data pass in its parameters) and a Gaussian decay-time
  // resolution
  int32_t bkg, res;
};
hipError_t launch_batch(int precision, int ma, int mb, const BatchArgs& a, hipStream_t s);
// The basis of a fit with fixed lineshapes: each event's Bose-symmetrised
// reduced chain amplitudes B_k, from its tier-0 cache (ld) at the lineshapes
// of p, into basis_columns(ma, mb) columns of bld values (Re, Im per chain of
// the kernels' chain set), in the amplitude precision (0: FP64, else FP32).
int basis_columns(int ma, int mb);
hipError_t launch_basis(int precision, int ma, int mb, const void* cache, int64_t ld, int64_t n,
                        const EvalParams& p, void* basis, int64_t bld, hipStream_t s);
// Workgroups the MC walk of a streamed server launches on `device` (0 on
// error).
int batch_mc_grid(int precision, int ma, int mb, int device);

// Per-event diagnostics kernel arguments.
struct TermsArgs {
  const void* cache;
  const double* t;  // NULL for MC
  int64_t ld, n;
  double* out;      // [n][5]
};

// Pseudo-experiment generation (Sec. 3.1): one launch examines candidates
// first .. first + n - 1 (n a multiple of BLOCK). Candidate i draws its
// uniforms from Philox4x32-10 with counter (i lo, i hi, j, stream), j = 0..5,
// and key (key0, key1).
struct GenConst {
  uint64_t first;
  int64_t n;
  uint32_t key0, key1, stream, pad;
  double M, m[4];   // parent and final-state masses
  double wmax;      // bound of the GENBOD weight
  double envelope;  // M_Phi: bound of |A|^2 + |Abar|^2 (data)
  double gamma, y;  // decay-time distribution exp(-Gamma t) cosh(y Gamma t)
  Tier0Const t0;
};
struct GenArgs {
  GenConst g;
  uint8_t* flags;        // [n]: bit 0 kept by GENBOD, bit 1 kept, bit 2 rate above the envelope
  uint32_t* bcount;      // [n / BLOCK] kept per block
  uint32_t* boff;        // [n / BLOCK] exclusive prefix of bcount
  uint32_t* total;       // kept in this launch
  int64_t* last;         // chunk index of the event that fills the output
  unsigned long long* counts;  // [2] kept by GENBOD, exceedances (up to the cut)
  double* p4;            // [n_out][16]
  double* t;             // [n_out] (data) or NULL
  int64_t* idx;          // [n_out] or NULL
  int64_t filled, n_out;
};
// flags, block counts and their prefix for a chunk (kind MXA_DATA evaluates
// Eq. (1) at p), then the kept events' output
hipError_t launch_gen_chunk(bool data, int ma, int mb, const GenArgs& a, const EvalParams& p,
                            hipStream_t s);
// GENBOD and exceedance counts over chunk candidates [0, limit)
hipError_t launch_gen_stats(const GenArgs& a, int64_t limit, hipStream_t s);

// Many parameter sets sharing the lineshapes: the data pass contracts each
// event's 16 reals (Re, Im of B_1..B_8) with W[16][ldw] (column 4 s + {0..3}:
// Re A, Im A, Re Abar, Im Abar of set s); the MC part comes from the Gram.
constexpr int MAX_SETS = 64;
struct MultiArgs {
  const void* cache;          // data tier-0 cache in R
  const double* t;            // data decay times
  int64_t ld, n;              // data sample
  int64_t epb;                // events per workgroup (multiple of BLOCK)
  int32_t nb;                 // workgroups along the events
  int32_t n_sets;
  int32_t ldw;                // 64 x number of 16-set chunks
  int32_t pad;
  const void* w;              // [16][ldw] in R
  const EvalParams* params;   // [n_sets]
  double* rows;               // [n_sets][3][nb][2]
  const double* gram;         // reduced MC Gram [8][8][2]
  int64_t n_mc;
  double* results;            // [n_sets][RES_WORDS]
};
hipError_t launch_multi(int precision, int ma, int mb, const MultiArgs& a, const EvalParams& p0,
                        hipStream_t s);

// The NLL and gradient of a context's evaluation from its published slot
// totals D (data) and M (MC; with G, the host copy of the Gram matrix, the
// MC totals are formed from it into M), written to a.result on the host.
void finalize_host(int ma, int mb, bool grad, const EvalArgs& a, const EvalParams& p, const double* D,
                   double* M, const double* G);
// sum over the MC sample of the time-integrated rate at p, from the host copy
// G of the Gram matrix (Nhat = that / n_mc)
double gram_sum_t(int ma, int mb, const EvalParams& p, const double* G);

// Launchers (kernels.hip). Return hipSuccess or the launch error.
hipError_t launch_tier0(const Tier0Const& k, const double* p4, const double* t, int64_t n, int64_t ld,
                        double* c64, float* c32, double* t64, unsigned* n_bad, hipStream_t s);
// Launches the data pass, the MC pass, the slot reduction and the kernel that
// publishes the totals to a.host_totals (then a.seq to a.result[7]); the
// optional events t0, t1 bracket the MC pass (the dominant kernel) on s.
hipError_t launch_eval(int precision, bool grad, int ma, int mb, const EvalArgs& a,
                       const EvalParams& p, hipStream_t s, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_terms(int precision, int ma, int mb, const TermsArgs& a, const EvalParams& p,
                        hipStream_t s);
hipError_t launch_gram(int precision, int ma, int mb, const GramArgs& a, const EvalParams& p,
                       hipStream_t s);
int slots_for(bool grad, int ma, int mb);
bool specialised(int ma, int mb);

// Host helpers shared by the C-ABI files (api.hip).
int32_t set_error(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Validate a model description (MXA_OK or MXA_EINVAL with the error set).
int32_t check_model_desc(const struct mxa_model_desc* m);
// Per-launch constants for parameter vector th (MXA_OK or MXA_EDOMAIN).
int32_t make_params(const struct mxa_model_desc& m, const double* th, EvalParams& P);
// 2 (n_a + n_ab) + 8, plus 1 for the background fraction of a model with a
// background component
int theta_count(const struct mxa_model_desc& m);
// Index in theta of the K*0 mass, the first of the six masses and widths:
// 2 (n_a + n_ab) + 2
int shape_offset(const struct mxa_model_desc& m);

}  // namespace mxa
