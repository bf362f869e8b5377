// Slot layout of the evaluation passes and the step from slot totals to the
// NLL and its gradient, shared by the device (the fit server's and the
// many-set finalisations) and the host (a context's evaluation, which forms
// them from the totals its last kernel publishes).
#pragma once

#include <math.h>

#include "internal.h"

namespace mxa {

constexpr int KS_SET = 0x07 | 0xC0;   // chains containing the K*0 lineshape
constexpr int RHO_SET = 0x3F;         // chains containing the rho0 lineshape
constexpr int A1_SET = 0x30;          // chains containing the a1 lineshape
constexpr int K1_SET = 0xC0;

constexpr int popc(int m) { return m == 0 ? 0 : (m & 1) + popc(m >> 1); }
constexpr int rank_in(int m, int k) { return popc(m & ((1 << k) - 1)); }
constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// ===========================================================================
// Accumulator slots of the passes. Each workgroup takes a contiguous range of
// data (or MC) events:
//   data: 0 sum(Gamma t - ln B), 1 sum|Gamma t - ln B|, 2 #(B <= 0),
//         3 sum w dB/dx, 4 sum w dB/dy,                     (w = 1/B)
//   MC:   0 sum|A|^2, 1 sum|Ab|^2, 2 sum Re(A Ab*), 3 sum Im(A Ab*), 4 -,
//   both (adjoint only): 5..10 (u, v) of K*0, rho0, a1;
//         11.. W_k = sum conj(G_A) beta_k (k in A_f), then conj(G_Ab) beta_k;
//   data with a background component, adjoint only: NS sum w B (the weight
//         of the normalisation gradient), NS + 1 sum d(-ln p)/df.
template <bool GRAD, int MA, int MB, bool BKG = false> struct Slots {
  static constexpr int NS = GRAD ? 11 + 2 * (popc(MA) + popc(MB)) : 4;
  static constexpr int NT = NS + (BKG && GRAD ? 2 : 0);  // slots written per row
  static constexpr int P = pow2_at_least(NT);
  static constexpr int NREG = 5;                       // FP64 register slots
  static constexpr int NADJ = GRAD ? NS - NREG : 1;    // adjoint slots
  // LDS words per thread for the adjoint slots of precision R
  template <class R> static constexpr int lds_words() { return sizeof(R) == 4 ? 1 : NADJ; }
};

// MC totals from the Gram matrix of the reduced chain amplitudes (Sec. 3.1
// normalisation with the lineshapes fixed): with U_k = sum_l conj(c'_l) G_kl
// and V_k = sum_l conj(cbar'_l) G_kl,
//   sum|A|^2 = sum_k c'_k U_k,  sum|Ab|^2 = sum_k cbar'_k V_k,
//   sum A Ab* = sum_k c'_k V_k,
//   W_k = hp U_k - (hr - i hi) V_k,  Wbar_k = hm V_k - (hr + i hi) U_k.
// The lineshape adjoint slots have no Gram form and are left NaN.
template <int MA, int MB>
__host__ __device__ inline void mc_from_gram(const EvalParams& p, const double* G, double* M) {
  const FinConst& f = p.fin;
  double ur[8], ui[8], vr[8], vi[8];
  for (int k = 0; k < 8; ++k) {
    ur[k] = ui[k] = vr[k] = vi[k] = 0.0;
    for (int l = 0; l < 8; ++l) {
      const double gr = G[(k * 8 + l) * 2], gi = G[(k * 8 + l) * 2 + 1];
      ur[k] += f.ca[l][0] * gr + f.ca[l][1] * gi;
      ui[k] += f.ca[l][0] * gi - f.ca[l][1] * gr;
      vr[k] += f.cb[l][0] * gr + f.cb[l][1] * gi;
      vi[k] += f.cb[l][0] * gi - f.cb[l][1] * gr;
    }
  }
  double a2 = 0.0, b2 = 0.0, xr = 0.0, xi = 0.0;
  for (int k = 0; k < 8; ++k) {
    a2 += f.ca[k][0] * ur[k] - f.ca[k][1] * ui[k];
    b2 += f.cb[k][0] * vr[k] - f.cb[k][1] * vi[k];
    xr += f.ca[k][0] * vr[k] - f.ca[k][1] * vi[k];
    xi += f.ca[k][0] * vi[k] + f.ca[k][1] * vr[k];
  }
  M[0] = a2;
  M[1] = b2;
  M[2] = xr;
  M[3] = xi;
  M[4] = 0.0;
  for (int s = 5; s < 11; ++s) M[s] = NAN;
  const double hp = p.mix.h_sum + p.mix.h_diff, hm = p.mix.h_sum - p.mix.h_diff;
  const double hr = 0.5 * p.mix.h_re, hi = 0.5 * p.mix.h_im;
  for (int k = 0; k < 8; ++k) {
    if (MA & (1 << k)) {
      const int s = 11 + 2 * popc(MA & ((1 << k) - 1));
      M[s] = hp * ur[k] - (hr * vr[k] + hi * vi[k]);
      M[s + 1] = hp * ui[k] - (hr * vi[k] - hi * vr[k]);
    }
    if (MB & (1 << k)) {
      const int s = 11 + 2 * popc(MA) + 2 * popc(MB & ((1 << k) - 1));
      M[s] = hm * vr[k] - (hr * ur[k] - hi * ui[k]);
      M[s + 1] = hm * vi[k] - (hr * ui[k] + hi * ur[k]);
    }
  }
}

// NLL, Nhat and the gradient from the data totals D and MC totals M. Threads
// tid = 0 .. nthr-1 of the calling workgroup share the gradient entries
// (thread 0 also writes the NLL words).
template <int MA, int MB, int NS>
__host__ __device__ inline void finalize(const EvalArgs& a, const EvalParams& p, const double* D,
                                         const double* M, bool grad, int tid = 0, int nthr = 1) {
  const MixConst& x = p.mix;
  const FinConst& f = p.fin;
  double* res = a.result;
  const double S1 = M[0] + M[1], S2 = M[0] - M[1], S3 = M[2], S4 = M[3];
  const double sumT = x.h_sum * S1 + x.h_diff * S2 - x.h_re * S3 - x.h_im * S4;
  const double nd = static_cast<double>(a.n_d);
  // with a background component D[0] is already -sum ln p (Nhat inside)
  const bool bkg = p.mix.g_bkg > 0.0;
  if (tid == 0) {
    const double nhat = sumT / static_cast<double>(a.n_m);
    const double lnh = log(nhat);
    const double nll = bkg ? D[0] : D[0] + nd * lnh;
    const bool bad = D[2] > 0.0 || !(nhat > 0.0) || !isfinite(nll);
    res[0] = bad ? INFINITY : nll;
    res[1] = nhat;
    res[2] = D[0];
    res[3] = bkg ? D[1] : D[1] + nd * fabs(lnh);
    res[4] = D[2];
    res[5] = sumT;
    res[6] = bad ? 1.0 : 0.0;
  }
  if (!grad) return;
  double* g = res + 8;
  // weight of the normalisation gradient: n_data, or sum w B with background
  const double fm = (bkg ? D[NS] : nd) / sumT;
  constexpr int WB = 11 + 2 * popc(MA);
  auto slot_a = [](int k) { return 11 + 2 * popc(MA & ((1 << k) - 1)); };
  auto slot_b = [](int k) { return WB + 2 * popc(MB & ((1 << k) - 1)); };
  // 2 Re sum_{k in set} (c'_k W_k + cbar'_k Wbar_k): parameter-only factors kappa_k
  auto kap = [&](const double* X, int set) {
    double s = 0.0;
    for (int k = 0; k < 8; ++k) {
      if (!(set & (1 << k))) continue;
      if (MA & (1 << k)) {
        const int sl = slot_a(k);
        s += f.ca[k][0] * X[sl] - f.ca[k][1] * X[sl + 1];
      }
      if (MB & (1 << k)) {
        const int sl = slot_b(k);
        s += f.cb[k][0] * X[sl] - f.cb[k][1] * X[sl + 1];
      }
    }
    return 2.0 * s;
  };
  // sums over events of w dB/dtheta (data) or dT/dtheta (MC) for the masses
  // and widths
  auto shape_term = [&](const double* X, int which) {
    switch (which) {
      case 0: return -2.0 * (f.ks_alpha_m * X[5] + f.ks_beta_m * X[6]) + f.lam_ks * kap(X, KS_SET);
      case 1: return -2.0 * f.ks_beta_g * X[6];
      case 2: return -2.0 * (f.rho_alpha_m * X[7] + f.rho_beta_m * X[8]) + f.lam_rho * kap(X, RHO_SET);
      case 3: return -2.0 * f.rho_beta_g * X[8];
      case 4: return -2.0 * (2.0 * f.a1_m0 * X[9] + f.a1_g0 * X[10]) + f.lam_a1d * kap(X, 0x20);
      default: return -2.0 * f.a1_m0 * X[10];
    }
  };
  const int nc = 2 * (f.na + f.nb);
  for (int j = tid; j < nc + 8 + (bkg ? 1 : 0); j += nthr) {
    double v;
    if (j == nc + 8) {
      v = D[NS + 1];  // background fraction
    } else if (j < nc) {
      // coefficients: Re and Im of A_f's, then of Abar_f's
      const bool in_a = j < 2 * f.na;
      const int q = in_a ? j / 2 : (j - 2 * f.na) / 2;
      const int k = in_a ? f.ka[q] : f.kb[q];
      const int s = in_a ? slot_a(k) : slot_b(k);
      v = (j & 1) ? f.kappa[k] * (2.0 * D[s + 1] - 2.0 * fm * M[s + 1])
                  : f.kappa[k] * (-2.0 * D[s] + 2.0 * fm * M[s]);
    } else if (j == nc) {
      v = -D[3] + fm * (f.dhdiff_dx * S2 - f.dhim_dx * S4);  // x
    } else if (j == nc + 1) {
      v = -D[4] + fm * (f.dhsum_dy * S1 - f.dhre_dy * S3);  // y
    } else {
      const int w = j - nc - 2;  // K*0 mass, width, rho0 mass, width, a1 mass, width
      v = -shape_term(D, w) + fm * shape_term(M, w);
    }
    g[j] = v;
  }
}

}  // namespace mxa
