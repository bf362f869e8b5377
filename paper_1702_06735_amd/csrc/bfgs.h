// BFGS minimiser as a state machine driven by function-and-gradient values.
//
// The fits of the sensitivity study (Sec. 4) minimise the NLL over the
// coefficients and x, y. A fit asks for the point it wants evaluated
// (`point()`), receives the NLL and gradient there (`tell()`), and decides the
// next point, so any number of fits can be advanced from one batched
// evaluation. Host code only; usable from C++ and from the host tests.
//
// Method: quasi-Newton BFGS on the free parameters in scaled coordinates
// u_i = (theta_i - theta0_i) / scale_i, with a backtracking line search under
// the Armijo condition and the inverse-Hessian update skipped when the
// curvature s.y is not positive. Converged when the scaled gradient's largest
// component falls below gtol; or when the estimated distance to the minimum,
// edm = g^T H^-1 g / 2 with the current inverse-Hessian estimate, and the
// decrease of f over the step both fall below edm_tol on two accepted steps in
// a row, once there have been at least as many accepted steps as free
// parameters (the usual stopping rule of likelihood fits, independent of the
// parameters' scales); or when two accepted steps in a row lower f by less
// than ftol max(1, |f|).
//
// Errors (optional): after the minimisation has finished (converged or out of
// evaluations), the machine asks for the gradient at u* +- h_i e_i for every
// free parameter, forms the Hessian of f by central differences of the
// gradient, H_ij = (g_j(u* + h_i e_i) - g_j(u* - h_i e_i)) / (2 h_i),
// symmetrised, and inverts it by a Cholesky factorisation. For f = -ln L the
// inverse is the covariance matrix of the estimates (the inverse of the
// observed information); the errors are the square roots of its diagonal in
// theta units. Steps: h_i = 0.1 sqrt(Hinv_ii) from the minimiser's
// inverse-Hessian estimate, clamped to [1e-3, 1] in scaled units.
#pragma once

#include <math.h>
#include <string.h>

#include <vector>

namespace mxa {

class Bfgs {
 public:
  enum Status { RUNNING = 0, CONVERGED = 1, MAX_EVALS = 2, FAILED = 3 };

  // n_theta: full parameter vector length; free_idx: indices of the free
  // parameters; scale: per-free-parameter scale (> 0).
  void init(const double* theta0, int n_theta, const int* free_idx, const double* scale, int n_free,
            int max_evals, double gtol, double ftol, double edm_tol = 0.0, bool errors = false) {
    n_ = n_free;
    want_errors_ = errors;
    errors_ok_ = false;
    fit_status_ = RUNNING;
    err_.assign(n_, 0.0);
    cov_.assign(static_cast<size_t>(n_) * n_, 0.0);
    edm_tol_ = edm_tol;
    nt_ = n_theta;
    th0_.assign(theta0, theta0 + n_theta);
    idx_.assign(free_idx, free_idx + n_free);
    sc_.assign(scale, scale + n_free);
    max_evals_ = max_evals;
    gtol_ = gtol;
    ftol_ = ftol;
    u_.assign(n_, 0.0);
    g_.assign(n_, 0.0);
    gbest_.assign(n_theta, NAN);
    H_.assign(static_cast<size_t>(n_) * n_, 0.0);
    for (int i = 0; i < n_; ++i) H_[i * n_ + i] = 1.0;
    d_.assign(n_, 0.0);
    gt_.assign(n_, 0.0);
    s_.assign(n_, 0.0);
    y_.assign(n_, 0.0);
    hy_.assign(n_, 0.0);
    hg_.assign(n_, 0.0);
    f_ = INFINITY;
    evals_ = 0;
    iters_ = 0;
    small_ = 0;
    edm_ok_ = 0;
    restarted_ = false;
    phase_ = FIRST;
    status_ = RUNNING;
    theta_.assign(th0_.begin(), th0_.end());
    cur_ = u_;
  }

  // parameter vector to evaluate next (valid while status() == RUNNING)
  const double* point() const { return theta_.data(); }

  // NLL value and full gradient (n_theta entries) at point()
  void tell(double f, const double* grad_full) {
    ++evals_;
    std::vector<double>& g = gt_;
    bool finite = isfinite(f);
    for (int i = 0; i < n_; ++i) {
      g[i] = grad_full[idx_[i]] * sc_[i];  // d f / d u_i
      finite = finite && isfinite(g[i]);
    }
    if (phase_ == HESSE) return hesse_tell(g, finite);
    if (phase_ == FIRST) {
      if (!finite) return finish(FAILED);
      f_ = f;
      g_ = g;
      gbest_.assign(grad_full, grad_full + nt_);
      if (gnorm(g_) <= gtol_) return finish(CONVERGED);
      return start_line_search(true);
    }
    // line search in progress: trial point cur_ = u_ + alpha_ d_
    const double slope = dot(g_, d_);
    if (finite && f <= f_ + 1e-4 * alpha_ * slope) {
      // accept
      for (int i = 0; i < n_; ++i) {
        s_[i] = cur_[i] - u_[i];
        y_[i] = g[i] - g_[i];
      }
      const double fprev = f_;
      u_ = cur_;
      f_ = f;
      g_ = g;
      gbest_.assign(grad_full, grad_full + nt_);
      ++iters_;
      update_inverse_hessian(s_, y_);
      if (gnorm(g_) <= gtol_) return finish(CONVERGED);
      // H g serves both the estimated distance and the next direction
      mat_vec(H_, g_, hg_);
      // the inverse-Hessian estimate needs about one accepted step per free
      // parameter before its edm can be trusted, and it can still miss
      // directions the minimiser has barely moved along: the step's actual
      // decrease must be below the tolerance too, on two steps in a row
      if (edm_tol_ > 0.0 && iters_ >= n_ && 0.5 * dot(g_, hg_) < edm_tol_ && fprev - f < edm_tol_) {
        if (++edm_ok_ >= 2) return finish(CONVERGED);
      } else {
        edm_ok_ = 0;
      }
      if (fprev - f <= ftol_ * fmax(1.0, fabs(f))) {
        if (++small_ >= 2) return finish(CONVERGED);
      } else {
        small_ = 0;
      }
      if (evals_ >= max_evals_) return finish(MAX_EVALS);
      return start_line_search(false, true);
    }
    // reject: shrink the step
    if (evals_ >= max_evals_) return finish(MAX_EVALS);
    if (finite) {
      // quadratic interpolation of the step, safeguarded to [0.1, 0.5] alpha
      const double denom = 2.0 * (f - f_ - alpha_ * slope);
      double a = denom > 0.0 ? -slope * alpha_ * alpha_ / denom : 0.5 * alpha_;
      alpha_ = fmin(fmax(a, 0.1 * alpha_), 0.5 * alpha_);
    } else {
      alpha_ *= 0.25;
    }
    if (alpha_ < 1e-12) {
      // no progress along d: restart from steepest descent once, then stop
      if (!restarted_) {
        restarted_ = true;
        for (int i = 0; i < n_ * n_; ++i) H_[i] = 0.0;
        for (int i = 0; i < n_; ++i) H_[i * n_ + i] = 1.0;
        return start_line_search(true);
      }
      return finish(CONVERGED);
    }
    set_trial();
  }

  Status status() const { return status_; }
  // errors were requested, computed, and the Hessian is positive definite
  bool errors_ok() const { return errors_ok_; }
  // errors of the free parameters (theta units, in free-parameter order)
  const double* errors() const { return err_.data(); }
  // covariance of the free parameters (theta units, n_free x n_free)
  const double* covariance() const { return cov_.data(); }
  int n_free() const { return n_; }
  int free_index(int i) const { return idx_[i]; }
  int evals() const { return evals_; }
  int iterations() const { return iters_; }
  double best_f() const { return f_; }
  // best parameter vector found so far
  void best(double* theta) const {
    for (int i = 0; i < nt_; ++i) theta[i] = th0_[i];
    for (int i = 0; i < n_; ++i) theta[idx_[i]] = th0_[idx_[i]] + sc_[i] * u_[i];
  }
  double grad_norm() const { return gnorm(g_); }
  // full gradient (n_theta entries, theta units) at the best point; NaN
  // before the first evaluation
  const double* best_grad() const { return gbest_.data(); }
  // estimated distance to the minimum, g^T H^-1 g / 2
  double edm() const {
    double e = 0.0;
    for (int i = 0; i < n_; ++i) {
      double v = 0.0;
      for (int j = 0; j < n_; ++j) v += H_[i * n_ + j] * g_[j];
      e += g_[i] * v;
    }
    return 0.5 * e;
  }

 private:
  enum Phase { FIRST, SEARCH, HESSE };

  static double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
  }
  static double gnorm(const std::vector<double>& g) {
    double m = 0.0;
    for (double v : g) m = fmax(m, fabs(v));
    return m;
  }

  void finish(Status s) {
    if (want_errors_ && s != FAILED && phase_ != HESSE) return start_hesse(s);
    status_ = s;
  }

  // error phase: 2 n gradient evaluations around the best point
  void start_hesse(Status s) {
    fit_status_ = s;
    phase_ = HESSE;
    h_.assign(n_, 0.0);
    for (int i = 0; i < n_; ++i) {
      const double hii = H_[i * n_ + i];
      h_[i] = fmin(1.0, fmax(1e-3, 0.1 * sqrt(hii > 0.0 ? hii : 0.0)));
    }
    gp_.assign(static_cast<size_t>(n_) * n_, 0.0);
    hk_ = 0;
    set_hesse_point();
  }
  void set_hesse_point() {
    const int i = hk_ / 2;
    const double sgn = (hk_ & 1) ? -1.0 : 1.0;
    for (int j = 0; j < nt_; ++j) theta_[j] = th0_[j];
    for (int j = 0; j < n_; ++j)
      theta_[idx_[j]] = th0_[idx_[j]] + sc_[j] * (u_[j] + (j == i ? sgn * h_[i] : 0.0));
  }
  void hesse_tell(const std::vector<double>& g, bool finite) {
    if (!finite) {
      status_ = fit_status_;
      return;
    }
    const int i = hk_ / 2;
    const double sgn = (hk_ & 1) ? -1.0 : 1.0;
    for (int j = 0; j < n_; ++j) gp_[i * n_ + j] += sgn * g[j] / (2.0 * h_[i]);
    if (++hk_ < 2 * n_) return set_hesse_point();
    // symmetrise, factorise A = L L^T, invert
    std::vector<double> A(static_cast<size_t>(n_) * n_), L(static_cast<size_t>(n_) * n_, 0.0);
    for (int a = 0; a < n_; ++a)
      for (int b = 0; b < n_; ++b) A[a * n_ + b] = 0.5 * (gp_[a * n_ + b] + gp_[b * n_ + a]);
    bool pd = true;
    for (int a = 0; a < n_ && pd; ++a) {
      for (int b = 0; b <= a; ++b) {
        double v = A[a * n_ + b];
        for (int k = 0; k < b; ++k) v -= L[a * n_ + k] * L[b * n_ + k];
        if (a == b) {
          if (!(v > 0.0)) {
            pd = false;
            break;
          }
          L[a * n_ + a] = sqrt(v);
        } else {
          L[a * n_ + b] = v / L[b * n_ + b];
        }
      }
    }
    if (pd) {
      // columns of A^-1 by forward and back substitution
      std::vector<double> col(n_);
      for (int c = 0; c < n_; ++c) {
        for (int a = 0; a < n_; ++a) {
          double v = (a == c) ? 1.0 : 0.0;
          for (int k = 0; k < a; ++k) v -= L[a * n_ + k] * col[k];
          col[a] = v / L[a * n_ + a];
        }
        for (int a = n_ - 1; a >= 0; --a) {
          double v = col[a];
          for (int k = a + 1; k < n_; ++k) v -= L[k * n_ + a] * col[k];
          col[a] = v / L[a * n_ + a];
        }
        for (int a = 0; a < n_; ++a) cov_[a * n_ + c] = col[a] * sc_[a] * sc_[c];
      }
      for (int a = 0; a < n_; ++a) err_[a] = sqrt(cov_[a * n_ + a]);
      errors_ok_ = true;
    }
    status_ = fit_status_;
  }

  // y = A x for the n x n matrix A
  void mat_vec(const std::vector<double>& A, const std::vector<double>& x, std::vector<double>& y) const {
    for (int i = 0; i < n_; ++i) {
      const double* a = A.data() + static_cast<size_t>(i) * n_;
      double v = 0.0;
      for (int j = 0; j < n_; ++j) v += a[j] * x[j];
      y[i] = v;
    }
  }

  // have_hg: hg_ already holds H g
  void start_line_search(bool steepest, bool have_hg = false) {
    if (!have_hg) mat_vec(H_, g_, hg_);
    for (int i = 0; i < n_; ++i) d_[i] = -hg_[i];
    double slope = dot(g_, d_);
    if (!(slope < 0.0)) {  // not a descent direction: fall back to -g
      for (int i = 0; i < n_; ++i) d_[i] = -g_[i];
      slope = dot(g_, d_);
    }
    // first step: at most a unit move in scaled coordinates
    alpha_ = 1.0;
    if (steepest && iters_ == 0) alpha_ = fmin(1.0, 1.0 / fmax(gnorm(g_), 1e-300));
    phase_ = SEARCH;
    set_trial();
  }

  void set_trial() {
    for (int i = 0; i < n_; ++i) cur_[i] = u_[i] + alpha_ * d_[i];
    for (int i = 0; i < nt_; ++i) theta_[i] = th0_[i];
    for (int i = 0; i < n_; ++i) theta_[idx_[i]] = th0_[idx_[i]] + sc_[i] * cur_[i];
  }

  void update_inverse_hessian(const std::vector<double>& s, const std::vector<double>& y) {
    const double sy = dot(s, y);
    if (!(sy > 1e-300)) return;
    if (iters_ == 1) {
      // scale the initial inverse Hessian by s.y / y.y
      const double gam = sy / dot(y, y);
      for (int i = 0; i < n_ * n_; ++i) H_[i] *= gam;
    }
    const double rho = 1.0 / sy;
    std::vector<double>& Hy = hy_;
    mat_vec(H_, y, Hy);
    const double yHy = dot(y, Hy);
    // symmetric rank-two update: the upper triangle, mirrored
    const double c = 1.0 + rho * yHy;
    for (int i = 0; i < n_; ++i) {
      double* hi = H_.data() + static_cast<size_t>(i) * n_;
      for (int j = i; j < n_; ++j) {
        const double v = hi[j] + rho * (c * s[i] * s[j] - Hy[i] * s[j] - s[i] * Hy[j]);
        hi[j] = v;
        H_[static_cast<size_t>(j) * n_ + i] = v;
      }
    }
  }

  int n_ = 0, nt_ = 0, max_evals_ = 0, evals_ = 0, iters_ = 0, small_ = 0, edm_ok_ = 0, hk_ = 0;
  bool restarted_ = false, want_errors_ = false, errors_ok_ = false;
  Status fit_status_ = RUNNING;
  std::vector<double> h_, gp_, err_, cov_;
  double gtol_ = 0.0, ftol_ = 0.0, edm_tol_ = 0.0, f_ = 0.0, alpha_ = 1.0;
  std::vector<double> th0_, sc_, u_, g_, H_, d_, cur_, theta_, gbest_;
  std::vector<double> gt_, s_, y_, hy_, hg_;  // scratch of tell()
  std::vector<int> idx_;
  Phase phase_ = FIRST;
  Status status_ = RUNNING;
};

}  // namespace mxa
