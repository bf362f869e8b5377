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
            int max_evals, double gtol, double ftol, double edm_tol = 0.0) {
    n_ = n_free;
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
    H_.assign(static_cast<size_t>(n_) * n_, 0.0);
    for (int i = 0; i < n_; ++i) H_[i * n_ + i] = 1.0;
    d_.assign(n_, 0.0);
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
    std::vector<double> g(n_);
    bool finite = isfinite(f);
    for (int i = 0; i < n_; ++i) {
      g[i] = grad_full[idx_[i]] * sc_[i];  // d f / d u_i
      finite = finite && isfinite(g[i]);
    }
    if (phase_ == FIRST) {
      if (!finite) return finish(FAILED);
      f_ = f;
      g_ = g;
      if (gnorm(g_) <= gtol_) return finish(CONVERGED);
      return start_line_search(true);
    }
    // line search in progress: trial point cur_ = u_ + alpha_ d_
    const double slope = dot(g_, d_);
    if (finite && f <= f_ + 1e-4 * alpha_ * slope) {
      // accept
      std::vector<double> s(n_), y(n_);
      for (int i = 0; i < n_; ++i) {
        s[i] = cur_[i] - u_[i];
        y[i] = g[i] - g_[i];
      }
      const double fprev = f_;
      u_ = cur_;
      f_ = f;
      g_ = g;
      ++iters_;
      update_inverse_hessian(s, y);
      if (gnorm(g_) <= gtol_) return finish(CONVERGED);
      // the inverse-Hessian estimate needs about one accepted step per free
      // parameter before its edm can be trusted, and it can still miss
      // directions the minimiser has barely moved along: the step's actual
      // decrease must be below the tolerance too, on two steps in a row
      if (edm_tol_ > 0.0 && iters_ >= n_ && edm() < edm_tol_ && fprev - f < edm_tol_) {
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
      return start_line_search(false);
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
  int evals() const { return evals_; }
  int iterations() const { return iters_; }
  double best_f() const { return f_; }
  // best parameter vector found so far
  void best(double* theta) const {
    for (int i = 0; i < nt_; ++i) theta[i] = th0_[i];
    for (int i = 0; i < n_; ++i) theta[idx_[i]] = th0_[idx_[i]] + sc_[i] * u_[i];
  }
  double grad_norm() const { return gnorm(g_); }
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
  enum Phase { FIRST, SEARCH };

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

  void finish(Status s) { status_ = s; }

  void start_line_search(bool steepest) {
    for (int i = 0; i < n_; ++i) {
      double v = 0.0;
      for (int j = 0; j < n_; ++j) v += H_[i * n_ + j] * g_[j];
      d_[i] = -v;
    }
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
    std::vector<double> Hy(n_);
    for (int i = 0; i < n_; ++i) {
      double v = 0.0;
      for (int j = 0; j < n_; ++j) v += H_[i * n_ + j] * y[j];
      Hy[i] = v;
    }
    const double yHy = dot(y, Hy);
    for (int i = 0; i < n_; ++i)
      for (int j = 0; j < n_; ++j)
        H_[i * n_ + j] += rho * ((1.0 + rho * yHy) * s[i] * s[j] - Hy[i] * s[j] - s[i] * Hy[j]);
  }

  int n_ = 0, nt_ = 0, max_evals_ = 0, evals_ = 0, iters_ = 0, small_ = 0, edm_ok_ = 0;
  bool restarted_ = false;
  double gtol_ = 0.0, ftol_ = 0.0, edm_tol_ = 0.0, f_ = 0.0, alpha_ = 1.0;
  std::vector<double> th0_, sc_, u_, g_, H_, d_, cur_, theta_;
  std::vector<int> idx_;
  Phase phase_ = FIRST;
  Status status_ = RUNNING;
};

}  // namespace mxa
