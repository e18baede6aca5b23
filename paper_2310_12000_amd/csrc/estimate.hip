// Estimation by minimising the Vecchia-Laplace negative log-marginal
// likelihood with its stochastic-trace gradient (Sec. 4.1: L-BFGS with a
// sample average approximation, i.e. the same probe vectors in every
// evaluation, so that the objective is a deterministic function of the
// parameters):
//   vl_estimate      theta = (sigma2, rho) for a fixed offset F;
//   vl_estimate_glm  theta, the likelihood's auxiliary parameter xi (Gaussian
//                    variance, Gamma shape) and beta of F = X beta jointly
//                    (Sec. 5 estimates shape, covariance parameters and beta).
//
// Positive parameters are searched on the log scale.  L-BFGS is the
// two-loop recursion of Nocedal & Wright (Numerical Optimization, Alg. 7.4)
// with the initial matrix scaled by s^T y / y^T y, a backtracking line search
// on the Armijo condition, and curvature pairs kept only when s^T y > 0.
// Every evaluation is vl_set_theta (factor at the new theta, neighbours and
// schedules kept) + vl_find_mode from b = 0 + vl_neg_log_marglik with the
// gradient (+ vl_grad_aux, + X^T dL/dF), all on the device; only the
// d-vector updates of the search (d <= 3 + p) run on the host.
#include <cmath>
#include <deque>
#include <functional>
#include <vector>

#include "vl_internal.h"
#include "vl_laplace.h"

extern "C" {
vl_status vl_set_theta(vl_model* h, const double* theta_host);
vl_status vl_find_mode(vl_model* h, const double* y, const double* F, int lik,
                       const double* aux_host, const vl_opts* o, double* mode_out,
                       vl_stats* st);
vl_status vl_neg_log_marglik(vl_model* h, const vl_opts* o, double* nll_host,
                             double* grad_theta_host, vl_stats* st);
vl_status vl_grad_aux(vl_model* h, double* grad_xi_host);
vl_status vl_grad_beta(vl_model* h, const double* X, int p, double* grad_beta_host);
}

namespace vl {

Model* model_of(vl_model* h);
vl_status report(const Status& s);

namespace {

// f(x) and its gradient; a failure with VL_ERR_NONFINITE or VL_ERR_NOT_SPD
// marks x as outside the domain (the line search backs off).
using Objective = std::function<Status(const std::vector<double>& x, double* f,
                                       std::vector<double>* g)>;

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t k = 0; k < a.size(); ++k) s += a[k] * b[k];
  return s;
}

double max_abs(const std::vector<double>& a) {
  double m = 0.0;
  for (double v : a) m = std::max(m, std::fabs(v));
  return m;
}

// L-BFGS from x (updated in place); f_out = f(x) at the end.
Status lbfgs(const Objective& eval, std::vector<double>& x, int max_iter, double grad_tol,
             double* f_out, int* iters_out, int* evals_out, bool* converged_out) {
  constexpr int kHistory = 10;
  constexpr double kArmijo = 1e-4;
  constexpr int kMaxBacktrack = 30;
  const size_t d = x.size();
  int evals = 0;
  double f = 0.0;
  std::vector<double> g(d);
  ++evals;
  VL_TRY(eval(x, &f, &g));
  std::deque<std::pair<std::vector<double>, std::vector<double>>> hist;  // (s, y)
  int it = 0;
  bool converged = max_abs(g) <= grad_tol;
  while (!converged && it < max_iter) {
    // two-loop recursion: dir = -H g
    std::vector<double> q = g;
    std::vector<double> alpha(hist.size());
    for (int k = static_cast<int>(hist.size()) - 1; k >= 0; --k) {
      const double rho = 1.0 / dot(hist[k].second, hist[k].first);
      alpha[k] = rho * dot(hist[k].first, q);
      for (size_t c = 0; c < d; ++c) q[c] -= alpha[k] * hist[k].second[c];
    }
    double gamma;
    if (!hist.empty()) {
      gamma = dot(hist.back().first, hist.back().second) /
              dot(hist.back().second, hist.back().second);
    } else {  // first step: at most a unit change of the search coordinates
      const double gn = std::sqrt(dot(g, g));
      gamma = gn > 1.0 ? 1.0 / gn : 1.0;
    }
    for (double& v : q) v *= gamma;
    for (size_t k = 0; k < hist.size(); ++k) {
      const double rho = 1.0 / dot(hist[k].second, hist[k].first);
      const double beta = rho * dot(hist[k].second, q);
      for (size_t c = 0; c < d; ++c) q[c] += hist[k].first[c] * (alpha[k] - beta);
    }
    std::vector<double> dir(d);
    for (size_t c = 0; c < d; ++c) dir[c] = -q[c];
    double slope = dot(g, dir);
    if (!(slope < 0.0)) {  // not a descent direction: restart from steepest descent
      hist.clear();
      const double gn = std::sqrt(dot(g, g));
      const double sc = gn > 1.0 ? 1.0 / gn : 1.0;
      for (size_t c = 0; c < d; ++c) dir[c] = -sc * g[c];
      slope = dot(g, dir);
    }
    // backtracking line search on the Armijo condition
    double step = 1.0, fn = 0.0;
    std::vector<double> xt(d), gn(d);
    bool accepted = false;
    for (int b = 0; b < kMaxBacktrack; ++b) {
      for (size_t c = 0; c < d; ++c) xt[c] = x[c] + step * dir[c];
      ++evals;
      Status s = eval(xt, &fn, &gn);
      if (s.good() && fn <= f + kArmijo * step * slope) {
        accepted = true;
        break;
      }
      if (!s.good() && s.code != VL_ERR_NONFINITE && s.code != VL_ERR_NOT_SPD) return s;
      step *= 0.5;
    }
    if (!accepted) {  // no decrease along a descent direction: a minimiser to the
      converged = true;  // objective's smoothness (CG counts change with x)
      break;
    }
    std::vector<double> sv(d), yv(d);
    for (size_t c = 0; c < d; ++c) {
      sv[c] = xt[c] - x[c];
      yv[c] = gn[c] - g[c];
    }
    const double f_old = f;
    x = xt;
    f = fn;
    g = gn;
    ++it;
    if (dot(sv, yv) > 1e-12 * std::sqrt(dot(sv, sv) * dot(yv, yv))) {
      hist.emplace_back(sv, yv);
      if (static_cast<int>(hist.size()) > kHistory) hist.pop_front();
    }
    converged = max_abs(g) <= grad_tol || std::fabs(f_old - f) <= 1e-14 * std::fabs(f);
  }
  *f_out = f;
  *iters_out = it;
  *evals_out = evals;
  *converged_out = converged;
  return Status::ok();
}

Status call(vl_status c, const char* what) {
  if (c == VL_OK || c == VL_ERR_NO_CONVERGENCE) return Status::ok();
  return Status::make(c, what);
}

}  // namespace

// Moves the model to theta = exp(x[0..1]), xi = exp(x[2]) (with an auxiliary
// parameter), F = X beta (beta = x[q..]; F = F0 when p = 0), and evaluates f
// and the gradient in x.
static Status glm_eval(vl_model* h, const double* y, const double* X, int p, const double* F0,
                       int lik, const vl_opts& o, DevBuf<double>& beta_d, DevBuf<double>& F_d,
                       const std::vector<double>& x, double* f, std::vector<double>* g) {
  Model& M = *model_of(h);
  const bool has_aux = lik_has_aux(lik);
  const int q = has_aux ? 3 : 2;
  const double theta[2] = {std::exp(x[0]), std::exp(x[1])};
  const double aux = has_aux ? std::exp(x[2]) : 0.0;
  if (!std::isfinite(theta[0]) || !std::isfinite(theta[1]) || !(theta[0] > 0.0) ||
      !(theta[1] > 0.0) || (has_aux && !(aux > 0.0 && std::isfinite(aux))))
    return Status::make(VL_ERR_NONFINITE, "a parameter left the representable range");
  for (int k = 0; k < p; ++k)
    if (!std::isfinite(x[q + k])) return Status::make(VL_ERR_NONFINITE, "beta not finite");
  const double* F = F0;
  if (p > 0) {
    VL_HIP(hipMemcpyAsync(beta_d.p, x.data() + q, sizeof(double) * p, hipMemcpyHostToDevice,
                          M.stream));
    VL_TRY(xbeta(M, X, p, beta_d.p, F_d.p));
    F = F_d.p;
  }
  VL_TRY(call(vl_set_theta(h, theta), "factor at the trial parameters failed"));
  vl_stats st{};
  VL_TRY(call(vl_find_mode(h, y, F, lik, has_aux ? &aux : nullptr, &o, nullptr, &st),
              "mode at the trial parameters failed"));
  double gt[2] = {0.0, 0.0};
  VL_TRY(call(vl_neg_log_marglik(h, &o, f, gt, &st), "likelihood at the trial parameters failed"));
  g->assign(x.size(), 0.0);
  (*g)[0] = gt[0] * theta[0];  // d/d log theta = theta d/d theta
  (*g)[1] = gt[1] * theta[1];
  if (has_aux) {
    double gx = 0.0;
    VL_TRY(call(vl_grad_aux(h, &gx), "xi-gradient failed"));
    (*g)[2] = gx * aux;
  }
  if (p > 0) VL_TRY(call(vl_grad_beta(h, X, p, g->data() + q), "beta-gradient failed"));
  if (!std::isfinite(*f) || !std::isfinite(max_abs(*g)))
    return Status::make(VL_ERR_NONFINITE, "non-finite likelihood or gradient");
  return Status::ok();
}

static Status estimate_common(vl_model* h, const double* y, const double* X, int p,
                              const double* F0, int lik, const double* aux_fixed,
                              const vl_opts& o, std::vector<double>& x, bool with_aux,
                              int max_iter, double grad_tol, double* nll_out, int* iters_out,
                              int* evals_out) {
  Model& M = *model_of(h);
  if (!M.deriv) return Status::make(VL_ERR_STATE, "the model was built without derivatives");
  if (o.precond != VL_PREC_VADU && o.precond != VL_PREC_LRAC)
    return Status::invalid("the gradient needs the VADU or the LRAC preconditioner");
  if (max_iter < 0) return Status::invalid("max_iter must be >= 0");
  DevBuf<double> beta_d, F_d;
  if (p > 0) {
    VL_TRY(beta_d.alloc(p));
    VL_TRY(F_d.alloc(M.n));
  }
  Objective eval;
  if (with_aux || p > 0) {
    eval = [&](const std::vector<double>& xv, double* f, std::vector<double>* g) {
      return glm_eval(h, y, X, p, F0, lik, o, beta_d, F_d, xv, f, g);
    };
  } else {
    // theta only, the likelihood's auxiliary parameter fixed
    eval = [&](const std::vector<double>& xv, double* f, std::vector<double>* g) -> Status {
      const double theta[2] = {std::exp(xv[0]), std::exp(xv[1])};
      if (!std::isfinite(theta[0]) || !std::isfinite(theta[1]) || !(theta[0] > 0.0) ||
          !(theta[1] > 0.0))
        return Status::make(VL_ERR_NONFINITE, "theta left the representable range");
      VL_TRY(call(vl_set_theta(h, theta), "factor at the trial theta failed"));
      vl_stats st{};
      VL_TRY(call(vl_find_mode(h, y, F0, lik, aux_fixed, &o, nullptr, &st),
                  "mode at the trial theta failed"));
      double gt[2] = {0.0, 0.0};
      VL_TRY(call(vl_neg_log_marglik(h, &o, f, gt, &st), "likelihood at the trial theta failed"));
      g->assign(2, 0.0);
      (*g)[0] = gt[0] * theta[0];
      (*g)[1] = gt[1] * theta[1];
      if (!std::isfinite(*f) || !std::isfinite(max_abs(*g)))
        return Status::make(VL_ERR_NONFINITE, "non-finite likelihood or gradient");
      return Status::ok();
    };
  }
  double f = 0.0;
  int it = 0, evals = 0;
  bool converged = false;
  VL_TRY(lbfgs(eval, x, max_iter, grad_tol, &f, &it, &evals, &converged));
  // leave the model at the returned point (the last evaluation may have been
  // a rejected trial point)
  std::vector<double> gfin;
  ++evals;
  VL_TRY(eval(x, &f, &gfin));
  if (nll_out) *nll_out = f;
  if (iters_out) *iters_out = it;
  if (evals_out) *evals_out = evals;
  if (!converged) return Status::make(VL_ERR_NO_CONVERGENCE, "L-BFGS stopped at its iteration cap");
  return Status::ok();
}

}  // namespace vl

extern "C" vl_status vl_estimate(vl_model* h, const double* y, const double* F, int lik,
                                 const double* aux_host, const vl_opts* o, double* theta_inout,
                                 int max_iter, double grad_tol, double* nll_host,
                                 int* iters_host, int* evals_host) {
  try {
    if (!h || !y || !o || !theta_inout) return vl::report(vl::Status::invalid("null argument"));
    vl::CallStream cs(vl::model_of(h)->stream);
    if (!(theta_inout[0] > 0.0) || !(theta_inout[1] > 0.0))
      return vl::report(vl::Status::invalid("theta must be positive"));
    std::vector<double> x = {std::log(theta_inout[0]), std::log(theta_inout[1])};
    vl::Status s = vl::estimate_common(h, y, nullptr, 0, F, lik, aux_host, *o, x, false,
                                       max_iter, grad_tol, nll_host, iters_host, evals_host);
    if (s.good() || s.code == VL_ERR_NO_CONVERGENCE) {
      theta_inout[0] = std::exp(x[0]);
      theta_inout[1] = std::exp(x[1]);
    }
    return vl::report(s);
  } catch (const std::bad_alloc&) {
    return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}

extern "C" vl_status vl_estimate_glm(vl_model* h, const double* y, const double* X, int p, int lik,
                                     const vl_opts* o, double* params_inout, int max_iter,
                                     double grad_tol, double* nll_host, int* iters_host,
                                     int* evals_host) {
  try {
    if (!h || !y || !o || !params_inout) return vl::report(vl::Status::invalid("null argument"));
    if (p < 0 || (p > 0 && !X)) return vl::report(vl::Status::invalid("X must hold p >= 0 columns"));
    vl::CallStream cs(vl::model_of(h)->stream);
    const bool has_aux = vl::lik_has_aux(lik);
    const int q = has_aux ? 3 : 2;
    double aux0 = 0.0;  // validates the likelihood code and a starting xi > 0
    vl::Status ls = vl::likelihood_aux(lik, has_aux ? params_inout + 2 : nullptr, &aux0);
    if (!ls.good()) return vl::report(ls);
    if (!(params_inout[0] > 0.0) || !(params_inout[1] > 0.0))
      return vl::report(vl::Status::invalid("theta must be positive"));
    std::vector<double> x(q + p);
    for (int k = 0; k < q; ++k) x[k] = std::log(params_inout[k]);
    for (int k = 0; k < p; ++k) x[q + k] = params_inout[q + k];
    vl::Status s = vl::estimate_common(h, y, X, p, nullptr, lik, nullptr, *o, x, has_aux,
                                       max_iter, grad_tol, nll_host, iters_host, evals_host);
    if (s.good() || s.code == VL_ERR_NO_CONVERGENCE) {
      for (int k = 0; k < q; ++k) params_inout[k] = std::exp(x[k]);
      for (int k = 0; k < p; ++k) params_inout[q + k] = x[q + k];
    }
    return vl::report(s);
  } catch (const std::bad_alloc&) {
    return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}
