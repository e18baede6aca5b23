// Estimation of the covariance parameters theta = (sigma2, rho) by
// minimising the Vecchia-Laplace negative log-marginal likelihood with its
// stochastic-trace gradient (Sec. 4.1: L-BFGS with a sample average
// approximation, i.e. the same probe vectors in every evaluation, so that the
// objective is a deterministic function of theta).
//
// The search runs on log theta (both parameters positive).  L-BFGS is the
// two-loop recursion of Nocedal & Wright (Numerical Optimization, Alg. 7.4)
// with the initial matrix scaled by s^T y / y^T y, a backtracking line search
// on the Armijo condition, and curvature pairs kept only when s^T y > 0.
// Every evaluation is vl_set_theta (factor at the new theta, neighbours and
// schedules kept) + vl_find_mode from b = 0 + vl_neg_log_marglik with the
// gradient, all on the device; only the 2-vector updates run on the host.
#include <array>
#include <cmath>
#include <deque>
#include <vector>

#include "vl_internal.h"

extern "C" {
vl_status vl_set_theta(vl_model* h, const double* theta_host);
vl_status vl_find_mode(vl_model* h, const double* y, const double* F, int lik,
                       const double* aux_host, const vl_opts* o, double* mode_out,
                       vl_stats* st);
vl_status vl_neg_log_marglik(vl_model* h, const vl_opts* o, double* nll_host,
                             double* grad_theta_host, vl_stats* st);
}

namespace vl {

Model* model_of(vl_model* h);
vl_status report(const Status& s);

namespace {

struct Eval {
  double f = 0.0;
  double g[2] = {0.0, 0.0};  // gradient in log theta
};

// NLL and its gradient in log theta at theta = exp(x).
Status evaluate(vl_model* h, const double* y, const double* F, int lik, const double* aux,
                const vl_opts& o, const double* x, Eval* e, int* evals) {
  const double theta[2] = {std::exp(x[0]), std::exp(x[1])};
  if (!std::isfinite(theta[0]) || !std::isfinite(theta[1]) || !(theta[0] > 0.0) ||
      !(theta[1] > 0.0))
    return Status::make(VL_ERR_NONFINITE, "theta left the representable range");
  ++*evals;
  vl_status c = vl_set_theta(h, theta);
  if (c != VL_OK) return Status::make(c, "factor at the trial theta failed");
  vl_stats st{};
  c = vl_find_mode(h, y, F, lik, aux, &o, nullptr, &st);
  if (c != VL_OK && c != VL_ERR_NO_CONVERGENCE) return Status::make(c, "mode at the trial theta failed");
  double gt[2] = {0.0, 0.0};
  c = vl_neg_log_marglik(h, &o, &e->f, gt, &st);
  if (c != VL_OK && c != VL_ERR_NO_CONVERGENCE)
    return Status::make(c, "likelihood at the trial theta failed");
  e->g[0] = gt[0] * theta[0];  // d/d log theta = theta d/d theta
  e->g[1] = gt[1] * theta[1];
  if (!std::isfinite(e->f) || !std::isfinite(e->g[0]) || !std::isfinite(e->g[1]))
    return Status::make(VL_ERR_NONFINITE, "non-finite likelihood or gradient");
  return Status::ok();
}

double dot2(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1]; }

}  // namespace

static Status estimate(vl_model* h, const double* y, const double* F, int lik, const double* aux,
                       const vl_opts& o, double* theta, int max_iter, double grad_tol,
                       double* nll_out, int* iters_out, int* evals_out) {
  Model& M = *model_of(h);
  if (!M.deriv) return Status::make(VL_ERR_STATE, "the model was built without derivatives");
  if (o.precond != VL_PREC_VADU) return Status::invalid("the gradient needs the VADU preconditioner");
  if (!(theta[0] > 0.0) || !(theta[1] > 0.0)) return Status::invalid("theta must be positive");
  if (max_iter < 0) return Status::invalid("max_iter must be >= 0");
  constexpr int kHistory = 10;
  constexpr double kArmijo = 1e-4;
  constexpr int kMaxBacktrack = 30;
  double x[2] = {std::log(theta[0]), std::log(theta[1])};
  Eval cur;
  int evals = 0;
  VL_TRY(evaluate(h, y, F, lik, aux, o, x, &cur, &evals));
  std::deque<std::array<double, 4>> hist;  // (s, y) pairs
  int it = 0;
  bool converged = std::max(std::fabs(cur.g[0]), std::fabs(cur.g[1])) <= grad_tol;
  while (!converged && it < max_iter) {
    // two-loop recursion: d = -H g
    double q[2] = {cur.g[0], cur.g[1]};
    std::vector<double> alpha(hist.size());
    for (int k = static_cast<int>(hist.size()) - 1; k >= 0; --k) {
      const double* s = &hist[k][0];
      const double* yv = &hist[k][2];
      const double rho = 1.0 / dot2(yv, s);
      alpha[k] = rho * dot2(s, q);
      q[0] -= alpha[k] * yv[0];
      q[1] -= alpha[k] * yv[1];
    }
    double gamma = 1.0;
    if (!hist.empty()) {
      const double* s = &hist.back()[0];
      const double* yv = &hist.back()[2];
      gamma = dot2(s, yv) / dot2(yv, yv);
    } else {
      // first step: at most a unit change of log theta
      const double gn = std::sqrt(dot2(cur.g, cur.g));
      gamma = gn > 1.0 ? 1.0 / gn : 1.0;
    }
    double r[2] = {gamma * q[0], gamma * q[1]};
    for (size_t k = 0; k < hist.size(); ++k) {
      const double* s = &hist[k][0];
      const double* yv = &hist[k][2];
      const double rho = 1.0 / dot2(yv, s);
      const double beta = rho * dot2(yv, r);
      r[0] += s[0] * (alpha[k] - beta);
      r[1] += s[1] * (alpha[k] - beta);
    }
    double d[2] = {-r[0], -r[1]};
    double slope = dot2(cur.g, d);
    if (!(slope < 0.0)) {  // not a descent direction: restart from steepest descent
      hist.clear();
      const double gn = std::sqrt(dot2(cur.g, cur.g));
      const double sc = gn > 1.0 ? 1.0 / gn : 1.0;
      d[0] = -sc * cur.g[0];
      d[1] = -sc * cur.g[1];
      slope = dot2(cur.g, d);
    }
    // backtracking line search on the Armijo condition
    double step = 1.0;
    Eval next;
    bool accepted = false;
    for (int b = 0; b < kMaxBacktrack; ++b) {
      const double xt[2] = {x[0] + step * d[0], x[1] + step * d[1]};
      Status s = evaluate(h, y, F, lik, aux, o, xt, &next, &evals);
      if (s.good() && next.f <= cur.f + kArmijo * step * slope) {
        accepted = true;
        break;
      }
      if (!s.good() && s.code != VL_ERR_NONFINITE && s.code != VL_ERR_NOT_SPD) return s;
      step *= 0.5;
    }
    if (!accepted) {  // no decrease along a descent direction: a minimiser to the
      converged = true;  // objective's smoothness (CG counts change with theta)
      break;
    }
    const double sv[2] = {step * d[0], step * d[1]};
    const double yv[2] = {next.g[0] - cur.g[0], next.g[1] - cur.g[1]};
    x[0] += sv[0];
    x[1] += sv[1];
    const double f_old = cur.f;
    cur = next;
    ++it;
    if (dot2(sv, yv) > 1e-12 * std::sqrt(dot2(sv, sv) * dot2(yv, yv))) {
      hist.push_back({sv[0], sv[1], yv[0], yv[1]});
      if (static_cast<int>(hist.size()) > kHistory) hist.pop_front();
    }
    converged = std::max(std::fabs(cur.g[0]), std::fabs(cur.g[1])) <= grad_tol ||
                std::fabs(f_old - cur.f) <= 1e-14 * std::fabs(cur.f);
  }
  // leave the model at the returned theta (the last evaluation may have been
  // a rejected trial point)
  Eval fin;
  VL_TRY(evaluate(h, y, F, lik, aux, o, x, &fin, &evals));
  theta[0] = std::exp(x[0]);
  theta[1] = std::exp(x[1]);
  if (nll_out) *nll_out = fin.f;
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
    return vl::report(vl::estimate(h, y, F, lik, aux_host, *o, theta_inout, max_iter, grad_tol,
                                   nll_host, iters_host, evals_host));
  } catch (const std::bad_alloc&) {
    return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}
