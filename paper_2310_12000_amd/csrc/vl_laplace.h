// Host drivers of the Laplace-level operations.
#pragma once

#include "vl_internal.h"

namespace vl {

struct GradInfo {
  double c[2] = {0, 0};
  double dlogdet[2] = {0, 0};
  double quad[2] = {0, 0};
  double implicit[2] = {0, 0};
  int grad_cg_iters = 0;
};

struct NllInfo {
  double gamma = 0, logdet = 0, loglik = 0, quadform = 0;
  int cg_iters_max = 0;
  GradInfo grad;
};

struct PredInfo {
  int cg_iters_max = 0;
};

// LRAC (lrac.hip)
Status lrac_build(Model& M, int k);
Status lrac_factor(Model& M, const double* W);
Status lrac_newton_solve(Model& M, const vl_opts& o, const double* rhs, double* b_out,
                         const int* forced);
Status lrac_slq(Model& M, const vl_opts& o, double* logdet_fixed, const int* forced,
                bool keep_z0 = false);
// For the gradients with P_LRAC: d L_k / d theta (pivots fixed), the
// leverages L_i M^{-1} L_i^T, Y = Sigma~ X, and per probe column the theta
// terms h_k = -(Sigma~ u)^T dSigma~^{-1} (Sigma~ v), r_k = 2 (L^T v).(dL_k^T v)
// with the known means trP_k = 2 tr(M^{-1} L^T W dL_k) (host arrays 2t, 2t, 2).
Status lrac_build_deriv(Model& M);
Status lrac_leverage(Model& M, double* lev);
Status lrac_sigma(Model& M, const double* X, double* Y, double* Tmp, int t);
Status lrac_theta_terms(Model& M, const double* SU, const double* SV, const double* V,
                        const double* W, int t, double* h, double* r, double* trP);

Status lik_rows(Model& M, const double* b, double* g, double* W, double* rhs, double* s,
                double* sq, double* dW);
Status find_mode(Model& M, const vl_opts& o, vl_stats* st);
Status neg_log_marglik(Model& M, const vl_opts& o, double* nll, double* grad, NllInfo* info);
Status predict(Model& M, const double* coords_p, int64_t np, const double* Fp,
               const vl_opts& o, double* mean_out, double* var_out, PredInfo* info);

// Lanczos predictive variances (lanczos.hip) at the test points whose
// neighbours and factor rows predict() has placed in M.pred_*
Status predict_lanczos_var(Model& M, int64_t np, const vl_opts& o, double* var_out,
                           PredInfo* info);

// F = X beta (X device n x p row-major, beta device p, F device n)
Status xbeta(Model& M, const double* X, int p, const double* beta, double* F);

// out (host, p) = X^T dL/dF for F = X beta (X device, n x p row-major)
Status grad_beta(Model& M, const double* X, int p, double* out);

}  // namespace vl
