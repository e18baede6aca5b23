// Vecchia-Laplace quantities on top of the sparse kernels and block CG:
//   Newton mode finding                       eq. (newton), Sec. 2.2
//   SLQ negative log-marginal likelihood      eqs. (VLA_loss), (logdetsplit),
//                                             (def_SLQ); VADU log det P =
//                                             log det(W + D^{-1}) (Sec. 3.1.1)
//   STE theta-gradient with control variates  eq. (grad_STE); App. A.3 and the
//                                             VADU formulas of App. A.4.1
//   predictive means / simulated variances    eq. (latentpostpredictive),
//                                             Alg. simAlgo (Sec. 3.3.1)
#include <algorithm>

#include "vl_internal.h"
#include "vl_ops.h"
#include "vl_laplace.h"

namespace vl {

// ------------------------------------------------------------ likelihoods
__device__ __forceinline__ double sigmoid(double x) { return 0.5 * (1.0 + tanh(0.5 * x)); }

__device__ __forceinline__ double lik_logp(int lik, double y, double mu, double aux) {
  if (lik == VL_LIK_BERNOULLI_LOGIT) {
    // y mu - log(1 + e^mu)
    const double sp = fmax(mu, 0.0) + log1p(exp(-fabs(mu)));
    return y * mu - sp;
  }
  if (lik == VL_LIK_POISSON_LOG) return y * mu - exp(mu) - lgamma(y + 1.0);
  if (lik == VL_LIK_GAMMA) {
    // shape a = aux, rate a e^{-mu} (mean e^mu)
    return aux * log(aux) - lgamma(aux) + (aux - 1.0) * log(y) - aux * mu - aux * y * exp(-mu);
  }
  const double r = y - mu;
  return -0.5 * r * r / aux - 0.5 * log(6.283185307179586 * aux);
}

// g = d log p / d mu, W = -d^2 log p / d mu^2, dW = d W / d mu
__device__ __forceinline__ void lik_derivs(int lik, double y, double mu, double aux, double* g,
                                           double* W, double* dW) {
  if (lik == VL_LIK_BERNOULLI_LOGIT) {
    const double p = sigmoid(mu);
    *g = y - p;
    *W = p * (1.0 - p);
    *dW = p * (1.0 - p) * (1.0 - 2.0 * p);
  } else if (lik == VL_LIK_POISSON_LOG) {
    const double e = exp(mu);
    *g = y - e;
    *W = e;
    *dW = e;
  } else if (lik == VL_LIK_GAMMA) {
    const double ay = aux * y * exp(-mu);
    *g = ay - aux;
    *W = ay;
    *dW = -ay;
  } else {
    *g = (y - mu) / aux;
    *W = 1.0 / aux;
    *dW = 0.0;
  }
}

// Derivatives in the auxiliary parameter xi (Gaussian xi = tau^2, Gamma
// xi = shape a): dlp = d log p / d xi less its row-independent part (the
// Gamma's log a + 1 - digamma(a), added on the host), dg = d^2 log p /
// d xi d mu, dWx = d W / d xi.
__device__ __forceinline__ void lik_xi_derivs(int lik, double y, double mu, double aux,
                                              double* dlp, double* dg, double* dWx) {
  if (lik == VL_LIK_GAMMA) {
    const double ye = y * exp(-mu);
    *dlp = log(y) - mu - ye;
    *dg = ye - 1.0;
    *dWx = ye;
  } else {  // Gaussian
    const double r = y - mu;
    const double it2 = 1.0 / (aux * aux);
    *dlp = 0.5 * r * r * it2 - 0.5 / aux;
    *dg = -r * it2;
    *dWx = -it2;
  }
}

// Per row: g, W, rhs = W b + g, s = 1 / (W + D^{-1}), sq = sqrt(W + D^{-1}),
// dW.  Any output may be null.
__global__ void lik_rows_kernel(int64_t n, int lik, double aux, const double* __restrict__ y,
                                const double* __restrict__ F, const double* __restrict__ b,
                                const double* __restrict__ dinv, double* __restrict__ g_out,
                                double* __restrict__ W_out, double* __restrict__ rhs_out,
                                double* __restrict__ s_out, double* __restrict__ sq_out,
                                double* __restrict__ dW_out, int* __restrict__ status) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double bi = b ? b[i] : 0.0;
  const double mu = (F ? F[i] : 0.0) + bi;
  double g, W, dW;
  lik_derivs(lik, y[i], mu, aux, &g, &W, &dW);
  // a Gamma response must be positive (log y enters the density)
  if (!isfinite(g) || !isfinite(W) || (lik == VL_LIK_GAMMA && !(y[i] > 0.0)))
    raise_error(status, kErrNonfinite);
  if (g_out) g_out[i] = g;
  if (W_out) W_out[i] = W;
  if (rhs_out) rhs_out[i] = W * bi + g;
  const double wd = W + dinv[i];
  if (s_out) s_out[i] = 1.0 / wd;
  if (sq_out) sq_out[i] = sqrt(wd);
  if (dW_out) dW_out[i] = dW;
}

Status lik_rows(Model& M, const double* b, double* g, double* W, double* rhs, double* s,
                double* sq, double* dW) {
  const int tb = 256;
  hipLaunchKernelGGL(lik_rows_kernel, dim3((unsigned)((M.n + tb - 1) / tb)), dim3(tb), 0,
                     M.stream, M.n, M.lik, M.aux, M.y.p, M.F.p, b, M.dinv.p, g, W, rhs, s, sq,
                     dW, M.status);
  return check_launch("likelihood rows");
}

// Sums over rows (t = 1 chunk grid), written as nsum partial arrays:
//   0: log p(y | F + b)   1: D^{-1} (B b)^2   2: log D   3: log(W + D^{-1})
__global__ __launch_bounds__(256) void laplace_terms_kernel(
    ChunkGrid g, int lik, double aux, const double* __restrict__ y,
    const double* __restrict__ F, const double* __restrict__ b, const double* __restrict__ Bb,
    const double* __restrict__ D, const double* __restrict__ W, double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  CHUNK_LOOP_BEGIN(g)
  (void)c;
  const double mu = (F ? F[i] : 0.0) + b[i];
  s0 += lik_logp(lik, y[i], mu, aux);
  const double di = D[i];
  s1 += Bb[i] * Bb[i] / di;
  if (W) {
    s2 += log(di);
    s3 += log(W[i] + 1.0 / di);
  }
  CHUNK_LOOP_END
  block_colsum(g, s0, part);
  block_colsum(g, s1, part + g.nchunk);
  block_colsum(g, s2, part + 2 * g.nchunk);
  block_colsum(g, s3, part + 3 * g.nchunk);
}

// The same per chunk of a row-chunk table (batching form).
__global__ __launch_bounds__(256) void seg_terms_kernel(
    SegArgs a, int nchunk, int lik, double aux, const double* __restrict__ y,
    const double* __restrict__ F, const double* __restrict__ b, const double* __restrict__ Bb,
    const double* __restrict__ D, const double* __restrict__ W, double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  SEG_LOOP_BEGIN(a)
  (void)c;
  const double mu = (F ? F[i] : 0.0) + b[i];
  s0 += lik_logp(lik, y[i], mu, aux);
  const double di = D[i];
  s1 += Bb[i] * Bb[i] / di;
  if (W) {
    s2 += log(di);
    s3 += log(W[i] + 1.0 / di);
  }
  SEG_LOOP_END
  seg_colsum(a, s0, part);
  seg_colsum(a, s1, part + nchunk);
  seg_colsum(a, s2, part + 2 * nchunk);
  seg_colsum(a, s3, part + 3 * nchunk);
}

Status seg_terms_launch(Model& M, SegArgs a, int nchunk, const double* b, const double* Bb,
                        const double* W, double* part) {
  hipLaunchKernelGGL(seg_terms_kernel, dim3(nchunk, 1), dim3(256), 0, M.stream, a, nchunk, M.lik,
                     M.aux, M.y.p, M.F.p, b, Bb, M.dval.p, W, part);
  return check_launch("seg terms");
}

// sums[k] = sum of the k-th partial array (nchunk entries each), in order
__global__ void sum_parts_kernel(const double* __restrict__ part, int nchunk, int nsum,
                                 double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= nsum) return;
  double s = 0.0;
  for (int j = 0; j < nchunk; ++j) s += part[(int64_t)k * nchunk + j];
  out[k] = s;
}

static Status host_sums(Model& M, const double* part, int nchunk, int nsum, double* out) {
  VL_TRY(M.red_out.reserve(64));
  hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, M.stream, part, nchunk, nsum,
                     M.red_out.p);
  VL_TRY(check_launch("sums"));
  VL_HIP(hipMemcpyAsync(out, M.red_out.p, sizeof(double) * nsum, hipMemcpyDeviceToHost,
                        M.stream));
  return sync_stream(M.stream);
}

// log p(y | F + b) summed, and b^T Sigma~^{-1} b = ||D^{-1/2} B b||^2, plus
// (with W) sum log D and sum log(W + D^{-1}).
static Status laplace_terms(Model& M, const double* b, const double* W, double out[4]) {
  VL_TRY(M.vec_d.reserve(M.n));
  VL_TRY(spmm_b(M, b, M.vec_d.p, 1, nullptr));
  ChunkGrid g = ChunkGrid::of(M.n, 1);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * 8));
  hipLaunchKernelGGL(laplace_terms_kernel, dim3(g.nchunk, 1), dim3(256), 0, M.stream, g, M.lik,
                     M.aux, M.y.p, M.F.p, b, M.vec_d.p, M.dval.p, W, M.red_part.p);
  VL_TRY(check_launch("laplace terms"));
  return host_sums(M, M.red_part.p, g.nchunk, 4, out);
}

// ------------------------------------------------------- VADU operators
CgOps vadu_ops(const double* W, const double* sdiag) {
  CgOps ops;
  ops.apply = [W](Model& M, const double* H, double* V, double* Tmp, int t) -> Status {
    // V = W o H + B^T (D^{-1} o (B H))
    VL_TRY(spmm_b(M, H, Tmp, t, M.dinv.p));
    return spmm_bt(M, Tmp, V, t, W, H);
  };
  ops.precond = [sdiag](Model& M, const double* R, double* Z, double* Y, int t) -> Status {
    // Z = B^{-1} ((W + D^{-1})^{-1} o (B^{-T} R))
    VL_TRY(trsm_bt_slot(M, R, Y, t, true, 0));
    return trsm_b_slot(M, Y, Z, t, sdiag, true, 1);
  };
  // the sync-free solves (t <= 64) need the sentinel fill; the level-scheduled
  // ones do not
  ops.needs_fill = [](const Model& M, int t) { return !(t > 64 || M.force_levels); };
  return ops;
}

// ------------------------------------------- LVA and diagonal preconditioners
// (P_1)_ii = (W + B^T D^{-1} B)_ii = W_i + 1/D_i + sum_j B_ji^2 / D_j over the
// entries of row i of B^T (Sec. 3.1.4).  Writes 1/P_1 (s), sqrt(P_1) (sq)
// and P_1 (p); sq and p may be null.
__global__ void p1_diag_kernel(int64_t n, const int* __restrict__ bt_ptr,
                               const int* __restrict__ bt_col, const double* __restrict__ bt_val,
                               const double* __restrict__ W, const double* __restrict__ dinv,
                               double* __restrict__ s_out, double* __restrict__ sq_out,
                               double* __restrict__ p_out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = bt_ptr[i]; k < bt_ptr[i + 1]; ++k) {
    const double v = bt_val[k];
    acc += v * v * dinv[bt_col[k]];
  }
  const double p = W[i] + (dinv[i] + acc);
  s_out[i] = 1.0 / p;
  if (sq_out) sq_out[i] = sqrt(p);
  if (p_out) p_out[i] = p;
}

static Status p1_diag(Model& M, double* s, double* sq, double* p) {
  hipLaunchKernelGGL(p1_diag_kernel, dim3((unsigned)((M.n + 255) / 256)), dim3(256), 0,
                     M.stream, M.n, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, M.W.p, M.dinv.p, s, sq,
                     p);
  return check_launch("P1 diagonal");
}

// Z[i, c] = s_i R[i, c] (n x t row-major)
__global__ void diag_scale_kernel(int64_t n, int t, const double* __restrict__ s,
                                  const double* __restrict__ R, double* __restrict__ Z) {
  const int64_t nt = n * t;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nt;
       e += (int64_t)gridDim.x * blockDim.x)
    Z[e] = s[e / t] * R[e];
}

// out_i = sqrt(in_i) (the LVA probe scale D^{-1/2} from D^{-1})
__global__ void sqrt_kernel(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(in[i]);
}

// sum_i log p_i over a t = 1 chunk grid
__global__ __launch_bounds__(256) void log_sum_kernel(ChunkGrid g, const double* __restrict__ p,
                                                      double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  (void)c;
  acc += log(p[i]);
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

// A as for VADU, P_1^{-1} R = R / P_1 (no triangular solves, no sentinel fill)
static CgOps diag_ops(const double* W, const double* sinv) {
  CgOps ops;
  ops.apply = [W](Model& M, const double* H, double* V, double* Tmp, int t) -> Status {
    VL_TRY(spmm_b(M, H, Tmp, t, M.dinv.p));
    return spmm_bt(M, Tmp, V, t, W, H);
  };
  ops.precond = [sinv](Model& M, const double* R, double* Z, double* Y, int t) -> Status {
    (void)Y;
    const int64_t nt = M.n * static_cast<int64_t>(t);
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((nt + 255) / 256, 8192));
    hipLaunchKernelGGL(diag_scale_kernel, dim3(g), dim3(256), 0, M.stream, M.n, t, sinv, R, Z);
    return check_launch("diagonal preconditioner");
  };
  ops.needs_fill = [](const Model&, int) { return false; };
  return ops;
}

// The operator and preconditioner of eq. (pcls1) at the current W, for
// VADU (sdiag = (W + D^{-1})^{-1}, already in s), LVA (P^{-1} = B^{-1} D
// B^{-T}: sdiag = D) or P_1 (s is overwritten with 1/P_1).
static CgOps pcls1_ops(Model& M, int precond, bool mixed, double* s) {
  if (precond == VL_PREC_DIAG) return diag_ops(M.W.p, s);
  const double* sdiag = precond == VL_PREC_LVA ? M.dval.p : s;
  return mixed ? vadu_ops_mixed(M.W.p, sdiag) : vadu_ops(M.W.p, sdiag);
}

// ------------------------------------------------------------------ mode
constexpr int kMaxHalvings = 30;
constexpr double kHalvingSlack = 1e-12;  // a decrease below this is rounding

// b = b_old + (b - b_old) / 2
__global__ void halve_step_kernel(int64_t n, const double* __restrict__ b_old,
                                  double* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = b_old[i] + 0.5 * (b[i] - b_old[i]);
}

Status find_mode(Model& M, const vl_opts& o, vl_stats* st) {
  const int64_t n = M.n;
  VL_TRY(M.mode.reserve(n));
  VL_TRY(M.W.reserve(n));
  VL_TRY(M.g.reserve(n));
  VL_TRY(M.vec_a.reserve(n));  // rhs
  VL_TRY(M.vec_b.reserve(n));  // (W + D^{-1})^{-1}
  VL_TRY(fill_double(M.mode.p, 0.0, n, M.stream));
  double terms[4];
  VL_TRY(laplace_terms(M, M.mode.p, nullptr, terms));
  double psi_old = terms[0] - 0.5 * terms[1];
  M.newton_cg_iters.clear();
  int it = 0;
  bool converged = false;
  int cg_total = 0, cg_max = 0;
  bool cg_cap = false;
  const bool lrac = o.precond == VL_PREC_LRAC;
  if (lrac) VL_TRY(lrac_build(M, o.lrac_rank));
  VL_TRY(M.mode_old.reserve(n));
  M.newton_halvings.clear();
  for (; it < o.max_newton;) {
    VL_TRY(lik_rows(M, M.mode.p, M.g.p, M.W.p, M.vec_a.p, M.vec_b.p, nullptr, nullptr));
    VL_TRY(copy_d2d(M.mode_old.p, M.mode.p, sizeof(double) * n, M.stream));
    std::vector<int> rbuf;
    const int* forced = replay_slice(o, it, 1, rbuf);  // Newton iteration `it`
    if (lrac) {
      // eq. (pcls2): (Sigma~ + W^{-1}) (W b') = Sigma~ (W b + g)
      VL_TRY(lrac_newton_solve(M, o, M.vec_a.p, M.mode.p, forced));
    } else {
      // eq. (pcls1): (W + Sigma~^{-1}) b' = W b + g with P_VADU, P_LVA or P_1
      if (o.precond == VL_PREC_DIAG) VL_TRY(p1_diag(M, M.vec_b.p, nullptr, nullptr));
      CgOps ops = pcls1_ops(M, o.precond, false, M.vec_b.p);
      VL_TRY(cg_solve(M, M.cg1, ops, 1, M.vec_a.p, o.cg_tol, o.max_cg, false, forced));
      VL_TRY(copy_d2d(M.mode.p, M.cg1.U.p, sizeof(double) * n, M.stream));
    }
    const int ci = M.cg1.host_iters[0];
    M.newton_cg_iters.push_back(ci);
    cg_total += ci;
    if (ci > cg_max) cg_max = ci;
    if (ci >= o.max_cg) cg_cap = true;
    ++it;
    VL_TRY(laplace_terms(M, M.mode.p, nullptr, terms));
    double psi_new = terms[0] - 0.5 * terms[1];
    // step halving while Psi does not increase (the paper gives no step
    // control; full steps diverge e.g. for Poisson counts)
    int halvings = 0;
    const double floor_psi = psi_old - kHalvingSlack * std::fabs(psi_old);  // rounding accepted
    while (halvings < kMaxHalvings && !(psi_new >= floor_psi)) {
      hipLaunchKernelGGL(halve_step_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                         M.stream, n, M.mode_old.p, M.mode.p);
      VL_TRY(check_launch("halve step"));
      VL_TRY(laplace_terms(M, M.mode.p, nullptr, terms));
      psi_new = terms[0] - 0.5 * terms[1];
      ++halvings;
    }
    M.newton_halvings.push_back(halvings);
    if (!(psi_new >= floor_psi)) {  // no increase even after halving: keep b
      VL_TRY(copy_d2d(M.mode.p, M.mode_old.p, sizeof(double) * n, M.stream));
      converged = true;
      break;
    }
    if (std::fabs(psi_new - psi_old) <= o.newton_tol * std::fabs(psi_old)) {
      converged = true;
      break;
    }
    psi_old = psi_new;
  }
  // W at the mode
  VL_TRY(lik_rows(M, M.mode.p, M.g.p, M.W.p, nullptr, nullptr, nullptr, nullptr));
  VL_TRY(read_status(M));
  M.has_mode = true;
  if (st) {
    st->newton_iters = it;
    st->cg_iters_total = cg_total;
    st->cg_iters_max = cg_max;
    st->hit_cap = (!converged || cg_cap) ? 1 : 0;
  }
  if (!converged || cg_cap)
    return Status::make(VL_ERR_NO_CONVERGENCE, "Newton or CG stopped at its iteration cap");
  return Status::ok();
}

// ----------------------------------------------------------- gradient
// Per probe column c (t <= 64, one wave covers whole rows): with u = A^{-1} z,
// v = P^{-1} z, Bu, Bv, dBu, dBv gathered once per row:
//   h_rho = dBu' D^{-1} Bv + Bu' D^{-1} dBv - Bu' D^{-2} dD_rho Bv
//   r_rho = 2 dBv' (W + D^{-1}) Bv - Bv' D^{-2} dD_rho Bv
//   h_s2  = -Bu' D^{-2} dD_s2 Bv,   r_s2 = -Bv' D^{-2} dD_s2 Bv    (dB_s2 = 0)
// and per row i the mu-derivative of the log-determinant (App. A.4.1):
//   h_ic = dW_i u_ic v_ic,  r_ic = dW_i (B v)_ic^2,
//   dlogdet/dmu_i = c_i dW_i / (W_i + 1/D_i) + mean_c (h_ic - c_i r_ic),
// with c_i = Cov_c(h, r) / Var_c(r) (0 when Var_c(r) <= 1e-10 mean_c(r)^2);
// dLdb_i = dlogdet/dmu_i / 2.  With dWx (d W / d xi, nullable) also the
// xi-terms summed over rows: h_xi = u' dWx v, r_xi = (Bv)' dWx (Bv).
__global__ __launch_bounds__(256) void grad_probe_kernel(
    ChunkGrid g, int m, const int* __restrict__ nbr, const double* __restrict__ bval,
    const double* __restrict__ dbval, const double* __restrict__ U,
    const double* __restrict__ V, const double* __restrict__ D,
    const double* __restrict__ dd_s2, const double* __restrict__ dd_rho,
    const double* __restrict__ W, const double* __restrict__ dW,
    const double* __restrict__ dWx, double* __restrict__ dLdb, double* __restrict__ part) {
  double h0 = 0.0, r0 = 0.0, h1 = 0.0, r1 = 0.0, hx = 0.0, rx = 0.0;
  const int t = g.t;
  const int lpr = 1 << g.L.lpr_log;
  const int lane = threadIdx.x & 63;
  const int c = lane & (lpr - 1);
  const int _w = threadIdx.x >> 6;
  const int _sub = lane >> g.L.lpr_log;
  const int64_t r0w = (int64_t)blockIdx.x * g.rpc;
  int64_t r1w = r0w + g.rpc;
  if (r1w > g.n) r1w = g.n;
  const int64_t step = 4LL << g.L.rpw_log;
  for (int64_t base = r0w + ((int64_t)_w << g.L.rpw_log); base < r1w; base += step) {
    const int64_t i = base + _sub;
    const bool valid = (i < r1w) && (c < t);
    double hm = 0.0, rm = 0.0;
    double wd = 1.0, dWi = 0.0;
    if (valid) {
      const int* nb = nbr + i * m;
      const double* bv = bval + i * m;
      const double* dbv = dbval + i * m;
      const double ui = U[i * t + c], vi = V[i * t + c];
      double Bu = ui, Bv = vi, dBu = 0.0, dBv = 0.0;
      for (int k = 0; k < m; ++k) {
        const int j = nb[k];
        if (j < 0) break;
        const double uj = U[(int64_t)j * t + c], vj = V[(int64_t)j * t + c];
        Bu += bv[k] * uj;
        Bv += bv[k] * vj;
        dBu += dbv[k] * uj;
        dBv += dbv[k] * vj;
      }
      const double di = 1.0 / D[i];
      const double di2 = di * di;
      wd = W[i] + di;
      dWi = dW[i];
      h1 += dBu * di * Bv + Bu * di * dBv - Bu * di2 * dd_rho[i] * Bv;
      r1 += 2.0 * dBv * wd * Bv - Bv * di2 * dd_rho[i] * Bv;
      h0 += -Bu * di2 * dd_s2[i] * Bv;
      r0 += -Bv * di2 * dd_s2[i] * Bv;
      hm = dWi * ui * vi;
      rm = dWi * Bv * Bv;
      if (dWx) {
        const double dx = dWx[i];
        hx += dx * ui * vi;
        rx += dx * Bv * Bv;
      }
    }
    // per-row moments over the t columns held by the lpr lanes of this row
    double sh = hm, sr = rm;
    for (int o = 1; o < lpr; o <<= 1) {
      sh += __shfl_xor(sh, o);
      sr += __shfl_xor(sr, o);
    }
    const double mh = sh / t, mr = sr / t;
    double vr = valid ? (rm - mr) * (rm - mr) : 0.0;
    double cv = valid ? (hm - mh) * (rm - mr) : 0.0;
    for (int o = 1; o < lpr; o <<= 1) {
      vr += __shfl_xor(vr, o);
      cv += __shfl_xor(cv, o);
    }
    if (valid && c == 0) {
      vr /= (t - 1);
      cv /= (t - 1);
      const double cc = (vr > 1e-10 * mr * mr) ? cv / vr : 0.0;
      dLdb[i] = 0.5 * (cc * dWi / wd + (mh - cc * mr));
    }
  }
  block_colsum(g, h0, part);
  block_colsum(g, r0, part + (int64_t)g.nchunk * t);
  block_colsum(g, h1, part + 2 * (int64_t)g.nchunk * t);
  block_colsum(g, r1, part + 3 * (int64_t)g.nchunk * t);
  if (dWx) {
    block_colsum(g, hx, part + 4 * (int64_t)g.nchunk * t);
    block_colsum(g, rx, part + 5 * (int64_t)g.nchunk * t);
  }
}

// LRAC form of the mu- and xi-terms (App. "Preconditioner LRAC"), per probe
// column c, with u = (Sigma~ + W^{-1})^{-1} z, v = P^{-1} z:
//   h_ic = dW_i u_ic v_ic / W_i^2,  r_ic = dW_i v_ic^2 / W_i^2,
//   dlogdet/dmu_i = dW_i / W_i + c_i (dW_i lev_i - dW_i / W_i) - mean_c(h - c_i r),
// dLdb_i = dlogdet/dmu_i / 2; with dWx (nullable) the xi sums over rows
// h_xi = sum_i dWx_i u_i v_i / W_i^2, r_xi = sum_i dWx_i v_i^2 / W_i^2.
__global__ __launch_bounds__(256) void lrac_mu_kernel(
    ChunkGrid g, const double* __restrict__ U, const double* __restrict__ V,
    const double* __restrict__ W, const double* __restrict__ dW, const double* __restrict__ lev,
    const double* __restrict__ dWx, double* __restrict__ dLdb, double* __restrict__ part) {
  double hx = 0.0, rx = 0.0;
  const int t = g.t;
  const int lpr = 1 << g.L.lpr_log;
  const int lane = threadIdx.x & 63;
  const int c = lane & (lpr - 1);
  const int _w = threadIdx.x >> 6;
  const int _sub = lane >> g.L.lpr_log;
  const int64_t r0w = (int64_t)blockIdx.x * g.rpc;
  int64_t r1w = r0w + g.rpc;
  if (r1w > g.n) r1w = g.n;
  const int64_t step = 4LL << g.L.rpw_log;
  for (int64_t base = r0w + ((int64_t)_w << g.L.rpw_log); base < r1w; base += step) {
    const int64_t i = base + _sub;
    const bool valid = (i < r1w) && (c < t);
    double hm = 0.0, rm = 0.0, Wi = 1.0, dWi = 0.0;
    if (valid) {
      const double ui = U[i * t + c], vi = V[i * t + c];
      Wi = W[i];
      dWi = dW[i];
      const double wi2 = 1.0 / (Wi * Wi);
      hm = dWi * wi2 * ui * vi;
      rm = dWi * wi2 * vi * vi;
      if (dWx) {
        const double dx = dWx[i] * wi2;
        hx += dx * ui * vi;
        rx += dx * vi * vi;
      }
    }
    double sh = hm, sr = rm;
    for (int o = 1; o < lpr; o <<= 1) {
      sh += __shfl_xor(sh, o);
      sr += __shfl_xor(sr, o);
    }
    const double mh = sh / t, mr = sr / t;
    double vr = valid ? (rm - mr) * (rm - mr) : 0.0;
    double cv = valid ? (hm - mh) * (rm - mr) : 0.0;
    for (int o = 1; o < lpr; o <<= 1) {
      vr += __shfl_xor(vr, o);
      cv += __shfl_xor(cv, o);
    }
    if (valid && c == 0) {
      vr /= (t - 1);
      cv /= (t - 1);
      const double cc = (vr > 1e-10 * mr * mr) ? cv / vr : 0.0;
      const double tw = dWi / Wi;
      dLdb[i] = 0.5 * (tw + cc * (dWi * lev[i] - tw) - (mh - cc * mr));
    }
  }
  if (dWx) {
    block_colsum(g, hx, part);
    block_colsum(g, rx, part + (int64_t)g.nchunk * t);
  }
}

// Row sums (t = 1 grid) of the LRAC xi traces: sum dWx / W, sum dWx lev.
__global__ __launch_bounds__(256) void lrac_xi_rows_kernel(ChunkGrid g,
                                                           const double* __restrict__ dWx,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ lev,
                                                           double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0;
  CHUNK_LOOP_BEGIN(g)
  (void)c;
  s0 += dWx[i] / W[i];
  s1 += dWx[i] * lev[i];
  CHUNK_LOOP_END
  block_colsum(g, s0, part);
  block_colsum(g, s1, part + g.nchunk);
}

// d W / d xi per row at the mode (input of grad_probe_kernel).
__global__ void xi_dw_kernel(int64_t n, int lik, double aux, const double* __restrict__ y,
                             const double* __restrict__ F, const double* __restrict__ b,
                             double* __restrict__ dWx) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double dlp, dg, dw;
  lik_xi_derivs(lik, y[i], (F ? F[i] : 0.0) + b[i], aux, &dlp, &dg, &dw);
  dWx[i] = dw;
}

// Row sums (t = 1 grid) for the xi-gradient: 0: sum dlp, 1: sum dWx / (W +
// D^{-1}) (= tr(P^{-1} dP/dxi)), 2: w' dg with w = A^{-1} dL/db.
__global__ __launch_bounds__(256) void grad_xi_rows_kernel(
    ChunkGrid g, int lik, double aux, const double* __restrict__ y,
    const double* __restrict__ F, const double* __restrict__ b, const double* __restrict__ W,
    const double* __restrict__ D, const double* __restrict__ w, double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  CHUNK_LOOP_BEGIN(g)
  (void)c;
  double dlp, dg, dw;
  lik_xi_derivs(lik, y[i], (F ? F[i] : 0.0) + b[i], aux, &dlp, &dg, &dw);
  s0 += dlp;
  s1 += dw / (W[i] + 1.0 / D[i]);
  s2 += w[i] * dg;
  CHUNK_LOOP_END
  block_colsum(g, s0, part);
  block_colsum(g, s1, part + g.nchunk);
  block_colsum(g, s2, part + 2 * g.nchunk);
}

// digamma(x) for x > 0: the recurrence psi(x) = psi(x + 1) - 1/x up to
// x >= 10, then the asymptotic series ln x - 1/(2x) - sum_k B_2k / (2k
// x^2k) through k = 6 (Abramowitz & Stegun 6.3.5 and 6.3.18); the first
// omitted term is below 1e-16 there.
static double digamma_host(double x) {
  double acc = 0.0;
  while (x < 10.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double i2 = 1.0 / (x * x);
  // B_2k / (2k) for k = 1..6: 1/12, -1/120, 1/252, -1/240, 1/132, -691/32760
  const double series =
      i2 * (1.0 / 12 -
            i2 * (1.0 / 120 -
                  i2 * (1.0 / 252 - i2 * (1.0 / 240 - i2 * (1.0 / 132 - i2 * (691.0 / 32760))))));
  return acc + std::log(x) - 0.5 / x - series;
}

// Row sums (t = 1 grid) for the explicit and implicit theta-terms:
// for k in {sigma2, rho}:
//   quad_k = 2 dBb' D^{-1} Bb - Bb' D^{-2} dD_k Bb        (= b' dSigma~^{-1} b)
//   impl_k = -(dBw' D^{-1} Bb + Bw' D^{-1} dBb - Bw' D^{-2} dD_k Bb)
//   trD_k  = sum dD_k / D,   trP_k = -sum D^{-2} dD_k / (W + D^{-1})
__global__ __launch_bounds__(256) void grad_rows_kernel(
    ChunkGrid g, int m, const int* __restrict__ nbr, const double* __restrict__ bval,
    const double* __restrict__ dbval, const double* __restrict__ b,
    const double* __restrict__ wv, const double* __restrict__ D,
    const double* __restrict__ dd_s2, const double* __restrict__ dd_rho,
    const double* __restrict__ W, double* __restrict__ part) {
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  CHUNK_LOOP_BEGIN(g)
  (void)c;
  const int* nb = nbr + i * m;
  const double* bv = bval + i * m;
  const double* dbv = dbval + i * m;
  double Bb = b[i], Bw = wv[i], dBb = 0.0, dBw = 0.0;
  for (int k = 0; k < m; ++k) {
    const int j = nb[k];
    if (j < 0) break;
    Bb += bv[k] * b[j];
    Bw += bv[k] * wv[j];
    dBb += dbv[k] * b[j];
    dBw += dbv[k] * wv[j];
  }
  const double di = 1.0 / D[i];
  const double di2 = di * di;
  const double wd = W[i] + di;
  const double d0 = dd_s2[i], d1 = dd_rho[i];
  // sigma2: dB = 0
  acc[0] += -Bb * di2 * d0 * Bb;
  acc[1] += Bw * di2 * d0 * Bb;
  acc[2] += d0 * di;
  acc[3] += -di2 * d0 / wd;
  // rho
  acc[4] += 2.0 * dBb * di * Bb - Bb * di2 * d1 * Bb;
  acc[5] += -(dBw * di * Bb + Bw * di * dBb - Bw * di2 * d1 * Bb);
  acc[6] += d1 * di;
  acc[7] += -di2 * d1 / wd;
  CHUNK_LOOP_END
  for (int k = 0; k < 8; ++k) block_colsum(g, acc[k], part + (int64_t)k * g.nchunk);
}

static double cv_weight(const std::vector<double>& h, const std::vector<double>& r) {
  const size_t t = h.size();
  double mh = 0.0, mr = 0.0;
  for (size_t c = 0; c < t; ++c) {
    mh += h[c];
    mr += r[c];
  }
  mh /= t;
  mr /= t;
  double vr = 0.0, cv = 0.0;
  for (size_t c = 0; c < t; ++c) {
    vr += (r[c] - mr) * (r[c] - mr);
    cv += (h[c] - mh) * (r[c] - mr);
  }
  vr /= (t - 1);
  cv /= (t - 1);
  return (vr > 1e-10 * mr * mr) ? cv / vr : 0.0;
}

// d L / d F = -g + dL/db - W o w, w = A^{-1} dL/db (the mode's response to
// the offset, App. "Gradients of Vecchia-Laplace approximations").
__global__ void grad_offset_kernel(int64_t n, const double* __restrict__ g,
                                   const double* __restrict__ dLdb, const double* __restrict__ W,
                                   const double* __restrict__ w, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (dLdb[i] - g[i]) - W[i] * w[i];
}

// Partial sums of X^T v over the chunks of rows (X n x p row-major).
__global__ __launch_bounds__(256) void xt_vec_kernel(ChunkGrid g, const double* __restrict__ X,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  acc += X[i * g.t + c] * v[i];
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

// F = X beta (X n x p row-major, beta device p)
__global__ void xbeta_kernel(int64_t n, int p, const double* __restrict__ X,
                             const double* __restrict__ beta, double* __restrict__ F) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < p; ++k) acc += X[i * p + k] * beta[k];
  F[i] = acc;
}

Status xbeta(Model& M, const double* X, int p, const double* beta, double* F) {
  hipLaunchKernelGGL(xbeta_kernel, dim3((unsigned)((M.n + 255) / 256)), dim3(256), 0, M.stream,
                     M.n, p, X, beta, F);
  return check_launch("X beta");
}

// out (host, p) = X^T grad_F: the gradient in beta when F = X beta.
Status grad_beta(Model& M, const double* X, int p, double* out) {
  if (!M.has_grad_F)
    return Status::make(VL_ERR_STATE, "no offset gradient: call vl_neg_log_marglik with a gradient");
  if (p < 1) return Status::invalid("p must be positive");
  ChunkGrid g = ChunkGrid::of(M.n, p);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * p + 64));
  VL_TRY(M.red_out.reserve(static_cast<size_t>(p) + 64));
  hipLaunchKernelGGL(xt_vec_kernel, dim3(g.nchunk, g.L.slices), dim3(256), 0, M.stream, g, X,
                     M.grad_F.p, M.red_part.p);
  VL_TRY(reduce_chunks(M.stream, M.red_part.p, g.nchunk, p, M.red_out.p));
  VL_HIP(hipMemcpyAsync(out, M.red_out.p, sizeof(double) * p, hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  return read_status(M);
}

static Status grad_theta(Model& M, const vl_opts& o, const double* sdiag, double* grad,
                         GradInfo* info) {
  const int t = M.cg.t;
  const int64_t n = M.n;
  if (t > 64) return Status::invalid("the gradient supports at most 64 probes");
  if (t < 2) return Status::invalid("the gradient needs at least 2 probes");
  VL_TRY(M.vec_c.reserve(n));   // dL/db
  VL_TRY(M.dWv.reserve(n));
  VL_TRY(lik_rows(M, M.mode.p, nullptr, nullptr, nullptr, nullptr, nullptr, M.dWv.p));
  const bool xi = lik_has_aux(M.lik);
  if (xi) {
    VL_TRY(M.vec_d.reserve(n));  // d W / d xi
    hipLaunchKernelGGL(xi_dw_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, M.stream,
                       n, M.lik, M.aux, M.y.p, M.F.p, M.mode.p, M.vec_d.p);
    VL_TRY(check_launch("xi dW"));
  }
  const int nblk = xi ? 6 : 4;
  ChunkGrid g = ChunkGrid::of(n, t);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * t * nblk + 64));
  hipLaunchKernelGGL(grad_probe_kernel, dim3(g.nchunk, 1), dim3(256), 0, M.stream, g, M.m,
                     M.nbr.p, M.bval.p, M.dbval_rho.p, M.cg.U.p, M.cg.Z0.p, M.dval.p,
                     M.dd_sigma2.p, M.dd_rho.p, M.W.p, M.dWv.p, xi ? M.vec_d.p : nullptr,
                     M.vec_c.p, M.red_part.p);
  VL_TRY(check_launch("grad probes"));
  VL_TRY(M.red_out.reserve(nblk * t + 64));
  for (int k = 0; k < nblk; ++k)
    VL_TRY(reduce_chunks(M.stream, M.red_part.p + (int64_t)k * g.nchunk * t, g.nchunk, t,
                         M.red_out.p + k * t));
  std::vector<double> hr(nblk * t);
  VL_HIP(hipMemcpyAsync(hr.data(), M.red_out.p, sizeof(double) * nblk * t,
                        hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  // w = A^{-1} dL/db  (implicit derivative of the mode, eq. grad_mode_par)
  CgOps ops = vadu_ops(M.W.p, sdiag);
  std::vector<int> rbuf;
  VL_TRY(cg_solve(M, M.cg1, ops, 1, M.vec_c.p, o.cg_tol, o.max_cg, false,
                  replay_slice(o, t, 1, rbuf)));  // entry t: after the probe columns
  info->grad_cg_iters = M.cg1.host_iters[0];
  VL_TRY(M.grad_F.reserve(n));
  hipLaunchKernelGGL(grad_offset_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     M.stream, n, M.g.p, M.vec_c.p, M.W.p, M.cg1.U.p, M.grad_F.p);
  VL_TRY(check_launch("grad offset"));
  M.has_grad_F = true;
  ChunkGrid g1 = ChunkGrid::of(n, 1);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g1.nchunk) * 8 + 64));
  hipLaunchKernelGGL(grad_rows_kernel, dim3(g1.nchunk, 1), dim3(256), 0, M.stream, g1, M.m,
                     M.nbr.p, M.bval.p, M.dbval_rho.p, M.mode.p, M.cg1.U.p, M.dval.p,
                     M.dd_sigma2.p, M.dd_rho.p, M.W.p, M.red_part.p);
  VL_TRY(check_launch("grad rows"));
  double rows[8];
  VL_TRY(host_sums(M, M.red_part.p, g1.nchunk, 8, rows));
  for (int k = 0; k < 2; ++k) {
    std::vector<double> h(hr.begin() + (2 * k) * t, hr.begin() + (2 * k + 1) * t);
    std::vector<double> r(hr.begin() + (2 * k + 1) * t, hr.begin() + (2 * k + 2) * t);
    const double c = cv_weight(h, r);
    double mean = 0.0;
    for (int q = 0; q < t; ++q) mean += h[q] - c * r[q];
    mean /= t;
    const double quad = rows[4 * k + 0], impl = rows[4 * k + 1];
    const double trD = rows[4 * k + 2], trP = rows[4 * k + 3];
    const double dlogdet = trD + c * trP + mean;
    grad[k] = 0.5 * quad + 0.5 * dlogdet + impl;
    info->c[k] = c;
    info->dlogdet[k] = dlogdet;
    info->quad[k] = quad;
    info->implicit[k] = impl;
  }
  M.has_grad_xi = false;
  if (xi) {
    // d L / d xi = -d log p / d xi + (1/2) d log det / d xi + w' d^2 log p /
    // d xi d mu, the log-determinant term by the VADU STE with control variate
    ChunkGrid gx = ChunkGrid::of(n, 1);
    VL_TRY(M.red_part.reserve(static_cast<size_t>(gx.nchunk) * 3 + 64));
    hipLaunchKernelGGL(grad_xi_rows_kernel, dim3(gx.nchunk, 1), dim3(256), 0, M.stream, gx,
                       M.lik, M.aux, M.y.p, M.F.p, M.mode.p, M.W.p, M.dval.p, M.cg1.U.p,
                       M.red_part.p);
    VL_TRY(check_launch("grad xi rows"));
    double xr[3];
    VL_TRY(host_sums(M, M.red_part.p, gx.nchunk, 3, xr));
    std::vector<double> h(hr.begin() + 4 * t, hr.begin() + 5 * t);
    std::vector<double> r(hr.begin() + 5 * t, hr.begin() + 6 * t);
    const double c = cv_weight(h, r);
    double mean = 0.0;
    for (int q = 0; q < t; ++q) mean += h[q] - c * r[q];
    mean /= t;
    double dlogp = xr[0];
    if (M.lik == VL_LIK_GAMMA)
      dlogp += static_cast<double>(n) * (std::log(M.aux) + 1.0 - digamma_host(M.aux));
    const double dlogdet = c * xr[1] + mean;
    M.grad_xi = -dlogp + 0.5 * dlogdet + xr[2];
    M.has_grad_xi = true;
  }
  return Status::ok();
}

// Gradients with P_LRAC (App. "Gradients of Vecchia-Laplace approximations"
// with the STE formulas of App. "Preconditioner LRAC"): theta, the offset F
// and, for a likelihood with one, xi.  The probe solves u = (Sigma~ +
// W^{-1})^{-1} z and v = P^{-1} z come from the SLQ block of the same call;
// the mode's response w = A^{-1} dL/db = W^{-1} (Sigma~ + W^{-1})^{-1} Sigma~
// dL/db (eq. pcls2).
static Status grad_lrac(Model& M, const vl_opts& o, double* grad, GradInfo* info) {
  const int t = M.cg.t;
  const int64_t n = M.n;
  if (t > 64) return Status::invalid("the gradient supports at most 64 probes");
  if (t < 2) return Status::invalid("the gradient needs at least 2 probes");
  VL_TRY(lrac_build_deriv(M));
  VL_TRY(M.dWv.reserve(n));
  VL_TRY(lik_rows(M, M.mode.p, nullptr, nullptr, nullptr, nullptr, nullptr, M.dWv.p));
  const bool xi = lik_has_aux(M.lik);
  DevBuf<double> lev, dWx, w, SU, SV, tmp;
  VL_TRY(lev.alloc(n));
  VL_TRY(lrac_leverage(M, lev.p));
  if (xi) {
    VL_TRY(dWx.alloc(n));
    hipLaunchKernelGGL(xi_dw_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, M.stream,
                       n, M.lik, M.aux, M.y.p, M.F.p, M.mode.p, dWx.p);
    VL_TRY(check_launch("xi dW"));
  }
  VL_TRY(M.vec_c.reserve(n));  // dL/db
  ChunkGrid g = ChunkGrid::of(n, t);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * t * 2 + 64));
  hipLaunchKernelGGL(lrac_mu_kernel, dim3(g.nchunk, 1), dim3(256), 0, M.stream, g, M.cg.U.p,
                     M.cg.Z0.p, M.W.p, M.dWv.p, lev.p, xi ? dWx.p : nullptr, M.vec_c.p,
                     M.red_part.p);
  VL_TRY(check_launch("lrac mu"));
  std::vector<double> hx(t), rx(t);
  if (xi) {
    VL_TRY(M.red_out.reserve(2 * static_cast<size_t>(t) + 64));
    for (int q = 0; q < 2; ++q)
      VL_TRY(reduce_chunks(M.stream, M.red_part.p + (int64_t)q * g.nchunk * t, g.nchunk, t,
                           M.red_out.p + q * t));
    VL_HIP(hipMemcpyAsync(hx.data(), M.red_out.p, sizeof(double) * t, hipMemcpyDeviceToHost,
                          M.stream));
    VL_HIP(hipMemcpyAsync(rx.data(), M.red_out.p + t, sizeof(double) * t,
                          hipMemcpyDeviceToHost, M.stream));
  }
  // theta terms from Sigma~ u, Sigma~ v (before the implicit solve reuses
  // the CG scratch)
  const size_t nt = static_cast<size_t>(n) * t;
  VL_TRY(SU.alloc(nt));
  VL_TRY(SV.alloc(nt));
  VL_TRY(tmp.alloc(nt));
  VL_TRY(lrac_sigma(M, M.cg.U.p, SU.p, tmp.p, t));
  VL_TRY(lrac_sigma(M, M.cg.Z0.p, SV.p, tmp.p, t));
  std::vector<double> h(2 * t), r(2 * t);
  double trP[2];
  VL_TRY(lrac_theta_terms(M, SU.p, SV.p, M.cg.Z0.p, M.W.p, t, h.data(), r.data(), trP));
  SU.release();
  SV.release();
  tmp.release();
  // w = A^{-1} dL/db by eq. (pcls2)
  VL_TRY(w.alloc(n));
  std::vector<int> rbuf;
  VL_TRY(lrac_newton_solve(M, o, M.vec_c.p, w.p, replay_slice(o, t, 1, rbuf)));
  info->grad_cg_iters = M.cg1.host_iters[0];
  VL_TRY(M.grad_F.reserve(n));
  hipLaunchKernelGGL(grad_offset_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     M.stream, n, M.g.p, M.vec_c.p, M.W.p, w.p, M.grad_F.p);
  VL_TRY(check_launch("grad offset"));
  M.has_grad_F = true;
  // b*^T dSigma~^{-1} b* and -w^T dSigma~^{-1} b* (the VADU row sums serve)
  ChunkGrid g1 = ChunkGrid::of(n, 1);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g1.nchunk) * 8 + 64));
  hipLaunchKernelGGL(grad_rows_kernel, dim3(g1.nchunk, 1), dim3(256), 0, M.stream, g1, M.m,
                     M.nbr.p, M.bval.p, M.dbval_rho.p, M.mode.p, w.p, M.dval.p,
                     M.dd_sigma2.p, M.dd_rho.p, M.W.p, M.red_part.p);
  VL_TRY(check_launch("grad rows"));
  double rows[8];
  VL_TRY(host_sums(M, M.red_part.p, g1.nchunk, 8, rows));
  for (int k = 0; k < 2; ++k) {
    std::vector<double> hk(h.begin() + k * t, h.begin() + (k + 1) * t);
    std::vector<double> rk(r.begin() + k * t, r.begin() + (k + 1) * t);
    const double c = cv_weight(hk, rk);
    double mean = 0.0;
    for (int q = 0; q < t; ++q) mean += hk[q] - c * rk[q];
    mean /= t;
    const double quad = rows[4 * k + 0], impl = rows[4 * k + 1];
    const double dlogdet = c * trP[k] + mean;
    grad[k] = 0.5 * quad + 0.5 * dlogdet + impl;
    info->c[k] = c;
    info->dlogdet[k] = dlogdet;
    info->quad[k] = quad;
    info->implicit[k] = impl;
  }
  M.has_grad_xi = false;
  if (xi) {
    ChunkGrid gx = ChunkGrid::of(n, 1);
    VL_TRY(M.red_part.reserve(static_cast<size_t>(gx.nchunk) * 3 + 64));
    hipLaunchKernelGGL(grad_xi_rows_kernel, dim3(gx.nchunk, 1), dim3(256), 0, M.stream, gx,
                       M.lik, M.aux, M.y.p, M.F.p, M.mode.p, M.W.p, M.dval.p, w.p, M.red_part.p);
    VL_TRY(check_launch("grad xi rows"));
    double xr[3];
    VL_TRY(host_sums(M, M.red_part.p, gx.nchunk, 3, xr));
    hipLaunchKernelGGL(lrac_xi_rows_kernel, dim3(gx.nchunk, 1), dim3(256), 0, M.stream, gx, dWx.p,
                       M.W.p, lev.p, M.red_part.p);
    VL_TRY(check_launch("lrac xi rows"));
    double lr[2];
    VL_TRY(host_sums(M, M.red_part.p, gx.nchunk, 2, lr));
    const double c = cv_weight(hx, rx);
    double mean = 0.0;
    for (int q = 0; q < t; ++q) mean += hx[q] - c * rx[q];
    mean /= t;
    double dlogp = xr[0];
    if (M.lik == VL_LIK_GAMMA)
      dlogp += static_cast<double>(n) * (std::log(M.aux) + 1.0 - digamma_host(M.aux));
    const double dlogdet = lr[0] + c * (lr[1] - lr[0]) - mean;
    M.grad_xi = -dlogp + 0.5 * dlogdet + xr[2];
    M.has_grad_xi = true;
  }
  return Status::ok();
}

// -------------------------------------------------------------- NLL (SLQ)
Status neg_log_marglik(Model& M, const vl_opts& o, double* nll, double* grad, NllInfo* info) {
  if (!M.has_mode) return Status::make(VL_ERR_STATE, "no mode: call vl_find_mode first");
  M.has_grad_F = false;
  M.has_grad_xi = false;
  if (grad && !M.deriv) return Status::make(VL_ERR_STATE, "model built without derivatives");
  const int64_t n = M.n;
  const int t = o.num_probes;
  if (t < 1) return Status::invalid("num_probes must be positive");
  VL_TRY(M.vec_a.reserve(n));  // sqrt(W + D^{-1})
  VL_TRY(M.vec_b.reserve(n));  // (W + D^{-1})^{-1}
  VL_TRY(lik_rows(M, M.mode.p, nullptr, M.W.p, nullptr, M.vec_b.p, M.vec_a.p, nullptr));
  const bool lrac = o.precond == VL_PREC_LRAC;
  if (o.precond != VL_PREC_VADU && o.precond != VL_PREC_LRAC && grad)
    return Status::invalid("the gradient needs the VADU or the LRAC preconditioner");
  double logdet_lrac = 0.0;
  if (lrac) {
    // eq. (logdetsplit2): log det(Sigma~ W + I) = sum log W + log det P_LRAC
    // + log det(P^{-1} (Sigma~ + W^{-1})), probes z = L eps_k + W^{-1/2} eps_n
    VL_TRY(lrac_build(M, o.lrac_rank));
    std::vector<int> rbuf;
    VL_TRY(lrac_slq(M, o, &logdet_lrac, replay_slice(o, 0, t, rbuf), grad != nullptr));
  } else {
    VL_TRY(M.rhs_blk.reserve(static_cast<size_t>(n) * t));
    // probes z_i = P^{1/2} eps_i with Cov(z_i) = P:
    //   VADU B^T ((W + D^{-1})^{1/2} o eps_i), LVA B^T (D^{-1/2} o eps_i),
    //   P_1 P_1^{1/2} o eps_i;
    // the CG blocks Z and H serve as scratch before the solve starts
    VL_TRY(M.cg.Z.reserve(static_cast<size_t>(n) * t));
    VL_TRY(M.cg.H.reserve(static_cast<size_t>(n) * t));
    if (o.precond == VL_PREC_DIAG) {
      VL_TRY(M.vec_e.reserve(n));  // P_1
      VL_TRY(p1_diag(M, M.vec_b.p, M.vec_a.p, M.vec_e.p));
      VL_TRY(probe_fill(M, M.rhs_blk.p, t, M.vec_a.p, o.seed, kTagSlq, 0));
    } else {
      if (o.precond == VL_PREC_LVA) {
        hipLaunchKernelGGL(sqrt_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           M.stream, n, M.dinv.p, M.vec_a.p);
        VL_TRY(check_launch("LVA probe scale"));
      }
      VL_TRY(spmm_bt_probe(M, M.rhs_blk.p, t, M.vec_a.p, o.seed, kTagSlq, 0, 0, nullptr, 0, 0,
                           M.cg.Z.p, M.cg.H.p));
    }
    // mixed form: FP32 preconditioner solves inside the FP64 block PCG (P_1
    // has none and stays FP64)
    const bool mixed = o.precision == VL_MIXED && o.precond != VL_PREC_DIAG;
    CgOps ops = pcls1_ops(M, o.precond, mixed, M.vec_b.p);
    // mixed form (FP32 solves for t > 64): the FP32 preconditioner's
    // deviation from FP64 on the first probe, before the CG overwrites Z/H
    M.last_f32_dev = 0.0;
    if (mixed)
      VL_TRY(precond_f32_deviation(M, o.precond == VL_PREC_LVA ? M.dval.p : M.vec_b.p,
                                   M.rhs_blk.p, t, &M.last_f32_dev));
    std::vector<int> rbuf;
    VL_TRY(cg_solve(M, M.cg, ops, t, M.rhs_blk.p, o.cg_tol, o.max_cg, grad != nullptr,
                    replay_slice(o, 0, t, rbuf)));
  }
  M.last_block_iters = M.cg.host_iters;
  VL_TRY(M.red_out.reserve(2 * t + 64));
  VL_TRY(tridiag_quadrature(M, M.cg, M.red_out.p));
  M.last_quad.resize(t);
  M.last_r0z0.resize(t);
  VL_HIP(hipMemcpyAsync(M.last_quad.data(), M.red_out.p, sizeof(double) * t,
                        hipMemcpyDeviceToHost, M.stream));
  VL_HIP(hipMemcpyAsync(M.last_r0z0.data(), M.cg.r0z0.p, sizeof(double) * t,
                        hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  VL_TRY(read_status(M));
  double gamma = 0.0;
  for (int c = 0; c < t; ++c) gamma += M.last_r0z0[c] * M.last_quad[c];
  gamma /= t;
  double terms[4];
  VL_TRY(laplace_terms(M, M.mode.p, M.W.p, terms));
  // eq. (logdetsplit): log det Sigma~ (= sum log D) + log det P + SLQ term,
  // log det P = log det(W + D^{-1}) (VADU), -sum log D (LVA), sum log P_1
  double logdet_fixed = 0.0;
  if (lrac) {
    logdet_fixed = logdet_lrac;
  } else if (o.precond == VL_PREC_VADU) {
    logdet_fixed = terms[2] + terms[3];
  } else if (o.precond == VL_PREC_LVA) {
    logdet_fixed = terms[2] - terms[2];
  } else {
    ChunkGrid g1 = ChunkGrid::of(n, 1);
    VL_TRY(M.red_part.reserve(static_cast<size_t>(g1.nchunk) + 64));
    hipLaunchKernelGGL(log_sum_kernel, dim3(g1.nchunk, 1), dim3(256), 0, M.stream, g1, M.vec_e.p,
                       M.red_part.p);
    VL_TRY(check_launch("log P1"));
    double lp = 0.0;
    VL_TRY(host_sums(M, M.red_part.p, g1.nchunk, 1, &lp));
    logdet_fixed = terms[2] + lp;
  }
  const double logdet = logdet_fixed + gamma;
  *nll = -terms[0] + 0.5 * terms[1] + 0.5 * logdet;
  int cg_max = 0;
  for (int v : M.cg.host_iters) cg_max = v > cg_max ? v : cg_max;
  if (info) {
    info->gamma = gamma;
    info->logdet = logdet;
    info->loglik = terms[0];
    info->quadform = terms[1];
    info->cg_iters_max = cg_max;
  }
  if (grad) {
    GradInfo gi;
    if (lrac) {
      VL_TRY(grad_lrac(M, o, grad, &gi));
    } else {
      VL_TRY(grad_theta(M, o, M.vec_b.p, grad, &gi));
    }
    if (info) info->grad = gi;
  }
  if (cg_max >= o.max_cg)
    return Status::make(VL_ERR_NO_CONVERGENCE, "CG stopped at its iteration cap");
  return Status::ok();
}

// -------------------------------------------------------------- predict
// omega_p = F_p - B_po b*, with B_po entries -A_p stored like B
__global__ void pred_mean_kernel(int64_t np, int m, const int* __restrict__ nbr,
                                 const double* __restrict__ bval, const double* __restrict__ b,
                                 const double* __restrict__ Fp, double* __restrict__ mean) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  double acc = 0.0;
  for (int k = 0; k < m; ++k) {
    const int j = nbr[p * m + k];
    if (j < 0) break;
    acc += bval[p * m + k] * b[j];
  }
  mean[p] = (Fp ? Fp[p] : 0.0) - acc;
}

// z4 = B_po u for a block of tt columns; part[p * slices + slice] = sum_c z4^2
__global__ __launch_bounds__(256) void pred_acc_kernel(int64_t np, int m, int tt, Lanes L,
                                                       const int* __restrict__ nbr,
                                                       const double* __restrict__ bval,
                                                       const double* __restrict__ U,
                                                       double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (unit >= units_of_hd(np, tt, L)) return;
  const int64_t rg = unit / L.slices;
  const int slice = static_cast<int>(unit - rg * L.slices);
  const int sub = lane >> L.lpr_log;
  const int lpr = 1 << L.lpr_log;
  const int c = slice * 64 + (lane & (lpr - 1));
  const int64_t p = (rg << L.rpw_log) + sub;
  double z = 0.0;
  if (p < np && c < tt) {
    for (int k = 0; k < m; ++k) {
      const int j = nbr[p * m + k];
      if (j < 0) break;
      z += bval[p * m + k] * U[(int64_t)j * tt + c];
    }
  }
  double s = z * z;
  for (int o = 1; o < lpr; o <<= 1) s += __shfl_xor(s, o);
  if (p < np && (lane & (lpr - 1)) == 0) part[p * L.slices + slice] = s;
}

// acc_p += sum over slices
__global__ void pred_acc_add_kernel(int64_t np, int slices, const double* __restrict__ part,
                                    double* __restrict__ acc) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  double s = 0.0;
  for (int k = 0; k < slices; ++k) s += part[p * slices + k];
  acc[p] += s;
}

__global__ void pred_var_kernel(int64_t np, const double* __restrict__ Dp,
                                const double* __restrict__ acc, double inv_s,
                                double* __restrict__ var) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < np) var[p] = Dp[p] + acc[p] * inv_s;
}

// sqrt(W), D^{-1/2}
__global__ void pred_scales_kernel(int64_t n, const double* __restrict__ W,
                                   const double* __restrict__ dinv, double* __restrict__ sw,
                                   double* __restrict__ sd) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  sw[i] = sqrt(W[i]);
  sd[i] = sqrt(dinv[i]);
}

Status predict(Model& M, const double* coords_p, int64_t np, const double* Fp,
               const vl_opts& o, double* mean_out, double* var_out, PredInfo* info) {
  if (!M.has_mode) return Status::make(VL_ERR_STATE, "no mode: call vl_find_mode first");
  const int m = M.m;
  VL_TRY(M.pred_nbr.reserve(static_cast<size_t>(np) * (m > 0 ? m : 1)));
  VL_TRY(M.pred_bval.reserve(static_cast<size_t>(np) * (m > 0 ? m : 1)));
  VL_TRY(M.pred_dval.reserve(np));
  M.last_np = np;
  if (np == 0) return Status::ok();
  VL_TRY(knn_query(M, coords_p, np, M.pred_nbr.p));
  VL_TRY(factor_rows(M, coords_p, np, M.pred_nbr.p, M.pred_bval.p, M.pred_dval.p, false,
                     nullptr, nullptr, nullptr));
  const int tb = 256;
  const unsigned gp = static_cast<unsigned>((np + tb - 1) / tb);
  hipLaunchKernelGGL(pred_mean_kernel, dim3(gp), dim3(tb), 0, M.stream, np, m, M.pred_nbr.p,
                     M.pred_bval.p, M.mode.p, Fp, mean_out);
  VL_TRY(check_launch("pred mean"));
  if (!var_out) {
    VL_TRY(sync_stream(M.stream));
    return read_status(M);
  }
  if (o.pred_method != VL_PRED_SIMULATION) return predict_lanczos_var(M, np, o, var_out, info);
  const int s = o.num_pred_samples;
  if (s < 1) return Status::invalid("num_pred_samples must be positive");
  const int64_t n = M.n;
  VL_TRY(M.vec_a.reserve(n));  // sqrt(W)
  VL_TRY(M.vec_b.reserve(n));  // (W + D^{-1})^{-1}
  VL_TRY(M.vec_c.reserve(n));  // D^{-1/2}
  VL_TRY(lik_rows(M, M.mode.p, nullptr, M.W.p, nullptr, M.vec_b.p, nullptr, nullptr));
  hipLaunchKernelGGL(pred_scales_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0,
                     M.stream, n, M.W.p, M.dinv.p, M.vec_a.p, M.vec_c.p);
  DevBuf<double> acc, part;
  VL_TRY(acc.alloc(np));
  VL_TRY(fill_double(acc.p, 0.0, np, M.stream));
  const int tile = (o.pred_tile > 0 && o.pred_tile < s) ? o.pred_tile : s;
  // mixed form: FP32 preconditioner solves inside the FP64 block PCG
  CgOps ops = o.precision == VL_MIXED ? vadu_ops_mixed(M.W.p, M.vec_b.p)
                                      : vadu_ops(M.W.p, M.vec_b.p);
  int cg_max = 0;
  M.last_block_iters.clear();
  for (int c0 = 0; c0 < s; c0 += tile) {
    const int tt = (s - c0 < tile) ? (s - c0) : tile;
    VL_TRY(M.rhs_blk.reserve(static_cast<size_t>(n) * tt));
    // z3 = W^{1/2} z1 + B^T (D^{-1/2} o z2), z1, z2 standard normal; the CG
    // blocks Z and H serve as scratch before the solve starts
    VL_TRY(M.cg.Z.reserve(static_cast<size_t>(n) * tt));
    VL_TRY(M.cg.H.reserve(static_cast<size_t>(n) * tt));
    VL_TRY(spmm_bt_probe(M, M.rhs_blk.p, tt, M.vec_c.p, o.seed, kTagPredZ2, c0, 1, M.vec_a.p,
                         kTagPredZ1, 1, M.cg.Z.p, M.cg.H.p));
    if (c0 == 0) {
      M.last_f32_dev = 0.0;
      if (o.precision == VL_MIXED)
        VL_TRY(precond_f32_deviation(M, M.vec_b.p, M.rhs_blk.p, tt, &M.last_f32_dev));
    }
    std::vector<int> rbuf;
    VL_TRY(cg_solve(M, M.cg, ops, tt, M.rhs_blk.p, o.pred_cg_tol, o.max_cg, false,
                    replay_slice(o, c0, tt, rbuf)));
    for (int v : M.cg.host_iters) {
      cg_max = v > cg_max ? v : cg_max;
      M.last_block_iters.push_back(v);
    }
    Lanes L = Lanes::of(tt);
    VL_TRY(part.reserve(static_cast<size_t>(np) * L.slices));
    const int64_t units = units_of_hd(np, tt, L);
    hipLaunchKernelGGL(pred_acc_kernel, dim3((unsigned)((units + 3) / 4)), dim3(256), 0,
                       M.stream, np, m, tt, L, M.pred_nbr.p, M.pred_bval.p, M.cg.U.p, part.p);
    hipLaunchKernelGGL(pred_acc_add_kernel, dim3(gp), dim3(tb), 0, M.stream, np, L.slices,
                       part.p, acc.p);
    VL_TRY(check_launch("pred acc"));
  }
  hipLaunchKernelGGL(pred_var_kernel, dim3(gp), dim3(tb), 0, M.stream, np, M.pred_dval.p, acc.p,
                     1.0 / s, var_out);
  VL_TRY(check_launch("pred var"));
  VL_TRY(sync_stream(M.stream));
  VL_TRY(read_status(M));
  if (info) info->cg_iters_max = cg_max;
  if (cg_max >= o.max_cg)
    return Status::make(VL_ERR_NO_CONVERGENCE, "CG stopped at its iteration cap");
  return Status::ok();
}

}  // namespace vl
