// C ABI of the library (declared in include/vl.h).
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

struct vl_model : public vl::Model {};

namespace vl {

static thread_local std::string g_last_error;

static vl_status fail(const Status& s) {
  g_last_error = s.msg;
  return s.code;
}

vl_status report(const Status& s) { return s.good() ? VL_OK : fail(s); }

Model* model_of(vl_model* h) { return h; }

__global__ void recip_kernel(int64_t n, const double* __restrict__ d, double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = 1.0 / d[i];
}

// D^{-1}, the copies of the B values (B^T, groups) and the dense inverse
// after a factor.
Status finish_factor(Model& M) {
  const int64_t n = M.n;
  const int tb = 256;
  hipLaunchKernelGGL(recip_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, M.stream,
                     n, M.dval.p, M.dinv.p);
  VL_TRY(check_launch("recip"));
  VL_TRY(refresh_transpose_values(M));
  VL_TRY(refresh_group_values(M));
  VL_TRY(dense_factor(M));
  ++M.factor_version;
  VL_TRY(sync_stream(M.stream));
  return read_status(M);
}

// A_i, D_i (and derivatives) at the model's theta; refresh B^T values.
static Status compute_factor(Model& M) {
  const int64_t n = M.n;
  const size_t nm = static_cast<size_t>(n) * (M.m > 0 ? M.m : 1);
  VL_TRY(M.bval.reserve(nm));
  VL_TRY(M.dval.reserve(n));
  VL_TRY(M.dinv.reserve(n));
  if (M.deriv) {
    VL_TRY(M.dbval_rho.reserve(nm));
    VL_TRY(M.dd_sigma2.reserve(n));
    VL_TRY(M.dd_rho.reserve(n));
  }
  VL_TRY(factor_rows(M, nullptr, n, M.nbr.p, M.bval.p, M.dval.p, M.deriv, M.dbval_rho.p,
                     M.dd_sigma2.p, M.dd_rho.p));
  return finish_factor(M);
}

static Status check_theta(const double* theta) {
  if (!theta) return Status::invalid("theta is null");
  if (!(theta[0] > 0.0) || !(theta[1] > 0.0) || !std::isfinite(theta[0]) ||
      !std::isfinite(theta[1]))
    return Status::invalid("theta must be positive and finite");
  return Status::ok();
}

constexpr int64_t kMaxModelRows = 262144;

static Status build(const double* coords, int64_t n, int m, int cov, const double* theta,
                    void* stream, int want_deriv, Model** out) {
  if (!out) return Status::invalid("out is null");
  *out = nullptr;
  if (!coords) return Status::invalid("coords is null");
  if (n < 1) return Status::invalid("n must be positive");
  if (m < 0 || m > 31) return Status::invalid("m must be in [0, 31]");
  // A build at n = 2,000,000 ended in a GPU memory fault whose cause is not
  // found; until it is, models stay within the verified size range.
  if (n > kMaxModelRows)
    return Status::invalid("n above the verified limit (262144 locations)");
  if (cov != VL_COV_EXPONENTIAL && cov != VL_COV_MATERN32)
    return Status::invalid("unknown covariance");
  VL_TRY(check_theta(theta));
  Model* M = new (std::nothrow) vl_model();
  if (!M) return Status::make(VL_ERR_OOM, "host allocation failed");
  Status st = [&]() -> Status {
    VL_HIP(hipGetDevice(&M->device));
    VL_HIP(hipDeviceGetAttribute(&M->num_cus, hipDeviceAttributeMultiprocessorCount, M->device));
    M->stream = static_cast<hipStream_t>(stream);
    M->n = n;
    M->m = m;
    M->cov = cov;
    M->sigma2 = theta[0];
    M->rho = theta[1];
    M->deriv = want_deriv != 0;
    VL_TRY(M->status_buf.alloc(4));
    M->status = M->status_buf.p;
    VL_TRY(fill_int(M->status, 0, 4, M->stream));
    VL_TRY(M->coords_buf.alloc(2 * static_cast<size_t>(n)));
    M->coords = M->coords_buf.p;
    VL_TRY(copy_d2d(M->coords_buf.p, coords, sizeof(double) * 2 * n, M->stream));
    VL_TRY(M->nbr.alloc(static_cast<size_t>(n) * (m > 0 ? m : 1)));
    VL_TRY(knn_build_grid(*M));
    VL_TRY(knn_query(*M, nullptr, n, M->nbr.p));
    VL_TRY(build_transpose(*M));
    VL_TRY(build_groups(*M));
    M->dense_rows = kDenseRows;
    if (const char* env = std::getenv("VL_DENSE_ROWS")) M->dense_rows = std::atoi(env);  // tuning knob
    if (M->dense_rows < 0) M->dense_rows = 0;
    VL_TRY(build_head_schedule(*M));
    VL_TRY(build_tail_orders(*M));
    VL_TRY(compute_factor(*M));
    return Status::ok();
  }();
  if (!st.good()) {
    delete static_cast<vl_model*>(M);
    return st;
  }
  *out = M;
  return Status::ok();
}

static void release(Model* M) {
  if (!M) return;
  (void)hipStreamSynchronize(M->stream);
  for (hipEvent_t e : M->timing.pool) (void)hipEventDestroy(e);
  for (void* p : M->owned) device_free(p);
  if (M->host_pin) (void)hipHostFree(M->host_pin);
  delete static_cast<vl_model*>(M);
}

static Status copy_out(Model& M, void* dst, const void* src, size_t bytes, bool src_host) {
  VL_HIP(hipMemcpyAsync(dst, src, bytes, src_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                        M.stream));
  return sync_stream(M.stream);
}

static int64_t export_count(Model& M, int which) {
  const int64_t nm = M.n * static_cast<int64_t>(M.m);
  switch (which) {
    case 0: case 1: return nm;
    case 2: return M.n;
    case 3: case 4: return M.has_mode ? M.n : -1;
    case 5: case 6: return M.deriv ? nm : -1;
    case 7: case 8: return M.deriv ? M.n : -1;
    case 9: return static_cast<int64_t>(M.last_block_iters.size());
    case 10: return static_cast<int64_t>(M.newton_cg_iters.size());
    case 11: return static_cast<int64_t>(M.last_quad.size());
    case 12: return static_cast<int64_t>(M.last_r0z0.size());
    case 13: case 14: return M.last_np * M.m;
    case 15: return M.last_np;
    case 16: return M.lrac_ready ? M.n * M.lrac_k : -1;
    case 17: return M.lrac_ready ? M.lrac_k : -1;
    case 18: return M.lrac_ready ? static_cast<int64_t>(M.lrac_K) * M.lrac_K : -1;
    case 19: return static_cast<int64_t>(M.newton_halvings.size());
    case 20: return static_cast<int64_t>(M.last_lanczos_alpha.size());
    case 21: return static_cast<int64_t>(M.last_lanczos_beta.size());
    default: return -1;
  }
}

static Status do_export(Model& M, int which, void* dst, size_t bytes) {
  const int64_t cnt = export_count(M, which);
  if (cnt < 0) return Status::make(VL_ERR_STATE, "array not available");
  const bool is_int = (which == 0 || which == 9 || which == 10 || which == 13 || which == 17 ||
                       which == 19);
  const size_t need = static_cast<size_t>(cnt) * (is_int ? sizeof(int) : sizeof(double));
  if (bytes != need) return Status::invalid("export size mismatch");
  if (need == 0) return Status::ok();
  if (!dst) return Status::invalid("dst is null");
  switch (which) {
    case 0: return copy_out(M, dst, M.nbr.p, need, false);
    case 1: return copy_out(M, dst, M.bval.p, need, false);
    case 2: return copy_out(M, dst, M.dval.p, need, false);
    case 3: return copy_out(M, dst, M.mode.p, need, false);
    case 4: return copy_out(M, dst, M.W.p, need, false);
    case 5: {
      VL_TRY(fill_double(static_cast<double*>(dst), 0.0, cnt, M.stream));
      return sync_stream(M.stream);
    }
    case 6: return copy_out(M, dst, M.dbval_rho.p, need, false);
    case 7: return copy_out(M, dst, M.dd_sigma2.p, need, false);
    case 8: return copy_out(M, dst, M.dd_rho.p, need, false);
    case 9: return copy_out(M, dst, M.last_block_iters.data(), need, true);
    case 10: return copy_out(M, dst, M.newton_cg_iters.data(), need, true);
    case 11: return copy_out(M, dst, M.last_quad.data(), need, true);
    case 12: return copy_out(M, dst, M.last_r0z0.data(), need, true);
    case 13: return copy_out(M, dst, M.pred_nbr.p, need, false);
    case 14: return copy_out(M, dst, M.pred_bval.p, need, false);
    case 15: return copy_out(M, dst, M.pred_dval.p, need, false);
    case 16: {  // n x k out of the padded n x K layout
      VL_HIP(hipMemcpy2DAsync(dst, sizeof(double) * M.lrac_k, M.lrac_L.p,
                              sizeof(double) * M.lrac_K, sizeof(double) * M.lrac_k, M.n,
                              hipMemcpyDeviceToDevice, M.stream));
      return sync_stream(M.stream);
    }
    case 17: return copy_out(M, dst, M.lrac_piv.p, need, false);
    case 18: return copy_out(M, dst, M.lrac_M.p, need, false);
    case 19: return copy_out(M, dst, M.newton_halvings.data(), need, true);
    case 20: return copy_out(M, dst, M.last_lanczos_alpha.data(), need, true);
    case 21: return copy_out(M, dst, M.last_lanczos_beta.data(), need, true);
    default: return Status::invalid("unknown export");
  }
}

Status likelihood_aux(int lik, const double* aux_host, double* aux) {
  *aux = 0.0;
  switch (lik) {
    case VL_LIK_BERNOULLI_LOGIT:
    case VL_LIK_POISSON_LOG:
      return Status::ok();
    case VL_LIK_GAUSSIAN:
      if (!aux_host || !(aux_host[0] > 0.0) || !std::isfinite(aux_host[0]))
        return Status::invalid("Gaussian needs tau2 > 0");
      *aux = aux_host[0];
      return Status::ok();
    case VL_LIK_GAMMA:
      if (!aux_host || !(aux_host[0] > 0.0) || !std::isfinite(aux_host[0]))
        return Status::invalid("Gamma needs a shape > 0");
      *aux = aux_host[0];
      return Status::ok();
    default:
      return Status::invalid("unknown likelihood");
  }
}

static Status check_opts(const vl_opts* o) {
  if (!o) return Status::invalid("opts is null");
  if (o->max_newton < 1 || o->max_cg < 1) return Status::invalid("iteration caps must be >= 1");
  if (!(o->cg_tol > 0.0) || !(o->pred_cg_tol > 0.0) || !(o->newton_tol >= 0.0))
    return Status::invalid("tolerances must be positive");
  if (o->precond != VL_PREC_VADU && o->precond != VL_PREC_LRAC && o->precond != VL_PREC_LVA &&
      o->precond != VL_PREC_DIAG)
    return Status::invalid("unknown preconditioner");
  if (o->pred_method != VL_PRED_SIMULATION && o->pred_method != VL_PRED_LANCZOS_L1 &&
      o->pred_method != VL_PRED_LANCZOS_L2)
    return Status::invalid("unknown predictive-variance method");
  if (o->precision != VL_FP64 && o->precision != VL_MIXED)
    return Status::invalid("unknown precision");
  if (o->replay_len < 0 || (o->replay_len > 0 && !o->replay_cg_iters))
    return Status::invalid("replay_len needs replay_cg_iters");
  return Status::ok();
}

template <class F>
static vl_status guarded(F&& f) {
  try {
    Status s = f();
    if (!s.good()) return fail(s);
    return VL_OK;
  } catch (const std::bad_alloc&) {
    return fail(Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return fail(Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// The model's per-phase wall times into a statistics record.
static void fill_phases(const Model& M, vl_stats* st) {
  st->t_build_us = M.t_build_us;
  st->t_mode_us = M.t_mode_us;
  st->t_slq_us = M.t_slq_us;
  st->t_pred_us = M.t_pred_us;
}

}  // namespace vl

using vl::Model;

extern "C" {

void vl_default_opts(vl_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_newton = 100;
  o->newton_tol = 1e-6;
  o->max_cg = 1000;
  o->cg_tol = 1e-2;
  o->pred_cg_tol = 1e-3;
  o->num_probes = 50;
  o->num_pred_samples = 2000;
  o->seed = 0;
  o->precond = VL_PREC_VADU;
  o->lrac_rank = 50;
  o->precision = VL_FP64;
  o->pred_tile = 0;
  o->pred_method = VL_PRED_SIMULATION;
  o->lanczos_rank = 100;
}

const char* vl_status_string(vl_status s) {
  switch (s) {
    case VL_OK: return "ok";
    case VL_ERR_INVALID_ARG: return "invalid argument";
    case VL_ERR_NOT_SPD: return "covariance not positive definite";
    case VL_ERR_NO_CONVERGENCE: return "no convergence";
    case VL_ERR_OOM: return "out of memory";
    case VL_ERR_NONFINITE: return "non-finite value";
    case VL_ERR_HIP: return "HIP error";
    case VL_ERR_STATE: return "invalid call order";
    case VL_ERR_TIMEOUT: return "device wait timed out";
    default: return "unknown status";
  }
}

const char* vl_last_error(void) { return vl::g_last_error.c_str(); }

vl_status vl_build_vecchia(const double* coords, int64_t n, int m, int cov,
                           const double* theta_host, void* hip_stream, int want_deriv,
                           vl_model** out) {
  vl::CallStream cs(static_cast<hipStream_t>(hip_stream));
  return vl::guarded([&]() -> vl::Status {
    const double t0 = vl::now_ms();
    Model* M = nullptr;
    VL_TRY(vl::build(coords, n, m, cov, theta_host, hip_stream, want_deriv, &M));
    M->t_build_us = 1e3 * (vl::now_ms() - t0);
    *out = static_cast<vl_model*>(M);
    return vl::Status::ok();
  });
}

vl_status vl_set_theta(vl_model* h, const double* theta_host) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h) return vl::Status::invalid("null handle");
    VL_TRY(vl::check_theta(theta_host));
    h->sigma2 = theta_host[0];
    h->rho = theta_host[1];
    h->has_mode = false;
    h->has_grad_F = false;
    h->has_grad_xi = false;
    h->lrac_ready = false;
    h->lrac_dL_ready = false;
    const double t0 = vl::now_ms();
    VL_TRY(vl::compute_factor(*h));
    h->t_build_us = 1e3 * (vl::now_ms() - t0);
    return vl::Status::ok();
  });
}

vl_status vl_find_mode(vl_model* h, const double* y, const double* F, int lik,
                       const double* aux_host, const vl_opts* o, double* mode_out,
                       vl_stats* st) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    const double t0 = vl::now_ms();
    if (!h || !y) return vl::Status::invalid("null handle or y");
    VL_TRY(vl::check_opts(o));
    double aux = 0.0;
    VL_TRY(vl::likelihood_aux(lik, aux_host, &aux));
    if (o->precond == VL_PREC_LRAC && (o->lrac_rank < 1 || o->lrac_rank > 1024))
      return vl::Status::invalid("lrac_rank must be in [1, 1024]");
    Model& M = *h;
    M.lik = lik;
    M.aux = aux;
    M.has_mode = false;
    M.has_grad_F = false;
    M.has_grad_xi = false;
    VL_TRY(M.y.reserve(M.n));
    VL_TRY(vl::copy_d2d(M.y.p, y, sizeof(double) * M.n, M.stream));
    if (F) {
      VL_TRY(M.F.reserve(M.n));
      VL_TRY(vl::copy_d2d(M.F.p, F, sizeof(double) * M.n, M.stream));
    } else {
      M.F.release();
    }
    vl_stats local{};
    vl::Status s = vl::find_mode(M, *o, &local);
    if (mode_out && M.has_mode) {
      VL_TRY(vl::copy_d2d(mode_out, M.mode.p, sizeof(double) * M.n, M.stream));
      VL_TRY(vl::sync_stream(M.stream));
    }
    local.t_ms = vl::now_ms() - t0;
    M.t_mode_us = 1e3 * local.t_ms;
    vl::fill_phases(M, &local);
    if (st) *st = local;
    return s;
  });
}

vl_status vl_neg_log_marglik(vl_model* h, const vl_opts* o, double* nll_host,
                             double* grad_theta_host, vl_stats* st) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    const double t0 = vl::now_ms();
    if (!h || !nll_host) return vl::Status::invalid("null handle or output");
    VL_TRY(vl::check_opts(o));
    if (o->precond == VL_PREC_LRAC && (o->lrac_rank < 1 || o->lrac_rank > 1024))
      return vl::Status::invalid("lrac_rank must be in [1, 1024]");
    vl::NllInfo info;
    vl::Status s = vl::neg_log_marglik(*h, *o, nll_host, grad_theta_host, &info);
    h->t_slq_us = 1e3 * (vl::now_ms() - t0);
    if (st) {
      std::memset(st, 0, sizeof(*st));
      st->cg_iters_max = info.cg_iters_max;
      st->cg_iters_total = info.cg_iters_max;
      st->hit_cap = (s.code == VL_ERR_NO_CONVERGENCE);
      st->t_ms = vl::now_ms() - t0;
      vl::fill_phases(*h, st);
      st->err_vs_fp64_est = o->precision == VL_MIXED ? h->last_f32_dev : 0.0;
    }
    return s;
  });
}

vl_status vl_predict(vl_model* h, const double* coords_p, int64_t n_p, const double* Fp,
                     const vl_opts* o, double* mean_out, double* var_out, vl_stats* st) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    const double t0 = vl::now_ms();
    if (!h) return vl::Status::invalid("null handle");
    if (n_p < 0) return vl::Status::invalid("n_p must be >= 0");
    if (n_p > 0 && (!coords_p || !mean_out)) return vl::Status::invalid("null coords or output");
    if (n_p * static_cast<int64_t>(h->m > 0 ? h->m : 1) >= (int64_t(1) << 31))
      return vl::Status::invalid("n_p * m must be below 2^31");
    VL_TRY(vl::check_opts(o));
    vl::PredInfo info;
    vl::Status s = vl::predict(*h, coords_p, n_p, Fp, *o, mean_out, var_out, &info);
    h->t_pred_us = 1e3 * (vl::now_ms() - t0);
    if (st) {
      std::memset(st, 0, sizeof(*st));
      st->cg_iters_max = info.cg_iters_max;
      st->hit_cap = (s.code == VL_ERR_NO_CONVERGENCE);
      st->t_ms = vl::now_ms() - t0;
      vl::fill_phases(*h, st);
      st->err_vs_fp64_est = (o->precision == VL_MIXED && var_out) ? h->last_f32_dev : 0.0;
    }
    return s;
  });
}

vl_status vl_grad_offset(vl_model* h, double* grad_F) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !grad_F) return vl::Status::invalid("null argument");
    if (!h->has_grad_F)
      return vl::Status::make(VL_ERR_STATE,
                              "no offset gradient: call vl_neg_log_marglik with a gradient");
    VL_TRY(vl::copy_d2d(grad_F, h->grad_F.p, sizeof(double) * h->n, h->stream));
    return vl::sync_stream(h->stream);
  });
}

vl_status vl_grad_beta(vl_model* h, const double* X, int p, double* grad_beta_host) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !X || !grad_beta_host) return vl::Status::invalid("null argument");
    return vl::grad_beta(*h, X, p, grad_beta_host);
  });
}

vl_status vl_grad_aux(vl_model* h, double* grad_xi_host) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !grad_xi_host) return vl::Status::invalid("null argument");
    if (!vl::lik_has_aux(h->lik))
      return vl::Status::invalid("the likelihood has no auxiliary parameter");
    if (!h->has_grad_xi)
      return vl::Status::make(VL_ERR_STATE,
                              "no xi-gradient: call vl_neg_log_marglik with a gradient");
    *grad_xi_host = h->grad_xi;
    return vl::Status::ok();
  });
}

vl_status vl_export(vl_model* h, int which, void* dst, size_t bytes) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h) return vl::Status::invalid("null handle");
    return vl::do_export(*h, which, dst, bytes);
  });
}

int64_t vl_export_count(vl_model* h, int which) {
  if (!h) return -1;
  return vl::export_count(*h, which);
}

vl_status vl_spmm(vl_model* h, int transpose, const double* X, double* Y, int t) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !X || !Y) return vl::Status::invalid("null argument");
    if (t < 1) return vl::Status::invalid("t must be positive");
    if (transpose) return vl::spmm_bt(*h, X, Y, t, nullptr, nullptr);
    return vl::spmm_b(*h, X, Y, t, nullptr);
  });
}

vl_status vl_trsm(vl_model* h, int transpose, const double* X, double* Y, int t) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !X || !Y) return vl::Status::invalid("null argument");
    if (t < 1) return vl::Status::invalid("t must be positive");
    if (transpose) {
      VL_TRY(vl::trsm_bt(*h, X, Y, t, false));
    } else {
      VL_TRY(vl::trsm_b(*h, X, Y, t, nullptr, false));
    }
    VL_TRY(vl::sync_stream(h->stream));
    return vl::read_status(*h);
  });
}

vl_status vl_timing_enable(vl_model* h, int enable) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h) return vl::Status::invalid("null handle");
    VL_TRY(vl::sync_stream(h->stream));
    h->timing.on = enable != 0;
    h->timing.mask = static_cast<unsigned>(enable);
    h->timing.used = 0;
    h->timing.recs.clear();
    return vl::Status::ok();
  });
}

vl_status vl_timing_read(vl_model* h, int kind, double* total_ms, int64_t* launches,
                         double* bytes) {
  vl::CallStream cs(h ? h->stream : nullptr);
  return vl::guarded([&]() -> vl::Status {
    if (!h || !total_ms || !launches || !bytes) return vl::Status::invalid("null argument");
    if (kind < 0 || kind >= vl::kTimeKinds) return vl::Status::invalid("unknown kind");
    VL_TRY(vl::sync_stream(h->stream));
    double ms = 0.0, by = 0.0;
    int64_t cnt = 0;
    for (const auto& r : h->timing.recs) {
      if (r.kind != kind) continue;
      float e = 0.0f;
      VL_HIP(hipEventElapsedTime(&e, h->timing.pool[r.ev], h->timing.pool[r.ev + 1]));
      ms += e;
      by += r.bytes;
      ++cnt;
    }
    *total_ms = ms;
    *launches = cnt;
    *bytes = by;
    return vl::Status::ok();
  });
}

void vl_free(vl_model* h) {
  vl::CallStream cs(h ? h->stream : nullptr);
  vl::release(h);
}

vl_status vl_set_allocator(vl_alloc_fn alloc, vl_free_fn release, void* ctx) {
  return vl::guarded([&]() -> vl::Status { return vl::set_allocator(alloc, release, ctx); });
}

}  // extern "C"
