// Predictive variances by preconditioned Lanczos (Sec. 3.3.2).
//
// k steps of the symmetric Lanczos process on
//   P_L1: M = P^{-1/2} A P^{-T/2},  P = B^T (W + D^{-1}) B, P^{-1/2} =
//         (W + D^{-1})^{-1/2} B^{-T} (eq. P_VADU_prec), A = W + Sigma~^{-1};
//   P_L2: M = P^{-1/2} (Sigma~ + W^{-1}) P^{-1/2},  P = diag(sigma^2 + 1/W)
//         (the diagonal of the original Sigma standing in for diag Sigma~,
//         whose exact value needs O(n^2) work),
// started from the mean column xbar of B_po^T mapped into M's coordinates
// (P^{-1/2} xbar, resp. P^{-1/2} Sigma~ xbar), with complete
// reorthogonalization (classical Gram-Schmidt against all earlier vectors,
// twice; Golub & Van Loan, Matrix Computations, Sec. 10.3.1).  With the
// tridiagonal T = L L^T (bidiagonal Cholesky, host) the variances are
//   P_L1: D_p + |L^{-1} g_j|^2,          g_j = row j of A_p P^{-T/2} Q,
//   P_L2: D_p + (L^{-1} g1_j)^T (L^{-1} g2_j),
//         g1_j = row j of A_p W^{-1} P^{-1/2} Q, g2_j = row j of A_p Sigma~ P^{-1/2} Q
// (B_po = -A_p; its sign cancels in each product).
//
// Layout: the Lanczos vectors as an n x k row-major block Q (row i holds
// q_0[i] .. q_{k-1}[i]), so the projections Q^T w read whole rows and the
// update w -= Q c is one contiguous row read per thread; the current vector
// also lives in a contiguous n-vector for the operator's sparse solves.
#include <algorithm>
#include <cmath>
#include <vector>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

namespace vl {

namespace {

// part[chunk * kc + c] = sum over the chunk's rows of Q[i * ld + c] w[i]
__global__ __launch_bounds__(256) void proj_kernel(ChunkGrid g, int ld,
                                                   const double* __restrict__ Q,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  acc += Q[i * ld + c] * w[i];
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

// w[i] -= sum_{c < kc} Q[i * ld + c] coef[c]
__global__ void orth_update_kernel(int64_t n, int ld, int kc, const double* __restrict__ Q,
                                   const double* __restrict__ coef, double* __restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* q = Q + i * ld;
  double acc = 0.0;
  for (int c = 0; c < kc; ++c) acc += q[c] * coef[c];
  w[i] -= acc;
}

// q = w / beta into column j of Q and into the contiguous vector qv
__global__ void lanczos_next_kernel(int64_t n, int ld, int j, double inv_beta,
                                    const double* __restrict__ w, double* __restrict__ Q,
                                    double* __restrict__ qv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = w[i] * inv_beta;
  Q[i * ld + j] = v;
  qv[i] = v;
}

// out = a o x (+ b o y when y is given)
__global__ void scale_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ x,
                             const double* __restrict__ b, const double* __restrict__ y,
                             double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = a[i] * x[i];
  if (y) v += b[i] * y[i];
  out[i] = v;
}

// Y[i, c] = a_i X[i * ldx + c] for c < k (n x k row-major output)
__global__ void scale_rows_kernel(int64_t n, int k, int ldx, const double* __restrict__ a,
                                  const double* __restrict__ X, double* __restrict__ Y) {
  const int64_t nk = n * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    Y[e] = a[i] * X[i * ldx + (e - i * k)];
  }
}

// P_L1 scale (W + D^{-1})^{-1/2}; P_L2 scale (sigma^2 + 1/W)^{-1/2} and
// (sigma^2 + 1/W)^{-1/2} / W
__global__ void lanczos_scales_kernel(int64_t n, int form, double sigma2,
                                      const double* __restrict__ W,
                                      const double* __restrict__ dinv, double* __restrict__ s,
                                      double* __restrict__ sw, double* __restrict__ winv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = W[i];
  if (form == 1) {
    s[i] = 1.0 / sqrt(w + dinv[i]);
  } else {
    const double si = 1.0 / sqrt(sigma2 + 1.0 / w);
    s[i] = si;
    sw[i] = si / w;
    winv[i] = 1.0 / w;
  }
}

// xbar_i = scale * sum of the A_p entries (test point r, slot k) with
// nbr_p[r, k] = i, in increasing r (the transpose's sorted rows)
__global__ void col_mean_kernel(int64_t n, const int* __restrict__ ptr,
                                const int* __restrict__ src, const double* __restrict__ vals,
                                double scale, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int p = ptr[i]; p < ptr[i + 1]; ++p) acc += vals[src[p]];
  out[i] = scale * acc;
}

// G[j, c] = sum_k A_p[j, k] Y[nbr_p[j, k], c]  (n_p x k, Y n x k row-major)
__global__ void pred_gather_kernel(int64_t np, int m, int k, const int* __restrict__ nbr,
                                   const double* __restrict__ ap, const double* __restrict__ Y,
                                   double* __restrict__ G) {
  const int64_t npk = np * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npk;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / k;
    const int c = static_cast<int>(e - j * k);
    double acc = 0.0;
    for (int q = 0; q < m; ++q) {
      const int nb = nbr[j * m + q];
      if (nb < 0) break;
      acc += ap[j * m + q] * Y[(int64_t)nb * k + c];
    }
    G[e] = acc;
  }
}

// var_j = D_p,j + (L^{-1} g1_j)^T (L^{-1} g2_j), L lower bidiagonal with
// diagonal ld and subdiagonal le (le[0] unused); g2 = null means g2 = g1.
__global__ void lanczos_var_kernel(int64_t np, int k, const double* __restrict__ ld,
                                   const double* __restrict__ le, const double* __restrict__ G1,
                                   const double* __restrict__ G2, const double* __restrict__ Dp,
                                   double* __restrict__ var) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= np) return;
  const double* g1 = G1 + j * k;
  const double* g2 = G2 ? G2 + j * k : nullptr;
  double z1 = 0.0, z2 = 0.0, acc = 0.0;
  for (int a = 0; a < k; ++a) {
    const double e = a > 0 ? le[a] : 0.0;
    z1 = (g1[a] - e * z1) / ld[a];
    if (g2) {
      z2 = (g2[a] - e * z2) / ld[a];
      acc += z1 * z2;
    } else {
      acc += z1 * z1;
    }
  }
  var[j] = Dp[j] + acc;
}

unsigned blocks_of(int64_t count) {
  return static_cast<unsigned>(std::min<int64_t>((count + 255) / 256, 8192));
}

}  // namespace

Status predict_lanczos_var(Model& M, int64_t np, const vl_opts& o, double* var_out,
                           PredInfo* info) {
  const int form = o.pred_method;
  const int64_t n = M.n;
  const int m = M.m;
  const int k = o.lanczos_rank;
  if (k < 1 || k > 4096 || k > n) return Status::invalid("lanczos_rank must be in [1, min(n, 4096)]");
  hipStream_t st = M.stream;
  const unsigned gn = static_cast<unsigned>((n + 255) / 256);
  // W at the mode and the form's diagonal scales
  VL_TRY(M.W.reserve(n));
  VL_TRY(lik_rows(M, M.mode.p, nullptr, M.W.p, nullptr, nullptr, nullptr, nullptr));
  DevBuf<double> s, sw, winv, xbar, qv, w, tmp, tmp2, Q, coef, part, red;
  VL_TRY(s.alloc(n));
  VL_TRY(sw.alloc(form == 2 ? n : 1));
  VL_TRY(winv.alloc(form == 2 ? n : 1));
  hipLaunchKernelGGL(lanczos_scales_kernel, dim3(gn), dim3(256), 0, st, n, form, M.sigma2,
                     M.W.p, M.dinv.p, s.p, sw.p, winv.p);
  VL_TRY(check_launch("lanczos scales"));
  // xbar = mean column of B_po^T = -(1/n_p) A_p^T 1, summed per training row
  // in increasing test-point order
  VL_TRY(xbar.alloc(n));
  {
    DevBuf<int> tptr, tcol, tsrc;
    int nnz = 0;
    VL_TRY(transpose_pattern(M, M.pred_nbr.p, np, m, n, tptr, tcol, tsrc, &nnz));
    hipLaunchKernelGGL(col_mean_kernel, dim3(gn), dim3(256), 0, st, n, tptr.p, tsrc.p,
                       M.pred_bval.p, -1.0 / static_cast<double>(np), xbar.p);
    VL_TRY(check_launch("lanczos start"));
    VL_TRY(sync_stream(st));
  }
  VL_TRY(qv.alloc(n));
  VL_TRY(w.alloc(n));
  VL_TRY(tmp.alloc(n));
  VL_TRY(tmp2.alloc(n));
  // start vector (unnormalised) into w: P_L1 s o B^{-T} xbar; P_L2 s o Sigma~ xbar
  if (form == 1) {
    VL_TRY(trsm_bt(M, xbar.p, tmp.p, 1, false));
  } else {
    VL_TRY(trsm_bt(M, xbar.p, tmp2.p, 1, false));
    VL_TRY(trsm_b(M, tmp2.p, tmp.p, 1, M.dval.p, false));
  }
  hipLaunchKernelGGL(scale_kernel, dim3(gn), dim3(256), 0, st, n, s.p, tmp.p, nullptr, nullptr,
                     w.p);
  VL_TRY(check_launch("lanczos start"));
  VL_TRY(Q.alloc(static_cast<size_t>(n) * k));
  VL_TRY(coef.alloc(k + 64));
  VL_TRY(red.alloc(64));
  size_t part_need = 64;
  for (int kc = 1; kc <= k; ++kc)
    part_need = std::max(part_need, static_cast<size_t>(ChunkGrid::of(n, kc).nchunk) * kc);
  VL_TRY(part.alloc(part_need));
  auto norm = [&](const double* v, double* out) -> Status {
    VL_TRY(dot_cols(M, v, v, 1, part.p, red.p));
    VL_HIP(hipMemcpyAsync(out, red.p, sizeof(double), hipMemcpyDeviceToHost, st));
    VL_TRY(sync_stream(st));
    *out = std::sqrt(*out);
    return Status::ok();
  };
  double b0 = 0.0;
  VL_TRY(norm(w.p, &b0));
  if (!(b0 > 0.0) || !std::isfinite(b0))
    return Status::make(VL_ERR_NONFINITE, "the Lanczos start vector is zero or not finite");
  hipLaunchKernelGGL(lanczos_next_kernel, dim3(gn), dim3(256), 0, st, n, k, 0, 1.0 / b0, w.p, Q.p,
                     qv.p);
  std::vector<double> alpha, beta;
  int kk = k;
  double amax = 0.0;
  for (int j = 0; j < k; ++j) {
    // w = M q_j
    if (form == 1) {
      // s o B^{-T} A B^{-1} (s o q)
      VL_TRY(trsm_b(M, qv.p, tmp.p, 1, s.p, false));
      VL_TRY(spmm_b(M, tmp.p, tmp2.p, 1, M.dinv.p));
      VL_TRY(spmm_bt(M, tmp2.p, w.p, 1, M.W.p, tmp.p));
      VL_TRY(trsm_bt(M, w.p, tmp.p, 1, false));
      hipLaunchKernelGGL(scale_kernel, dim3(gn), dim3(256), 0, st, n, s.p, tmp.p, nullptr,
                         nullptr, w.p);
    } else {
      // s o (Sigma~ (s o q) + W^{-1} o (s o q))
      hipLaunchKernelGGL(scale_kernel, dim3(gn), dim3(256), 0, st, n, s.p, qv.p, nullptr, nullptr,
                         tmp2.p);
      VL_TRY(trsm_bt(M, tmp2.p, tmp.p, 1, false));
      VL_TRY(trsm_b(M, tmp.p, w.p, 1, M.dval.p, false));
      // tmp = Sigma~ y + W^{-1} o y, then w = s o tmp
      hipLaunchKernelGGL(scale_kernel, dim3(gn), dim3(256), 0, st, n, winv.p, tmp2.p,
                         nullptr, nullptr, tmp.p);
      VL_TRY(check_launch("lanczos op"));
      hipLaunchKernelGGL(scale_kernel, dim3(gn), dim3(256), 0, st, n, s.p, w.p, s.p, tmp.p,
                         tmp2.p);
      VL_HIP(hipMemcpyAsync(w.p, tmp2.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    VL_TRY(check_launch("lanczos op"));
    // complete reorthogonalization against q_0 .. q_j, twice; alpha_j =
    // q_j^T M q_j from the first pass
    const int kc = j + 1;
    ChunkGrid g = ChunkGrid::of(n, kc);
    double a_j = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(proj_kernel, dim3(g.nchunk, g.L.slices), dim3(256), 0, st, g, k, Q.p,
                         w.p, part.p);
      VL_TRY(check_launch("lanczos projection"));
      VL_TRY(reduce_chunks(st, part.p, g.nchunk, kc, coef.p));
      if (pass == 0) {
        VL_HIP(hipMemcpyAsync(&a_j, coef.p + j, sizeof(double), hipMemcpyDeviceToHost, st));
      }
      hipLaunchKernelGGL(orth_update_kernel, dim3(gn), dim3(256), 0, st, n, k, kc, Q.p, coef.p,
                         w.p);
      VL_TRY(check_launch("lanczos update"));
    }
    VL_TRY(sync_stream(st));
    alpha.push_back(a_j);
    amax = std::max(amax, std::fabs(a_j));
    if (j + 1 == k) break;
    double bj = 0.0;
    VL_TRY(norm(w.p, &bj));
    if (!std::isfinite(bj)) return Status::make(VL_ERR_NONFINITE, "Lanczos vector not finite");
    if (bj <= 1e-13 * amax) {  // an invariant subspace: stop with rank j + 1
      kk = j + 1;
      break;
    }
    beta.push_back(bj);
    hipLaunchKernelGGL(lanczos_next_kernel, dim3(gn), dim3(256), 0, st, n, k, j + 1, 1.0 / bj,
                       w.p, Q.p, qv.p);
    VL_TRY(check_launch("lanczos next"));
  }
  // T = L L^T, L lower bidiagonal
  std::vector<double> ldg(kk), le(kk, 0.0);
  for (int a = 0; a < kk; ++a) {
    double d = alpha[a];
    if (a > 0) {
      le[a] = beta[a - 1] / ldg[a - 1];
      d -= le[a] * le[a];
    }
    if (!(d > 0.0)) return Status::make(VL_ERR_NOT_SPD, "the Lanczos matrix is not positive definite");
    ldg[a] = std::sqrt(d);
  }
  DevBuf<double> dl, de, Y, Y2, G1, G2;
  VL_TRY(dl.alloc(kk));
  VL_TRY(de.alloc(kk));
  VL_HIP(hipMemcpyAsync(dl.p, ldg.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
  VL_HIP(hipMemcpyAsync(de.p, le.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
  const int64_t nk = n * static_cast<int64_t>(kk);
  VL_TRY(Y.alloc(nk));
  VL_TRY(Y2.alloc(nk));
  VL_TRY(G1.alloc(static_cast<size_t>(np) * kk));
  const int64_t npk = np * static_cast<int64_t>(kk);
  if (form == 1) {
    // G = A_p B^{-1} (s o Q)
    hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks_of(nk)), dim3(256), 0, st, n, kk, k, s.p,
                       Q.p, Y2.p);
    VL_TRY(check_launch("lanczos scale rows"));
    VL_TRY(trsm_b(M, Y2.p, Y.p, kk, nullptr, false));
    hipLaunchKernelGGL(pred_gather_kernel, dim3(blocks_of(npk)), dim3(256), 0, st, np, m, kk,
                       M.pred_nbr.p, M.pred_bval.p, Y.p, G1.p);
  } else {
    VL_TRY(G2.alloc(static_cast<size_t>(np) * kk));
    // G1 = A_p ((s / W) o Q), G2 = A_p Sigma~ (s o Q)
    hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks_of(nk)), dim3(256), 0, st, n, kk, k, sw.p,
                       Q.p, Y.p);
    hipLaunchKernelGGL(pred_gather_kernel, dim3(blocks_of(npk)), dim3(256), 0, st, np, m, kk,
                       M.pred_nbr.p, M.pred_bval.p, Y.p, G1.p);
    hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks_of(nk)), dim3(256), 0, st, n, kk, k, s.p,
                       Q.p, Y2.p);
    VL_TRY(check_launch("lanczos scale rows"));
    VL_TRY(trsm_bt(M, Y2.p, Y.p, kk, false));
    VL_TRY(trsm_b(M, Y.p, Y2.p, kk, M.dval.p, false));
    hipLaunchKernelGGL(pred_gather_kernel, dim3(blocks_of(npk)), dim3(256), 0, st, np, m, kk,
                       M.pred_nbr.p, M.pred_bval.p, Y2.p, G2.p);
  }
  VL_TRY(check_launch("lanczos gather"));
  hipLaunchKernelGGL(lanczos_var_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, np,
                     kk, dl.p, de.p, G1.p, form == 2 ? G2.p : nullptr, M.pred_dval.p, var_out);
  VL_TRY(check_launch("lanczos variances"));
  VL_TRY(sync_stream(st));
  VL_TRY(read_status(M));
  M.last_lanczos_alpha = alpha;
  M.last_lanczos_beta = beta;
  if (info) info->cg_iters_max = 0;
  return Status::ok();
}

}  // namespace vl
