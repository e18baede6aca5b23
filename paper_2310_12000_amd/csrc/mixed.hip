// Mixed-precision form of the block solves: the n x t blocks, the values of
// B and B^T and the sparse products and triangular solves in FP32; every sum
// (row sums of the sparse kernels, CG dot products) accumulated in FP64; the
// solution refined in FP64 against the FP64 operator:
//   u = FP32-PCG(A, rhs);  repeat: r = rhs - A u (FP64);  stop when every
//   column has ||r||_2 < tol;  u += FP32-PCG(A, r).
// The Lanczos coefficients (and r0^T z0) of the first FP32 run feed the
// stochastic Lanczos quadrature; the tridiagonal eigensolve stays FP64.  The
// Newton mode update and the neighbour Cholesky stay FP64 everywhere.
//
// The FP32 triangular solves use the level-scheduled launches for every
// block width (one launch per level; no sentinel fill, no polling).
#include <algorithm>
#include <cmath>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

namespace vl {

// ------------------------------------------------------------ FP32 values
__global__ void to_f32_kernel(int64_t count, const double* __restrict__ x, float* __restrict__ y) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) y[e] = static_cast<float>(x[e]);
}

__global__ void to_f64_kernel(int64_t count, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) y[e] = static_cast<double>(x[e]);
}

__global__ void add_f32_kernel(int64_t count, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) y[e] += static_cast<double>(x[e]);
}

static unsigned nblk(int64_t count) { return static_cast<unsigned>((count + 255) / 256); }

Status to_f32(Model& M, const double* x, float* y, int64_t count) {
  if (count <= 0) return Status::ok();
  hipLaunchKernelGGL(to_f32_kernel, dim3(nblk(count)), dim3(256), 0, M.stream, count, x, y);
  return check_launch("to_f32");
}

// FP32 copies of the B and B^T values, refreshed once per factor.
static Status ensure_f32_values(Model& M) {
  if (M.f32_version == M.factor_version) return Status::ok();
  const int64_t nm = M.n * static_cast<int64_t>(M.m > 0 ? M.m : 1);
  VL_TRY(M.bval_f.reserve(nm));
  VL_TRY(M.bt_val_f.reserve(M.nnz > 0 ? M.nnz : 1));
  VL_TRY(to_f32(M, M.bval.p, M.bval_f.p, M.n * static_cast<int64_t>(M.m)));
  VL_TRY(to_f32(M, M.bt_val.p, M.bt_val_f.p, M.nnz));
  M.f32_version = M.factor_version;
  return Status::ok();
}

// ---------------------------------------------------- FP32 sparse kernels
// One wave per (row, 64-column slice), rows in spatial order.
//   ell:   Y_i = rs_i (X_i + sum_k vals[i,k] X_{nbr[i,k]})
//   csr_t: Y_j = d_j V_j + X_j + sum_e btval[e] X_{btcol[e]}
__global__ __launch_bounds__(256) void spmm_ell_f32_kernel(int64_t n, int m, int t, int slices,
                                                           const int* __restrict__ order,
                                                           const int* __restrict__ nbr,
                                                           const float* __restrict__ vals,
                                                           const float* __restrict__ X,
                                                           const double* __restrict__ rs,
                                                           float* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int64_t r = unit / slices;
  if (r >= n) return;
  const int c = static_cast<int>(unit - r * slices) * 64 + lane;
  if (c >= t) return;
  const int64_t i = order ? order[r] : r;
  double acc = X[i * t + c];
  for (int k0 = 0; k0 < m; k0 += 8) {
    int js[8];
    float vv[8], xs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      js[k] = (k0 + k < m) ? nbr[i * m + k0 + k] : -1;
      vv[k] = (k0 + k < m) ? vals[i * m + k0 + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[k] = js[k] >= 0 ? X[(int64_t)js[k] * t + c] : 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += static_cast<double>(vv[k]) * static_cast<double>(xs[k]);
  }
  if (rs) acc *= rs[i];
  Y[i * t + c] = static_cast<float>(acc);
}

__global__ __launch_bounds__(256) void spmm_csr_t_f32_kernel(
    int64_t n, int t, int slices, const int* __restrict__ order, const int* __restrict__ ptr,
    const int* __restrict__ col, const float* __restrict__ val, const float* __restrict__ X,
    const double* __restrict__ d, const float* __restrict__ V, float* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  const int64_t r = unit / slices;
  if (r >= n) return;
  const int c = static_cast<int>(unit - r * slices) * 64 + lane;
  if (c >= t) return;
  const int64_t i = order ? order[r] : r;
  double acc = X[i * t + c];
  const int b = ptr[i], e = ptr[i + 1];
  for (int q = b; q < e; q += 8) {
    int cs[8];
    float vs[8], xs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cs[k] = (q + k < e) ? col[q + k] : -1;
      vs[k] = (q + k < e) ? val[q + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[k] = cs[k] >= 0 ? X[(int64_t)cs[k] * t + c] : 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += static_cast<double>(vs[k]) * static_cast<double>(xs[k]);
  }
  if (d) acc += d[i] * static_cast<double>(V[i * t + c]);
  Y[i * t + c] = static_cast<float>(acc);
}

// Level-scheduled FP32 solve of one level; block (k, s) solves row rows[k]
// for the blockDim.x columns of slice s.
//   Y_i = rs_i X_i - sum_q vals[q] Y_{idx[q]},  q in [q0, e) (idx < 0 ends the row)
template <bool LOWER>
__global__ __launch_bounds__(256) void trsm_level_f32_kernel(int t, const int* __restrict__ rows,
                                                             int m, const int* __restrict__ ptr,
                                                             const int* __restrict__ idx,
                                                             const float* __restrict__ vals,
                                                             const float* __restrict__ X,
                                                             const double* __restrict__ rs,
                                                             float* __restrict__ Y) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t i = rows[blockIdx.x];
  if (c >= t) return;
  int q, e;
  if (LOWER) {
    q = static_cast<int>(i * m);
    e = q + m;
  } else {
    q = ptr[i];
    e = ptr[i + 1];
  }
  double acc = X[i * t + c];
  if (rs) acc *= rs[i];
  for (; q < e; q += 8) {
    int cb[8];
    float vb[8], yv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cb[k] = (q + k < e) ? idx[q + k] : -1;
      vb[k] = (q + k < e) ? vals[q + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) yv[k] = cb[k] >= 0 ? Y[(int64_t)cb[k] * t + c] : 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc -= static_cast<double>(vb[k]) * static_cast<double>(yv[k]);
  }
  Y[i * t + c] = static_cast<float>(acc);
}

static Status trsm_levels_f32(Model& M, bool lower, const float* X, float* Y, int t,
                              const double* rowscale) {
  const std::vector<int>& lp = lower ? M.lvl_ptr_f : M.lvl_ptr_b;
  const int* order = lower ? M.full_order_f.p : M.full_order_b.p;
  if (lp.size() < 2 || lp.back() != M.n) return Status::make(VL_ERR_STATE, "no level schedule");
  const int tb = t <= 64 ? 64 : 256;
  const unsigned gy = static_cast<unsigned>((t + tb - 1) / tb);
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    if (lower) {
      hipLaunchKernelGGL(trsm_level_f32_kernel<true>, dim3(rows, gy), dim3(tb), 0, M.stream, t,
                         order + lp[l], M.m, nullptr, M.nbr.p, M.bval_f.p, X, rowscale, Y);
    } else {
      hipLaunchKernelGGL(trsm_level_f32_kernel<false>, dim3(rows, gy), dim3(tb), 0, M.stream, t,
                         order + lp[l], 0, M.bt_ptr.p, M.bt_col.p, M.bt_val_f.p, X, nullptr, Y);
    }
  }
  return check_launch(lower ? "trsm level f32 lower" : "trsm level f32 upper");
}

static unsigned units_grid(int64_t n, int t) {
  const int64_t slices = (t + 63) / 64;
  return static_cast<unsigned>((n * slices + 3) / 4);
}

CgOpsF vadu_ops_f32(const double* W, const double* sdiag) {
  CgOpsF ops;
  ops.apply = [W](Model& M, const float* H, float* V, float* Tmp, int t) -> Status {
    // V = W o H + B^T (D^{-1} o (B H))
    const int slices = (t + 63) / 64;
    const int* ord = static_cast<const int*>(M.grid_pts);
    hipLaunchKernelGGL(spmm_ell_f32_kernel, dim3(units_grid(M.n, t)), dim3(256), 0, M.stream,
                       M.n, M.m, t, slices, ord, M.nbr.p, M.bval_f.p, H, M.dinv.p, Tmp);
    hipLaunchKernelGGL(spmm_csr_t_f32_kernel, dim3(units_grid(M.n, t)), dim3(256), 0, M.stream,
                       M.n, t, slices, ord, M.bt_ptr.p, M.bt_col.p, M.bt_val_f.p, Tmp, W, H, V);
    return check_launch("vadu apply f32");
  };
  ops.precond = [sdiag](Model& M, const float* R, float* Z, float* Y, int t) -> Status {
    // Z = B^{-1} ((W + D^{-1})^{-1} o (B^{-T} R))
    VL_TRY(trsm_levels_f32(M, false, R, Y, t, nullptr));
    return trsm_levels_f32(M, true, Y, Z, t, sdiag);
  };
  return ops;
}

// ------------------------------------------------------------- refinement
// res = float(rhs - AU) and per-column partial sums of (rhs - AU)^2 in FP64.
__global__ __launch_bounds__(256) void residual_kernel(ChunkGrid g, const double* __restrict__ rhs,
                                                       const double* __restrict__ AU,
                                                       float* __restrict__ res,
                                                       double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  const int64_t o = i * g.t + c;
  const double r = rhs[o] - AU[o];
  res[o] = static_cast<float>(r);
  acc += r * r;
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

Status block_solve_mixed(Model& M, CgState& S, const CgOps& ops64, const CgOpsF& ops32, int t,
                         const double* rhs, double tol, int max_iter, bool keep_z0,
                         int max_refine, MixedInfo* info) {
  const int64_t n = M.n, nt = n * static_cast<int64_t>(t);
  VL_TRY(ensure_f32_values(M));
  VL_TRY(M.mx_rhs.reserve(nt));
  VL_TRY(to_f32(M, rhs, M.mx_rhs.p, nt));
  VL_TRY(cg_solve_f32(M, S, ops32, t, M.mx_rhs.p, tol, max_iter, keep_z0));
  // widen the FP32 solution (and z_0) into FP64 blocks of S
  hipLaunchKernelGGL(to_f64_kernel, dim3(nblk(nt)), dim3(256), 0, M.stream, nt,
                     reinterpret_cast<const float*>(S.U.p), S.V.p);
  S.U.swap(S.V);
  if (keep_z0) {
    hipLaunchKernelGGL(to_f64_kernel, dim3(nblk(nt)), dim3(256), 0, M.stream, nt,
                       reinterpret_cast<const float*>(S.Z0.p), S.Tmp.p);
    S.Z0.swap(S.Tmp);
  }
  VL_TRY(check_launch("widen"));
  if (info) {
    info->first_iters = S.host_iters;
    info->refinements = 0;
    info->refine_iters_max = 0;
  }
  ChunkGrid g = ChunkGrid::of(n, t);
  VL_TRY(M.mx_a.reserve(nt));
  VL_TRY(M.mx_b.reserve(nt));
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * t));
  VL_TRY(M.red_out.reserve(2 * static_cast<size_t>(t) + 64));
  std::vector<double> rr(t);
  for (int k = 0;; ++k) {
    // FP64 residual of the current solution against the FP64 operator
    VL_TRY(ops64.apply(M, S.U.p, M.mx_a.p, M.mx_b.p, t));
    hipLaunchKernelGGL(residual_kernel, dim3(g.nchunk, g.L.slices), dim3(256), 0, M.stream, g,
                       rhs, M.mx_a.p, M.mx_rhs.p, M.red_part.p);
    VL_TRY(reduce_chunks(M.stream, M.red_part.p, g.nchunk, t, M.red_out.p));
    VL_HIP(hipMemcpyAsync(rr.data(), M.red_out.p, sizeof(double) * t, hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
    double worst = 0.0;
    for (int c = 0; c < t; ++c) worst = std::max(worst, std::sqrt(rr[c]));
    if (info) info->final_residual = worst;
    if (worst < tol || k >= max_refine) break;
    // correction: FP32 PCG on the residual, added in FP64
    VL_TRY(cg_solve_f32(M, M.cgm, ops32, t, M.mx_rhs.p, tol, max_iter, false));
    hipLaunchKernelGGL(add_f32_kernel, dim3(nblk(nt)), dim3(256), 0, M.stream, nt,
                       reinterpret_cast<const float*>(M.cgm.U.p), S.U.p);
    VL_TRY(check_launch("refine"));
    if (info) {
      info->refinements = k + 1;
      for (int v : M.cgm.host_iters) info->refine_iters_max = std::max(info->refine_iters_max, v);
    }
  }
  S.host_iters = info ? info->first_iters : S.host_iters;
  return read_status(M);
}

}  // namespace vl
