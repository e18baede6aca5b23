// Mixed-precision form of the block solves.  The preconditioner solves
//   Z = B^{-1} ((W + D^{-1})^{-1} o (B^{-T} R))      (P_VADU, Sec. 3.1.1)
// run in FP32: FP32 copies of the B and B^T values, FP32 n x t blocks for the
// intermediate and the result, every row sum accumulated in FP64.  They sit
// inside the FP64 block PCG: the operator W + B^T D^{-1} B, the residual
// recurrence, the dot products and the Lanczos coefficients stay FP64, so the
// outer iteration refines each FP32 solve against the FP64 operator and the
// stopping test applies to the FP64 residual.  The Newton update, the
// neighbour Cholesky, the tridiagonal eigensolve and all assembly stay FP64.
//
// The FP32 solves are level-scheduled (one launch per level of the
// dependency DAG; no sentinel fill, no polling).
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

// ------------------------------------------------------ FP32 level solves
// One level; block (k, s) solves row rows[k] for the blockDim.x columns of
// slice s:  Y_i = rs_i X_i - sum_q vals[q] Y_{idx[q]}  (idx < 0 ends the row),
// Y stored in FP32 (and, with Yd, also in FP64 for the CG), sums in FP64.
template <bool LOWER, typename TX>
__global__ __launch_bounds__(256) void trsm_level_mx_kernel(int t, const int* __restrict__ rows,
                                                            int m, const int* __restrict__ ptr,
                                                            const int* __restrict__ idx,
                                                            const float* __restrict__ vals,
                                                            const TX* __restrict__ X,
                                                            const double* __restrict__ rs,
                                                            float* __restrict__ Y,
                                                            double* __restrict__ Yd) {
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
  double acc = static_cast<double>(X[i * t + c]);
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
  if (Yd) Yd[i * t + c] = static_cast<double>(static_cast<float>(acc));
}

// Levels of long B^T rows (average length above 16): 4 waves per 64 columns
// share a row's entries (wave w takes q0 + w, q0 + w + 4, ...), partial sums
// added in wave order.
template <typename TX>
__global__ __launch_bounds__(256) void trsm_level_mx_split_kernel(
    int t, const int* __restrict__ rows, const int* __restrict__ ptr, const int* __restrict__ idx,
    const float* __restrict__ vals, const TX* __restrict__ X, float* __restrict__ Y) {
  __shared__ double s_part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + lane;
  const int64_t i = rows[blockIdx.x];
  const int b = ptr[i], e = ptr[i + 1];
  double part = 0.0;
  if (c < t) {
    for (int q = b + w; q < e; q += 4 * 8) {
      int cb[8];
      float vb[8], yv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        cb[k] = (q + 4 * k < e) ? idx[q + 4 * k] : -1;
        vb[k] = (q + 4 * k < e) ? vals[q + 4 * k] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) yv[k] = cb[k] >= 0 ? Y[(int64_t)cb[k] * t + c] : 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) part += static_cast<double>(vb[k]) * static_cast<double>(yv[k]);
    }
  }
  s_part[w][lane] = part;
  __syncthreads();
  if (w == 0 && c < t)
    Y[i * t + c] = static_cast<float>(static_cast<double>(X[i * t + c]) -
                                      (((s_part[0][lane] + s_part[1][lane]) + s_part[2][lane]) +
                                       s_part[3][lane]));
}

// Y (FP32) = B^{-T} X with X FP64.
static Status upper_f32(Model& M, const double* X, float* Y, int t) {
  const std::vector<int>& lp = M.lvl_ptr_b;
  const std::vector<int64_t>& lnz = M.lvl_nnz_b;
  if (lp.size() < 2 || lp.back() != M.n) return Status::make(VL_ERR_STATE, "no level schedule");
  const int tb = t <= 64 ? 64 : 256;
  const unsigned gy = static_cast<unsigned>((t + tb - 1) / tb);
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    const int* r = M.full_order_b.p + lp[l];
    if (lnz[l] > 16LL * rows) {
      hipLaunchKernelGGL(trsm_level_mx_split_kernel<double>, dim3(rows, (t + 63) / 64),
                         dim3(256), 0, M.stream, t, r, M.bt_ptr.p, M.bt_col.p, M.bt_val_f.p, X,
                         Y);
    } else {
      hipLaunchKernelGGL((trsm_level_mx_kernel<false, double>), dim3(rows, gy), dim3(tb), 0,
                         M.stream, t, r, 0, M.bt_ptr.p, M.bt_col.p, M.bt_val_f.p, X, nullptr, Y,
                         nullptr);
    }
  }
  return check_launch("trsm level f32 upper");
}

// Y (FP32) and Yd (FP64) = B^{-1} (rs o X) with X FP32.
static Status lower_f32(Model& M, const float* X, float* Y, double* Yd, int t,
                        const double* rs) {
  const std::vector<int>& lp = M.lvl_ptr_f;
  if (lp.size() < 2 || lp.back() != M.n) return Status::make(VL_ERR_STATE, "no level schedule");
  const int tb = t <= 64 ? 64 : 256;
  const unsigned gy = static_cast<unsigned>((t + tb - 1) / tb);
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    hipLaunchKernelGGL((trsm_level_mx_kernel<true, float>), dim3(rows, gy), dim3(tb), 0,
                       M.stream, t, M.full_order_f.p + lp[l], M.m, nullptr, M.nbr.p, M.bval_f.p,
                       X, rs, Y, Yd);
  }
  return check_launch("trsm level f32 lower");
}

CgOps vadu_ops(const double* W, const double* sdiag);

CgOps vadu_ops_mixed(const double* W, const double* sdiag) {
  CgOps ops = vadu_ops(W, sdiag);  // the FP64 operator
  ops.precond = [sdiag](Model& M, const double* R, double* Z, double* Y, int t) -> Status {
    (void)Y;
    VL_TRY(ensure_f32_values(M));
    const size_t nt = static_cast<size_t>(M.n) * t;
    VL_TRY(M.mx_rhs.reserve(nt));
    VL_TRY(M.mx_f2.reserve(nt));
    VL_TRY(upper_f32(M, R, M.mx_rhs.p, t));
    return lower_f32(M, M.mx_rhs.p, M.mx_f2.p, Z, t, sdiag);
  };
  ops.needs_fill = [](const Model&, int) { return false; };
  return ops;
}

}  // namespace vl
