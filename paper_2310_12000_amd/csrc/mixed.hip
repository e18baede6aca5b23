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
// Blocks wider than 64 columns use level-scheduled FP32 solves (one launch
// per level of the dependency DAG; no sentinel fill, no polling; FP32 B
// values), and B^T solves fold the head rows' tail entries in one launch
// between the tail and the head levels; the leading rows covered by the
// dense inverse G come from its FP64 GEMM, which reads and writes the FP32
// blocks.  Narrower blocks run the FP64 path's kernels (dense leading block,
// sync-free tail) with FP32 right-hand sides and results: FP64 B values and
// G, FP64 sums.
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
// A thread covers VEC adjacent columns (16-byte accesses: VEC = 4 floats when
// the width allows), so a wave gathers 256 columns of a neighbour row with one
// instruction; every column keeps its own FP64 accumulator.
int level_vec(int t, int elem_bytes, const void* a, const void* b, const void* c);

// Forward level: block (k, s) solves row rows[k] for its slice of columns,
// Y_i = rs_i X_i - sum_k vals[i,k] Y_{nbr[i,k]} in slot order (an empty slot
// ends the row); Y stored in FP32 and, with Yd, also in FP64 for the CG; the
// sum in FP64.
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_mx_lower_kernel(
    int t, const int* __restrict__ rows, int m, const int* __restrict__ idx,
    const float* __restrict__ vals, const float* __restrict__ X, const double* __restrict__ rs,
    float* __restrict__ Y, double* __restrict__ Yd) {
  const int c = (blockIdx.y * blockDim.x + threadIdx.x) * VEC;
  const int64_t i = rows[blockIdx.x];
  if (c >= t) return;
  const int* nb = idx + i * m;
  const float* vb = vals + i * m;
  float x[VEC];
  vld<VEC>(X + i * t + c, x);
  double acc[VEC];
  const double s = rs ? rs[i] : 1.0;
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = rs ? static_cast<double>(x[v]) * s : static_cast<double>(x[v]);
  for (int q = 0; q < m; q += 8) {
    int cb[8];
    float w[8], y[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cb[k] = (q + k < m) ? nb[q + k] : -1;
      w[k] = (q + k < m) ? vb[q + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] >= 0) {
        vld<VEC>(Y + (int64_t)cb[k] * t + c, y[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) y[k][v] = 0.0f;
      }
    }
    bool ended = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] < 0) ended = true;
      if (!ended) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          acc[v] -= static_cast<double>(w[k]) * static_cast<double>(y[k][v]);
      }
    }
    if (ended) break;
  }
  float out[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) out[v] = static_cast<float>(acc[v]);
  vst<VEC>(Y + i * t + c, out);
  if (Yd) {
    double od[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) od[v] = static_cast<double>(out[v]);
    vst<VEC>(Yd + i * t + c, od);
  }
}

// Backward level over the entries [ptr[i], pend ? pend[i] : ptr[i + 1]); X in
// FP64 (the PCG residual, or the folded head right-hand side), Y in FP32, the
// sum in FP64.
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_mx_upper_kernel(
    int t, const int* __restrict__ rows, const int* __restrict__ ptr,
    const int* __restrict__ pend, const int* __restrict__ idx, const float* __restrict__ vals,
    const double* __restrict__ X, float* __restrict__ Y) {
  const int c = (blockIdx.y * blockDim.x + threadIdx.x) * VEC;
  const int64_t i = rows[blockIdx.x];
  if (c >= t) return;
  int q = ptr[i];
  const int e = pend ? pend[i] : ptr[i + 1];
  double acc[VEC];
  vld<VEC>(X + i * t + c, acc);
  for (; q < e; q += 8) {
    int cb[8];
    float w[8], y[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cb[k] = (q + k < e) ? idx[q + k] : -1;
      w[k] = (q + k < e) ? vals[q + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] >= 0) {
        vld<VEC>(Y + (int64_t)cb[k] * t + c, y[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) y[k][v] = 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (cb[k] >= 0) {
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          acc[v] -= static_cast<double>(w[k]) * static_cast<double>(y[k][v]);
      }
  }
  float out[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) out[v] = static_cast<float>(acc[v]);
  vst<VEC>(Y + i * t + c, out);
}

// Backward levels of long rows (average length above 16): 4 waves per
// 64 * VEC columns share a row's entries, partial sums added in wave order.
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_mx_split_kernel(
    int t, const int* __restrict__ rows, const int* __restrict__ ptr,
    const int* __restrict__ pend, const int* __restrict__ idx, const float* __restrict__ vals,
    const double* __restrict__ X, float* __restrict__ Y) {
  const int c = (blockIdx.y * 64 + (threadIdx.x & 63)) * VEC;
  const int64_t i = rows[blockIdx.x];
  const int b = ptr[i], e = pend ? pend[i] : ptr[i + 1];
  double tot[VEC];
  if (!split_row_sum<VEC>(t, c, b, e, idx, vals, Y, tot)) return;
  double x[VEC];
  vld<VEC>(X + i * t + c, x);
  float out[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) out[v] = static_cast<float>(x[v] - tot[v]);
  vst<VEC>(Y + i * t + c, out);
}

template <int VEC>
static void launch_upper_f32(Model& M, bool split, int rows, int t, const int* r, const int* pend,
                             const double* X, float* Y) {
  const int tb = t <= 64 ? 64 : 256;
  if (split) {
    const dim3 grid(rows, (t + 64 * VEC - 1) / (64 * VEC));
    hipLaunchKernelGGL(trsm_level_mx_split_kernel<VEC>, grid, dim3(256), 0, M.stream, t, r,
                       M.bt_ptr.p, pend, M.bt_col.p, M.bt_val_f.p, X, Y);
  } else {
    const dim3 grid(rows, (t + tb * VEC - 1) / (tb * VEC));
    hipLaunchKernelGGL(trsm_level_mx_upper_kernel<VEC>, grid, dim3(tb), 0, M.stream, t, r,
                       M.bt_ptr.p, pend, M.bt_col.p, M.bt_val_f.p, X, Y);
  }
}

static Status upper_levels_f32(Model& M, const std::vector<int>& lp,
                               const std::vector<int64_t>& lnz, const int* order, const int* pend,
                               const double* X, float* Y, int t) {
  const int vec = level_vec(t, 4, X, Y, nullptr);
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    const bool split = lnz[l] > 16LL * rows;
    const int* r = order + lp[l];
    if (vec == 4) {
      launch_upper_f32<4>(M, split, rows, t, r, pend, X, Y);
    } else if (vec == 2) {
      launch_upper_f32<2>(M, split, rows, t, r, pend, X, Y);
    } else {
      launch_upper_f32<1>(M, split, rows, t, r, pend, X, Y);
    }
  }
  return check_launch("trsm level f32 upper");
}

// Y (FP32) = B^T^{-1} X with X FP64: tail rows by level, the fold of the head
// rows' tail entries (FP64), then the head rows by head-internal level; with
// the dense leading rows, the head rows from Kw on by their levels and the
// rows below Kw from G's leading block (as in the FP64 wide solves).
static Status upper_f32(Model& M, const double* X, float* Y, int t) {
  const int64_t H = M.head_rows;
  if (M.hlv_ptr_b.size() < 2 || M.hlv_ptr_b.back() != H ||
      (M.n > H && (M.tlvl_ptr_b.size() < 2 || M.tlvl_ptr_b.back() != M.n - H)))
    return Status::make(VL_ERR_STATE, "no level schedule");
  if (M.n > H)
    VL_TRY(upper_levels_f32(M, M.tlvl_ptr_b, M.tlvl_nnz_b, M.tail_order_b.p, nullptr, X, Y, t));
  VL_TRY(M.lvl_fold.reserve(static_cast<size_t>(H) * t));
  VL_TRY(fold_launch_f32(M, X, Y, M.lvl_fold.p, t));
  if (M.dense_wide > 0) {
    if (M.dhlv_ptr_b.size() < 2 || M.dhlv_ptr_b.back() != H - M.dense_wide)
      return Status::make(VL_ERR_STATE, "no level schedule");
    VL_TRY(upper_levels_f32(M, M.dhlv_ptr_b, M.dhlv_nnz_b, M.dhlv_rows_b.p, M.head_split.p,
                            M.lvl_fold.p, Y, t));
    return dense_wide_upper_f32(M, M.lvl_fold.p, Y, t);
  }
  return upper_levels_f32(M, M.hlv_ptr_b, M.hlv_nnz_b, M.hlv_rows_b.p, M.head_split.p,
                          M.lvl_fold.p, Y, t);
}

template <int VEC>
static void launch_lower_f32(Model& M, int rows, int t, const int* r, const float* X,
                             const double* rs, float* Y, double* Yd) {
  const int tb = t <= 64 ? 64 : 256;
  const dim3 grid(rows, (t + tb * VEC - 1) / (tb * VEC));
  hipLaunchKernelGGL(trsm_level_mx_lower_kernel<VEC>, grid, dim3(tb), 0, M.stream, t, r, M.m,
                     M.nbr.p, M.bval_f.p, X, rs, Y, Yd);
}

// Y (FP32) and Yd (FP64) = B^{-1} (rs o X) with X FP32: the full level
// order or, with the dense leading rows, those from G's leading block and
// the rest by the levels computed with them known.
static Status lower_f32(Model& M, const float* X, float* Y, double* Yd, int t,
                        const double* rs) {
  const bool dense = M.dense_wide > 0;
  const std::vector<int>& lp = dense ? M.dlvl_ptr_f : M.lvl_ptr_f;
  const int* order = dense ? M.dfull_order_f.p : M.full_order_f.p;
  if (lp.size() < 2 || lp.back() != M.n - (dense ? M.dense_wide : 0))
    return Status::make(VL_ERR_STATE, "no level schedule");
  if (dense) VL_TRY(dense_wide_lower_f32(M, X, Y, Yd, t, rs));
  const int vec = level_vec(t, 4, X, Y, Yd);
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    const int* r = order + lp[l];
    if (vec == 4) {
      launch_lower_f32<4>(M, rows, t, r, X, rs, Y, Yd);
    } else if (vec == 2) {
      launch_lower_f32<2>(M, rows, t, r, X, rs, Y, Yd);
    } else {
      launch_lower_f32<1>(M, rows, t, r, X, rs, Y, Yd);
    }
  }
  return check_launch("trsm level f32 lower");
}

CgOps vadu_ops(const double* W, const double* sdiag);

__global__ void column_kernel(int64_t n, int t, const double* __restrict__ X,
                              double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[i * t];
}

// Relative 2-norm deviation of the FP32 preconditioner application (the
// level-scheduled FP32 solves of the mixed form) from the FP64 one on the
// first column of X (n x t): z = B^{-1} (sdiag o B^{-T} x) both ways.
// Z (FP64) = Zf (FP32) widened
__global__ void to_f64_kernel(int64_t count, const float* __restrict__ x, double* __restrict__ y) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) y[e] = static_cast<double>(x[e]);
}

Status precond_f32_deviation(Model& M, const double* sdiag, const double* X, int t,
                             double* dev) {
  const int64_t n = M.n;
  VL_TRY(ensure_f32_values(M));
  VL_TRY(M.mx_chk.reserve(static_cast<size_t>(4 * n)));
  double* x = M.mx_chk.p;
  double* z64 = x + n;
  double* z32 = z64 + n;
  float* f1 = reinterpret_cast<float*>(z32 + n);
  float* f2 = f1 + n;
  const int tb = 256;
  hipLaunchKernelGGL(column_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, M.stream,
                     n, t, X, x);
  VL_TRY(check_launch("column"));
  VL_TRY(M.vec_d.reserve(n));
  VL_TRY(trsm_bt_slot(M, x, M.vec_d.p, 1, false, 0));
  VL_TRY(trsm_b_slot(M, M.vec_d.p, z64, 1, sdiag, false, 1));
  if (t <= 64 && !M.force_levels && !M.bd_use) {  // the narrow FP32 kernels the block uses
    VL_TRY(trsm_bt_f32_narrow(M, x, f1, 1));
    VL_TRY(trsm_b_f32_narrow(M, f1, f2, 1, sdiag));
    hipLaunchKernelGGL(to_f64_kernel, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, M.stream,
                       n, f2, z32);
    VL_TRY(check_launch("to_f64"));
  } else {
    VL_TRY(upper_f32(M, x, f1, 1));
    VL_TRY(lower_f32(M, f1, f2, z32, 1, sdiag));
  }
  std::vector<double> a(n), b(n);
  VL_HIP(hipMemcpyAsync(a.data(), z64, sizeof(double) * n, hipMemcpyDeviceToHost, M.stream));
  VL_HIP(hipMemcpyAsync(b.data(), z32, sizeof(double) * n, hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  VL_TRY(read_status(M));
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    num += (b[i] - a[i]) * (b[i] - a[i]);
    den += a[i] * a[i];
  }
  *dev = den > 0.0 ? std::sqrt(num / den) : 0.0;
  return Status::ok();
}

CgOps vadu_ops_mixed(const double* W, const double* sdiag) {
  CgOps ops = vadu_ops(W, sdiag);  // the FP64 operator
  // FP32 solves at every width: wide blocks level-scheduled with FP32 B
  // values; narrow blocks (t <= 64) through the dense block and sync-free tail
  // with FP32 right-hand sides and results, which fill their own FP32
  // outputs with the sentinel (the FP64 blocks need no fill).
  ops.precond = [sdiag](Model& M, const double* R, double* Z, double* Y, int t) -> Status {
    (void)Y;
    const size_t nt = static_cast<size_t>(M.n) * t;
    VL_TRY(M.mx_rhs.reserve(nt));
    VL_TRY(M.mx_f2.reserve(nt));
    if (t <= 64 && !M.force_levels && !M.bd_use) {
      VL_TRY(trsm_bt_f32_narrow(M, R, M.mx_rhs.p, t));
      VL_TRY(trsm_b_f32_narrow(M, M.mx_rhs.p, M.mx_f2.p, t, sdiag));
      hipLaunchKernelGGL(to_f64_kernel, dim3(nblk(static_cast<int64_t>(nt))), dim3(256), 0,
                         M.stream, static_cast<int64_t>(nt), M.mx_f2.p, Z);
      return check_launch("to_f64");
    }
    VL_TRY(ensure_f32_values(M));
    VL_TRY(upper_f32(M, R, M.mx_rhs.p, t));
    return lower_f32(M, M.mx_rhs.p, M.mx_f2.p, Z, t, sdiag);
  };
  ops.needs_fill = [](const Model&, int) { return false; };
  return ops;
}

}  // namespace vl
