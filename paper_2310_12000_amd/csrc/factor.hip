// Vecchia factor (Sec. 2.1): for every row i with neighbour set N(i) of size k,
//   A_i = Sigma_{N(i)}^{-1} Sigma_{N(i),i},  D_i = Sigma_ii - Sigma_{N(i),i}^T A_i,
// stored as B-matrix entries B_{i,N(i)} = -A_i (ELL, n x m) and D.  With
// derivatives (appendix "Derivatives of the Vecchia-approximated precision"):
//   dA_i = Sigma_N^{-1} (d Sigma_{N,i} - d Sigma_N A_i),
//   dD_i = d Sigma_ii - d Sigma_{N,i}^T A_i - Sigma_{N,i}^T dA_i,
// for theta = (sigma2, rho); for sigma2 the covariance scales linearly, so
// dA = 0 and dD = D / sigma2 exactly.
//
// One wave per row.  Lane c holds column c of the augmented SPD matrix
//   [ Sigma_N      Sigma_{N,i} ]
//   [ Sigma_{N,i}^T  Sigma_ii  ]
// (k + 1 columns, query last) in registers.  A right-looking Cholesky with
// lanes = columns broadcasts each finished column with v_readlane, so every
// update is a register FMA; the last row of the factor holds
// l = L_N^{-1} Sigma_{N,i} and its last pivot is D_i.  Back substitution
// L_N^T A_i = l then needs only broadcasts of finished unknowns.
// FP64 throughout: the neighbour covariances reach condition numbers near 1e9.
#include "vl_internal.h"

namespace vl {

template <int MM>
__global__ __launch_bounds__(256) void factor_kernel(
    const double* __restrict__ xy, const double* __restrict__ q_xy, int64_t nrows,
    const int* __restrict__ nbr, int m, int kind, double sigma2, double rho, int want_deriv,
    double* __restrict__ bval, double* __restrict__ dval, double* __restrict__ dbval_rho,
    double* __restrict__ dd_sigma2, double* __restrict__ dd_rho, int* __restrict__ status) {
  const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= nrows) return;  // uniform per wave
  const int* nb = nbr + w * m;
  const int jn = (lane < m) ? nb[lane] : -1;
  const int k = __popcll(__ballot(jn >= 0));  // neighbours form a prefix
  double px = 0.0, py = 0.0;
  if (lane < k) {
    px = xy[2 * (int64_t)jn];
    py = xy[2 * (int64_t)jn + 1];
  } else if (lane == k) {
    px = q_xy ? q_xy[2 * w] : xy[2 * w];
    py = q_xy ? q_xy[2 * w + 1] : xy[2 * w + 1];
  }

  // column `lane` of the augmented covariance
  double col[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    double rx = readlane(px, r), ry = readlane(py, r);
    double v = 0.0;
    if (r <= k && lane <= k) v = cov_eval(kind, sqdist(px, py, rx, ry), sigma2, rho);
    col[r] = v;
  }
  // covariance between this lane's neighbour and the query, kept for dD
  double cq = 0.0;
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r == k) cq = col[r];

  // right-looking Cholesky, lanes = columns (uniform predicates instead of
  // early exits, so every register index stays static after unrolling)
  bool spd = true;
  double dpiv = 0.0;
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    if (spd && j <= k) {
      const double piv = readlane(col[j], j);
      if (!(piv > 0.0)) {
        spd = false;
      } else if (j == k) {
        dpiv = piv;  // D_i = Sigma_ii - l^T l
      } else {
        const double dj = sqrt(piv);
        if (lane == j) {
          col[j] = dj;
#pragma unroll
          for (int r = j + 1; r < MM; ++r) col[r] = col[r] / dj;
        }
        double lcj = 0.0;
#pragma unroll
        for (int r = j + 1; r < MM; ++r) {
          if (r <= k) {
            const double lrj = readlane(col[r], j);
            if (lane == r) lcj = lrj;
            if (lane > j && lane <= r) col[r] -= lrj * lcj;
          }
        }
      }
    }
  }
  if (!spd) {
    if (lane == 0) raise_error(status, kErrNotSpd);
    return;
  }

  // l_lane = L[k][lane], diag = L[lane][lane]
  double l = 0.0, diag = 1.0;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    if (r == k) l = col[r];
    if (r == lane) diag = col[r];
  }

  // back substitution L_N^T a = l
  double a = 0.0;
  {
    double acc = 0.0;
#pragma unroll
    for (int j = MM - 1; j >= 0; --j) {
      if (j < k) {
        const double aj = readlane((l - acc) / diag, j);
        if (lane == j) a = aj;
        if (lane < j) acc += col[j] * aj;
      }
    }
  }

  double* brow = bval + w * m;
  if (lane < m) brow[lane] = (lane < k) ? -a : 0.0;
  if (lane == 0) dval[w] = dpiv;

  if (!want_deriv) return;

  // ---- d / d rho ----
  double dcol[MM];
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    double rx = readlane(px, r), ry = readlane(py, r);
    double v = 0.0;
    if (r <= k && lane <= k) v = cov_drho(kind, sqdist(px, py, rx, ry), sigma2, rho);
    dcol[r] = v;
  }
  double dcq = 0.0;
#pragma unroll
  for (int r = 0; r < MM; ++r)
    if (r == k) dcq = dcol[r];
  // rhs_c = d Sigma_{c,i} - sum_r d Sigma_{c,r} a_r  (d Sigma_N symmetric)
  double rhs = dcq;
#pragma unroll
  for (int r = 0; r < MM; ++r) {
    if (r < k) rhs -= dcol[r] * readlane(a, r);
  }
  // forward substitution L y = rhs
  double y = 0.0;
  {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      if (j < k) {
        const double yj = readlane((rhs - acc) / diag, j);
        if (lane == j) y = yj;
        double lcj = 0.0;
#pragma unroll
        for (int c = j + 1; c < MM; ++c) {
          if (c < k) {
            const double s = readlane(col[c], j);
            if (lane == c) lcj = s;
          }
        }
        if (lane > j && lane < k) acc += lcj * yj;
      }
    }
  }
  // back substitution L^T x = y
  double da = 0.0;
  {
    double acc = 0.0;
#pragma unroll
    for (int j = MM - 1; j >= 0; --j) {
      if (j < k) {
        const double xj = readlane((y - acc) / diag, j);
        if (lane == j) da = xj;
        if (lane < j) acc += col[j] * xj;
      }
    }
  }
  // dD = - dc^T a - c^T da
  double part = (lane < k) ? (dcq * a + cq * da) : 0.0;
  part = wave_sum(part);
  if (lane < m) dbval_rho[w * m + lane] = (lane < k) ? -da : 0.0;
  if (lane == 0) {
    dd_rho[w] = -part;
    dd_sigma2[w] = dpiv / sigma2;
  }
}

Status factor_rows(Model& M, const double* q_xy, int64_t nrows, const int* nbr, double* bval,
                   double* dval, bool deriv, double* dbval_rho, double* dd_sigma2,
                   double* dd_rho) {
  if (nrows == 0) return Status::ok();
  const int m = M.m;
  const int waves_per_block = 4;
  const unsigned gb = static_cast<unsigned>((nrows + waves_per_block - 1) / waves_per_block);
  const dim3 blk(64 * waves_per_block);
#define VL_FACTOR_LAUNCH(MMV)                                                                 \
  hipLaunchKernelGGL(factor_kernel<MMV>, dim3(gb), blk, 0, M.stream, M.coords, q_xy, nrows,   \
                     nbr, m, M.cov, M.sigma2, M.rho, deriv ? 1 : 0, bval, dval, dbval_rho,     \
                     dd_sigma2, dd_rho, M.status)
  if (m + 1 <= 8) {
    VL_FACTOR_LAUNCH(8);
  } else if (m + 1 <= 16) {
    VL_FACTOR_LAUNCH(16);
  } else if (m + 1 <= 24) {
    VL_FACTOR_LAUNCH(24);
  } else if (m + 1 <= 32) {
    VL_FACTOR_LAUNCH(32);
  } else {
    return Status::invalid("m exceeds 31");
  }
#undef VL_FACTOR_LAUNCH
  return check_launch("vecchia factor");
}

}  // namespace vl
