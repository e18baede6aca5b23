// Low-rank pivoted-Cholesky preconditioner P_LRAC = L_k L_k^T + W^{-1}
// (Sec. 3.1.2, eq. P_LRAC) and the operator Sigma~ + W^{-1} of eq. (pcls2).
//
//   L_k   n x k pivoted Cholesky factor of the covariance matrix Sigma built
//         from the coordinates: the pivot is the largest residual diagonal
//         (first index on ties), column j = (Sigma[:, p] - L L^T[:, p]) /
//         sqrt(d_p), d -= column^2.  Stored row-major n x K, K = k rounded
//         up to 16, with zero columns past k.
//   M     I_K + L^T W L (K x K), its Cholesky factor C and log det M; the
//         padded columns give identity rows, so log det M is that of the
//         k x k matrix.  log det P = log det M - sum log W (determinant lemma).
//   P^{-1} R = W o R - W o (L M^{-1} (L^T (W o R)))   (Woodbury), M^{-1}
//         formed once per factor from C and applied as a K x K product
//
// The dense panels L^T diag(w) X (K x t, a reduction over the n rows) and
// L Y (n x t) run on the FP64 matrix cores (v_mfma_f64_16x16x4f64): a wave
// owns 16 x 16 output tiles and steps through the contraction 4 at a time.
// Operand layout of one step, lane l = 16 q + i (q = l / 16, i = l mod 16):
// A[i][q] and B[q][i] in, D[q + 4 r][i] (r = 0..3) out (measured on gfx950).
#include <algorithm>
#include <vector>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

namespace vl {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------- pivoted Cholesky
__global__ void pc_init_kernel(int64_t n, int K, double sigma2, double* __restrict__ d,
                               double* __restrict__ L, int* __restrict__ piv,
                               double* __restrict__ pval) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) d[g] = sigma2;  // c(0) = sigma2 for both covariance functions
  for (int64_t e = g; e < n * K; e += (int64_t)gridDim.x * blockDim.x) L[e] = 0.0;
  if (g == 0) {
    piv[0] = 0;  // all diagonals equal: the first index
    pval[0] = sigma2;
  }
}

// Column j with pivot piv[j] (pval[j] = its residual diagonal), the update of
// d, and per-block (max d, smallest index) candidates for the next pivot.
__global__ __launch_bounds__(256) void pc_column_kernel(
    int64_t n, int K, int j, const double* __restrict__ coords, int kind, double sigma2,
    double rho, const int* __restrict__ piv, const double* __restrict__ pval,
    double* __restrict__ d, double* __restrict__ L, double* __restrict__ part_v,
    int* __restrict__ part_i, int* __restrict__ status) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int p = piv[j];
  const double dp = pval[j];
  if (!(dp > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_error(status, kErrNotSpd);
  }
  const double inv = 1.0 / sqrt(dp);
  const double px = coords[2 * (int64_t)p], py = coords[2 * (int64_t)p + 1];
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double c = cov_eval(kind, sqdist(coords[2 * i], coords[2 * i + 1], px, py), sigma2, rho);
    double dot = 0.0;
    for (int l = 0; l < j; ++l) dot += L[i * K + l] * L[(int64_t)p * K + l];
    const double v = (c - dot) * inv;
    L[i * K + j] = v;
    const double dn = d[i] - v * v;
    d[i] = dn;
    if (dn > best) {  // rows visited in increasing order: the first maximum stays
      best = dn;
      bi = static_cast<int>(i);
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v2 = sv[threadIdx.x + o];
      const int i2 = si[threadIdx.x + o];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_v[blockIdx.x] = sv[0];
    part_i[blockIdx.x] = si[0];
  }
}

__global__ __launch_bounds__(256) void pc_argmax_kernel(int nparts, const double* __restrict__ part_v,
                                                        const int* __restrict__ part_i, int j,
                                                        const double* __restrict__ d,
                                                        int* __restrict__ piv,
                                                        double* __restrict__ pval) {
  __shared__ double sv[256];
  __shared__ int si[256];
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int b = threadIdx.x; b < nparts; b += 256) {
    const double v = part_v[b];
    const int i = part_i[b];
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double v2 = sv[threadIdx.x + o];
      const int i2 = si[threadIdx.x + o];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    piv[j + 1] = si[0];
    pval[j + 1] = d[si[0]];
  }
}

// ------------------------------------------------------------ MFMA panels
// part[blk] (K x ldp) = sum over the block's rows r of L[r, :]^T (w_r X[r, :]),
// columns of X beyond t read as 0.  Each block covers rows [r0, r1); wave w
// owns tiles w, w + 4, ... of the (K / 16) x (ldp / 16) tile grid.
__global__ __launch_bounds__(256) void gram_kernel(int64_t n, int K, int64_t rows_per_block,
                                                   const double* __restrict__ L,
                                                   const double* __restrict__ w,
                                                   const double* __restrict__ X, int ldx, int t,
                                                   int ldp, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i = lane & 15;
  const int64_t r0 = blockIdx.x * rows_per_block;
  int64_t r1 = r0 + rows_per_block;
  if (r1 > n) r1 = n;
  const int ta = K / 16, tb = ldp / 16;
  double* out = part + (int64_t)blockIdx.x * K * ldp;
  for (int tile = wave; tile < ta * tb; tile += 4) {
    const int a = tile / tb, b = tile - (tile / tb) * tb;
    const int col = b * 16 + i;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r = r0; r < r1; r += 4) {
      const int64_t rr = r + q;
      const bool in = rr < r1;
      const double av = in ? L[rr * K + a * 16 + i] : 0.0;
      const double bv = (in && col < t) ? (w ? w[rr] : 1.0) * X[rr * ldx + col] : 0.0;
      acc = mfma16x16x4(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(int64_t)(a * 16 + q + 4 * r) * ldp + b * 16 + i] = acc[r];
  }
}

// out (K x ldp) = sum of the parts (deterministic): a block takes 64
// consecutive elements; wave w adds parts w, w + 4, ... in order (each read
// a coalesced 512-byte row of the part array), then the four wave sums are
// added in wave order.
__global__ __launch_bounds__(256) void gram_reduce_kernel(int nparts, int64_t size,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ out) {
  __shared__ double sw[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t e = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (e < size)
    for (int b = wave; b < nparts; b += 4) s += part[(int64_t)b * size + e];
  sw[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && e < size) out[e] = ((sw[0][lane] + sw[1][lane]) + sw[2][lane]) + sw[3][lane];
}

// Z (n x t) = epilogue(L Y), Y K x ldy; one 16 x 16 output tile per wave.
//   mode 0:  Z = w o (R - L Y)                       (Woodbury)
//   mode 1:  Z = L Y + eps_n / sqrt(W), eps_n Rademacher (probe of P_LRAC)
__global__ __launch_bounds__(256) void panel_kernel(int64_t n, int K, const double* __restrict__ L,
                                                    const double* __restrict__ Y, int ldy, int t,
                                                    int mode, const double* __restrict__ w,
                                                    const double* __restrict__ R,
                                                    uint64_t seed, double* __restrict__ Z) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i = lane & 15;
  const int tcols = (t + 15) / 16;
  const int64_t tile = blockIdx.x * 4 + wave;
  const int64_t rt = tile / tcols;
  const int ct = static_cast<int>(tile - rt * tcols);
  const int64_t row0 = rt * 16;
  if (row0 >= n) return;
  const int col = ct * 16 + i;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t ra = row0 + i;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const double av = ra < n ? L[ra * K + k0 + q] : 0.0;
    const double bv = col < t ? Y[(int64_t)(k0 + q) * ldy + col] : 0.0;
    acc = mfma16x16x4(av, bv, acc);
  }
  if (col >= t) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + q + 4 * r;
    if (row >= n) continue;
    const int64_t e = row * t + col;
    if (mode == 0) {
      Z[e] = w[row] * (R[e] - acc[r]);
    } else {
      Z[e] = acc[r] + rademacher(seed, kTagLracN, (uint64_t)col, (uint64_t)row) / sqrt(w[row]);
    }
  }
}

// Cholesky of M (K x K, row-major, in place: lower factor) by one block, and
// log det M = 2 sum log C_jj.
__global__ __launch_bounds__(256) void small_cholesky_kernel(int K, double* __restrict__ Mx,
                                                             double* __restrict__ logdet,
                                                             int* __restrict__ status) {
  extern __shared__ double a[];
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) a[e] = Mx[e];
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    if (threadIdx.x == 0) {
      double s = a[j * K + j];
      for (int l = 0; l < j; ++l) s -= a[j * K + l] * a[j * K + l];
      if (!(s > 0.0)) raise_error(status, kErrNotSpd);
      a[j * K + j] = sqrt(s > 0.0 ? s : 1.0);
    }
    __syncthreads();
    const double djj = a[j * K + j];
    for (int i = j + 1 + threadIdx.x; i < K; i += blockDim.x) {
      double s = a[i * K + j];
      for (int l = 0; l < j; ++l) s -= a[i * K + l] * a[j * K + l];
      a[i * K + j] = s / djj;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int r = e / K, c = e - (e / K) * K;
    Mx[e] = c <= r ? a[e] : 0.0;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < K; ++j) s += log(a[j * K + j]);
    *logdet = 2.0 * s;
  }
}

// M = I + G (G = L^T W L), in place.
__global__ void add_identity_kernel(int K, double* __restrict__ Mx) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < K) Mx[e * K + e] += 1.0;
}

// Minv (K x K) = M^{-1} from the Cholesky factor C (M = C C^T): column b by
// C y = e_b, C^T x = y; one thread per column, once per factor.
__global__ void chol_inverse_kernel(int K, const double* __restrict__ C,
                                    double* __restrict__ Minv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= K) return;
  for (int i = 0; i < K; ++i) {
    double v = (i == b) ? 1.0 : 0.0;
    for (int l = 0; l < i; ++l) v -= C[i * K + l] * Minv[(int64_t)l * K + b];
    Minv[(int64_t)i * K + b] = v / C[i * K + i];
  }
  for (int i = K - 1; i >= 0; --i) {
    double v = Minv[(int64_t)i * K + b];
    for (int l = i + 1; l < K; ++l) v -= C[l * K + i] * Minv[(int64_t)l * K + b];
    Minv[(int64_t)i * K + b] = v / C[i * K + i];
  }
}

// Y (K x ld) = Minv S (columns < t): one thread per output element.
__global__ void small_gemm_kernel(int K, int t, int ld, const double* __restrict__ Minv,
                                  const double* __restrict__ S, double* __restrict__ Y) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * ld) return;
  const int a = static_cast<int>(e / ld), c = static_cast<int>(e - (e / ld) * ld);
  if (c >= t) {
    Y[e] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int b = 0; b < K; ++b) acc += Minv[(int64_t)a * K + b] * S[(int64_t)b * ld + c];
  Y[e] = acc;
}

// E (K x ld): Rademacher eps_k for rows < k, 0 for the padded rows.
__global__ void lrac_probe_k_kernel(int K, int k, int t, int ld, uint64_t seed,
                                    double* __restrict__ E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * ld) return;
  const int r = e / ld, c = e - (e / ld) * ld;
  E[e] = (r < k && c < t) ? rademacher(seed, kTagLracK, (uint64_t)c, (uint64_t)r) : 0.0;
}

// V += H / W
__global__ void add_div_kernel(int64_t n, int t, const double* __restrict__ H,
                               const double* __restrict__ W, double* __restrict__ V) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * t) return;
  V[e] += H[e] / W[e / t];
}

// b = U / W
__global__ void div_kernel(int64_t n, const double* __restrict__ U, const double* __restrict__ W,
                           double* __restrict__ b) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) b[e] = U[e] / W[e];
}

static unsigned blocks_for(int64_t count) {
  return static_cast<unsigned>((count + 255) / 256);
}

// ------------------------------------- derivative of the pivoted Cholesky
// Forward-mode derivative of the pivoted Cholesky steps with the pivots held
// fixed (q = 0: sigma2, q = 1: rho): with s = sqrt(d_p), column j =
// (Sigma[:, p] - L L_p^T) / s and d_p's derivative dd_p,
//   dL[:, j] = (dSigma[:, p] - dL L_p^T - L dL_p^T - L[:, j] dd_p / (2 s)) / s,
//   dd -= 2 L[:, j] o dL[:, j].
// snap[2 j + q] = dd_q[piv[j]] before column j (read by every row).
__global__ void pc_deriv_snap_kernel(int j, const int* __restrict__ piv,
                                     const double* __restrict__ dd0,
                                     const double* __restrict__ dd1, double* __restrict__ snap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int p = piv[j];
    snap[2 * j] = dd0[p];
    snap[2 * j + 1] = dd1[p];
  }
}

__global__ __launch_bounds__(256) void pc_deriv_column_kernel(
    int64_t n, int K, int j, const double* __restrict__ coords, int kind, double sigma2,
    double rho, const int* __restrict__ piv, const double* __restrict__ pval,
    const double* __restrict__ L, double* __restrict__ dL0, double* __restrict__ dL1,
    double* __restrict__ dd0, double* __restrict__ dd1, const double* __restrict__ snap) {
  const int p = piv[j];
  const double sq = sqrt(pval[j]);
  const double ds0 = snap[2 * j] / (2.0 * sq), ds1 = snap[2 * j + 1] / (2.0 * sq);
  const double px = coords[2 * (int64_t)p], py = coords[2 * (int64_t)p + 1];
  const double* Lp = L + (int64_t)p * K;
  const double* dLp0 = dL0 + (int64_t)p * K;
  const double* dLp1 = dL1 + (int64_t)p * K;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d2 = sqdist(coords[2 * i], coords[2 * i + 1], px, py);
    double n0 = cov_eval(kind, d2, 1.0, rho);  // d c / d sigma2 = c / sigma2
    double n1 = cov_drho(kind, d2, sigma2, rho);
    const double* Li = L + i * K;
    double* dLi0 = dL0 + i * K;
    double* dLi1 = dL1 + i * K;
    double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0;
    for (int l = 0; l < j; ++l) {
      a0 += dLi0[l] * Lp[l];
      b0 += Li[l] * dLp0[l];
      a1 += dLi1[l] * Lp[l];
      b1 += Li[l] * dLp1[l];
    }
    const double lij = Li[j];
    const double v0 = ((n0 - a0 - b0) - lij * ds0) / sq;
    const double v1 = ((n1 - a1 - b1) - lij * ds1) / sq;
    dLi0[j] = v0;
    dLi1[j] = v1;
    dd0[i] -= 2.0 * lij * v0;
    dd1[i] -= 2.0 * lij * v1;
  }
}

// dd_sigma2 = 1 (c(0) = sigma2), dd_rho = 0, dL = 0
__global__ void pc_deriv_init_kernel(int64_t n, int K, double* __restrict__ dL0,
                                     double* __restrict__ dL1, double* __restrict__ dd0,
                                     double* __restrict__ dd1) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) {
    dd0[g] = 1.0;
    dd1[g] = 0.0;
  }
  for (int64_t e = g; e < n * K; e += (int64_t)gridDim.x * blockDim.x) {
    dL0[e] = 0.0;
    dL1[e] = 0.0;
  }
}

// lev[i] = L_i M^{-1} L_i^T = |C^{-1} L_i^T|^2 (C the Cholesky factor of M)
__global__ void lrac_leverage_kernel(int64_t n, int K, const double* __restrict__ L,
                                     const double* __restrict__ C, double* __restrict__ lev) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double y[128];
  const double* Li = L + i * K;
  double acc = 0.0;
  for (int a = 0; a < K; ++a) {
    double v = Li[a];
    for (int l = 0; l < a; ++l) v -= C[a * K + l] * y[l];
    v /= C[a * K + a];
    y[a] = v;
    acc += v * v;
  }
  lev[i] = acc;
}

// Per column c of the n x t blocks X, Y: part_k[chunk, c] = sum over the
// chunk's rows of X^T (d Sigma~^{-1} / d theta_k) Y restricted to the row,
// i.e. dBx' D^{-1} By + Bx' D^{-1} dBy - Bx' D^{-2} dD_k By (dB_sigma2 = 0).
__global__ __launch_bounds__(256) void dprec_form_kernel(
    ChunkGrid g, int m, const int* __restrict__ nbr, const double* __restrict__ bval,
    const double* __restrict__ dbval, const double* __restrict__ X,
    const double* __restrict__ Y, const double* __restrict__ D,
    const double* __restrict__ dd_s2, const double* __restrict__ dd_rho,
    double* __restrict__ part) {
  double s0 = 0.0, s1 = 0.0;
  const int t = g.t;
  CHUNK_LOOP_BEGIN(g)
  const int* nb = nbr + i * m;
  const double* bv = bval + i * m;
  const double* dbv = dbval + i * m;
  double Bx = X[i * t + c], By = Y[i * t + c], dBx = 0.0, dBy = 0.0;
  for (int k = 0; k < m; ++k) {
    const int jn = nb[k];
    if (jn < 0) break;
    const double xj = X[(int64_t)jn * t + c], yj = Y[(int64_t)jn * t + c];
    Bx += bv[k] * xj;
    By += bv[k] * yj;
    dBx += dbv[k] * xj;
    dBy += dbv[k] * yj;
  }
  const double di = 1.0 / D[i];
  const double di2 = di * di;
  s0 += -Bx * di2 * dd_s2[i] * By;
  s1 += dBx * di * By + Bx * di * dBy - Bx * di2 * dd_rho[i] * By;
  CHUNK_LOOP_END
  block_colsum(g, s0, part);
  block_colsum(g, s1, part + (int64_t)g.nchunk * t);
}

// ---------------------------------------------------------------- drivers
static int padded_rank(int k) { return (k + 15) / 16 * 16; }

Status lrac_build(Model& M, int k) {
  if (k < 1) return Status::invalid("lrac_rank must be positive");
  if (k > M.n) k = static_cast<int>(M.n);
  if (M.lrac_ready && M.lrac_k == k) return Status::ok();
  const int K = padded_rank(k);
  const int64_t n = M.n;
  VL_TRY(M.lrac_L.reserve(static_cast<size_t>(n) * K));
  VL_TRY(M.lrac_piv.reserve(k + 1));
  VL_TRY(M.lrac_pval.reserve(k + 1));
  VL_TRY(M.vec_c.reserve(n));  // residual diagonal
  const int nb = 512;
  VL_TRY(M.lrac_part.reserve(static_cast<size_t>(nb) * 2));
  double* part_v = M.lrac_part.p;
  int* part_i = reinterpret_cast<int*>(M.lrac_part.p + nb);
  hipLaunchKernelGGL(pc_init_kernel, dim3(blocks_for(n)), dim3(256), 0, M.stream, n, K,
                     M.sigma2, M.vec_c.p, M.lrac_L.p, M.lrac_piv.p, M.lrac_pval.p);
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL(pc_column_kernel, dim3(nb), dim3(256), 0, M.stream, n, K, j, M.coords,
                       M.cov, M.sigma2, M.rho, M.lrac_piv.p, M.lrac_pval.p, M.vec_c.p,
                       M.lrac_L.p, part_v, part_i, M.status);
    hipLaunchKernelGGL(pc_argmax_kernel, dim3(1), dim3(256), 0, M.stream, nb, part_v, part_i,
                       j, M.vec_c.p, M.lrac_piv.p, M.lrac_pval.p);
  }
  VL_TRY(check_launch("pivoted cholesky"));
  VL_TRY(sync_stream(M.stream));
  VL_TRY(read_status(M));
  M.lrac_k = k;
  M.lrac_K = K;
  M.lrac_ready = true;
  M.lrac_dL_ready = false;
  return Status::ok();
}

static Status gram_with(Model& M, const double* Lm, const double* w, const double* X, int ldx,
                        int t, int ldp, double* out);

// Parts of the K x ldp gram products: one block per 256 CUs' worth of rows.
static Status gram(Model& M, const double* w, const double* X, int ldx, int t, int ldp,
                   double* out) {
  return gram_with(M, M.lrac_L.p, w, X, ldx, t, ldp, out);
}

// The same with another n x K left factor (the derivative of L).
static Status gram_with(Model& M, const double* Lm, const double* w, const double* X, int ldx,
                        int t, int ldp, double* out) {
  const int K = M.lrac_K;
  const int64_t n = M.n;
  int nblk = 512;
  int64_t rpb = (n + nblk - 1) / nblk;
  rpb = (rpb + 3) / 4 * 4;
  nblk = static_cast<int>((n + rpb - 1) / rpb);
  const int64_t size = static_cast<int64_t>(K) * ldp;
  VL_TRY(M.lrac_gpart.reserve(static_cast<size_t>(nblk) * size));
  hipLaunchKernelGGL(gram_kernel, dim3(nblk), dim3(256), 0, M.stream, n, K, rpb, Lm, w, X,
                     ldx, t, ldp, M.lrac_gpart.p);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((size + 63) / 64)), dim3(256), 0,
                     M.stream, nblk, size, M.lrac_gpart.p, out);
  return check_launch("gram");
}

// M = I + L^T W L, its Cholesky factor (in lrac_M) and log det M (device).
Status lrac_factor(Model& M, const double* W) {
  const int K = M.lrac_K;
  VL_TRY(M.lrac_M.reserve(static_cast<size_t>(K) * K + 8));
  VL_TRY(gram(M, W, M.lrac_L.p, K, K, K, M.lrac_M.p));
  hipLaunchKernelGGL(add_identity_kernel, dim3(1), dim3(K), 0, M.stream, K, M.lrac_M.p);
  hipLaunchKernelGGL(small_cholesky_kernel, dim3(1), dim3(256), sizeof(double) * K * K,
                     M.stream, K, M.lrac_M.p, M.lrac_M.p + K * K, M.status);
  VL_TRY(M.lrac_Minv.reserve(static_cast<size_t>(K) * K));
  hipLaunchKernelGGL(chol_inverse_kernel, dim3((K + 63) / 64), dim3(64), 0, M.stream, K,
                     M.lrac_M.p, M.lrac_Minv.p);
  return check_launch("lrac factor");
}

// Z = P_LRAC^{-1} R over t columns.
static Status lrac_precond(Model& M, const double* W, const double* R, double* Z, int t) {
  const int K = M.lrac_K;
  const int ldp = (t + 15) / 16 * 16;
  VL_TRY(M.lrac_S.reserve(static_cast<size_t>(K) * ldp));
  VL_TRY(M.lrac_S2.reserve(static_cast<size_t>(K) * ldp));
  VL_TRY(gram(M, W, R, t, t, ldp, M.lrac_S.p));
  // M^{-1} (L^T W R) with the explicit inverse (K x K, once per factor)
  hipLaunchKernelGGL(small_gemm_kernel, dim3(blocks_for((int64_t)K * ldp)), dim3(256), 0,
                     M.stream, K, t, ldp, M.lrac_Minv.p, M.lrac_S.p, M.lrac_S2.p);
  const int64_t tiles = ((M.n + 15) / 16) * ((t + 15) / 16);
  hipLaunchKernelGGL(panel_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, M.stream,
                     M.n, K, M.lrac_L.p, M.lrac_S2.p, ldp, t, 0, W, R, 0ull, Z);
  return check_launch("lrac precond");
}

// V = Sigma~ H + H / W, Sigma~ H = B^{-1} (D o (B^{-T} H)).
static Status sigma_apply(Model& M, const double* H, double* V, double* Tmp, int t,
                          const double* W) {
  VL_TRY(trsm_bt_slot(M, H, Tmp, t, false, 0));
  VL_TRY(trsm_b_slot(M, Tmp, V, t, M.dval.p, false, 1));
  if (W) {
    hipLaunchKernelGGL(add_div_kernel, dim3(blocks_for(M.n * t)), dim3(256), 0, M.stream, M.n, t,
                       H, W, V);
    VL_TRY(check_launch("add div"));
  }
  return Status::ok();
}

CgOps lrac_ops(const double* W) {
  CgOps ops;
  ops.apply = [W](Model& M, const double* H, double* V, double* Tmp, int t) -> Status {
    return sigma_apply(M, H, V, Tmp, t, W);
  };
  ops.precond = [W](Model& M, const double* R, double* Z, double* Y, int t) -> Status {
    (void)Y;
    return lrac_precond(M, W, R, Z, t);
  };
  ops.needs_fill = [](const Model&, int) { return false; };
  return ops;
}

// One Newton step of eq. (pcls2): (Sigma~ + W^{-1}) (W b') = Sigma~ rhs.
Status lrac_newton_solve(Model& M, const vl_opts& o, const double* rhs, double* b_out,
                         const int* forced) {
  const int64_t n = M.n;
  VL_TRY(M.vec_d.reserve(n));
  VL_TRY(M.vec_e.reserve(n));
  VL_TRY(lrac_factor(M, M.W.p));
  VL_TRY(sigma_apply(M, rhs, M.vec_d.p, M.vec_e.p, 1, nullptr));
  CgOps ops = lrac_ops(M.W.p);
  VL_TRY(cg_solve(M, M.cg1, ops, 1, M.vec_d.p, o.cg_tol, o.max_cg, false, forced));
  hipLaunchKernelGGL(div_kernel, dim3(blocks_for(n)), dim3(256), 0, M.stream, n, M.cg1.U.p,
                     M.W.p, b_out);
  return check_launch("lrac newton");
}

Status lrac_build_deriv(Model& M) {
  if (!M.lrac_ready) return Status::make(VL_ERR_STATE, "no LRAC factor");
  if (M.lrac_dL_ready) return Status::ok();
  const int64_t n = M.n;
  const int K = M.lrac_K, k = M.lrac_k;
  VL_TRY(M.lrac_dL.reserve(static_cast<size_t>(2) * n * K));
  VL_TRY(M.lrac_dd.reserve(static_cast<size_t>(2) * n));
  VL_TRY(M.lrac_snap.reserve(static_cast<size_t>(2) * k + 2));
  double* dL0 = M.lrac_dL.p;
  double* dL1 = M.lrac_dL.p + static_cast<size_t>(n) * K;
  double* dd0 = M.lrac_dd.p;
  double* dd1 = M.lrac_dd.p + n;
  hipLaunchKernelGGL(pc_deriv_init_kernel, dim3(std::min<int64_t>(blocks_for(n * K), 8192)),
                     dim3(256), 0, M.stream, n, K, dL0, dL1, dd0, dd1);
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL(pc_deriv_snap_kernel, dim3(1), dim3(64), 0, M.stream, j, M.lrac_piv.p,
                       dd0, dd1, M.lrac_snap.p);
    hipLaunchKernelGGL(pc_deriv_column_kernel, dim3(512), dim3(256), 0, M.stream, n, K, j,
                       M.coords, M.cov, M.sigma2, M.rho, M.lrac_piv.p, M.lrac_pval.p,
                       M.lrac_L.p, dL0, dL1, dd0, dd1, M.lrac_snap.p);
  }
  VL_TRY(check_launch("pivoted cholesky derivative"));
  M.lrac_dL_ready = true;
  return Status::ok();
}

Status lrac_leverage(Model& M, double* lev) {
  if (M.lrac_K > 128) return Status::invalid("the LRAC gradient supports k <= 128");
  hipLaunchKernelGGL(lrac_leverage_kernel, dim3(blocks_for(M.n)), dim3(256), 0, M.stream, M.n,
                     M.lrac_K, M.lrac_L.p, M.lrac_M.p, lev);
  return check_launch("lrac leverage");
}

Status lrac_sigma(Model& M, const double* X, double* Y, double* Tmp, int t) {
  return sigma_apply(M, X, Y, Tmp, t, nullptr);
}

Status lrac_theta_terms(Model& M, const double* SU, const double* SV, const double* V,
                        const double* W, int t, double* h, double* r, double* trP) {
  const int64_t n = M.n;
  const int K = M.lrac_K;
  // h_k = -(Sigma~ u)^T (d Sigma~^{-1} / d theta_k) (Sigma~ v), per column
  ChunkGrid g = ChunkGrid::of(n, t);
  VL_TRY(M.red_part.reserve(static_cast<size_t>(g.nchunk) * t * 2 + 64));
  hipLaunchKernelGGL(dprec_form_kernel, dim3(g.nchunk, g.L.slices), dim3(256), 0, M.stream, g,
                     M.m, M.nbr.p, M.bval.p, M.dbval_rho.p, SU, SV, M.dval.p, M.dd_sigma2.p,
                     M.dd_rho.p, M.red_part.p);
  VL_TRY(check_launch("lrac h"));
  VL_TRY(M.red_out.reserve(2 * static_cast<size_t>(t) + 64));
  for (int q = 0; q < 2; ++q)
    VL_TRY(reduce_chunks(M.stream, M.red_part.p + (int64_t)q * g.nchunk * t, g.nchunk, t,
                         M.red_out.p + q * t));
  std::vector<double> hv(2 * t);
  VL_HIP(hipMemcpyAsync(hv.data(), M.red_out.p, sizeof(double) * 2 * t, hipMemcpyDeviceToHost,
                        M.stream));
  // r_k = 2 (L^T v) . (dL_k^T v) per column; tr(M^{-1} (dL^T W L + L^T W dL)) =
  // 2 tr(M^{-1} L^T W dL)
  const int ldp = (t + 15) / 16 * 16;
  DevBuf<double> lv, dlv, gw;
  VL_TRY(lv.alloc(static_cast<size_t>(K) * ldp));
  VL_TRY(dlv.alloc(static_cast<size_t>(2) * K * ldp));
  VL_TRY(gw.alloc(static_cast<size_t>(2) * K * K));
  VL_TRY(gram(M, nullptr, V, t, t, ldp, lv.p));
  for (int q = 0; q < 2; ++q) {
    const double* dLq = M.lrac_dL.p + static_cast<size_t>(q) * n * K;
    VL_TRY(gram_with(M, dLq, nullptr, V, t, t, ldp, dlv.p + static_cast<size_t>(q) * K * ldp));
    VL_TRY(gram(M, W, dLq, K, K, K, gw.p + static_cast<size_t>(q) * K * K));  // L^T W dL_q
  }
  std::vector<double> lvh(static_cast<size_t>(K) * ldp), dlvh(static_cast<size_t>(2) * K * ldp),
      gwh(static_cast<size_t>(2) * K * K), Ch(static_cast<size_t>(K) * K);
  VL_HIP(hipMemcpyAsync(lvh.data(), lv.p, sizeof(double) * lvh.size(), hipMemcpyDeviceToHost,
                        M.stream));
  VL_HIP(hipMemcpyAsync(dlvh.data(), dlv.p, sizeof(double) * dlvh.size(), hipMemcpyDeviceToHost,
                        M.stream));
  VL_HIP(hipMemcpyAsync(gwh.data(), gw.p, sizeof(double) * gwh.size(), hipMemcpyDeviceToHost,
                        M.stream));
  VL_HIP(hipMemcpyAsync(Ch.data(), M.lrac_M.p, sizeof(double) * Ch.size(), hipMemcpyDeviceToHost,
                        M.stream));
  VL_TRY(sync_stream(M.stream));
  for (int q = 0; q < 2; ++q) {
    for (int c = 0; c < t; ++c) {
      h[q * t + c] = -hv[q * t + c];
      double acc = 0.0;
      for (int a = 0; a < K; ++a)
        acc += lvh[static_cast<size_t>(a) * ldp + c] *
               dlvh[static_cast<size_t>(q) * K * ldp + static_cast<size_t>(a) * ldp + c];
      r[q * t + c] = 2.0 * acc;
    }
    // tr(M^{-1} G), G = L^T W dL_q: column b of M^{-1} G by two triangular
    // solves with the Cholesky factor C (M = C C^T), summing the diagonal
    double tr = 0.0;
    std::vector<double> y(K);
    const double* G = gwh.data() + static_cast<size_t>(q) * K * K;
    for (int b = 0; b < K; ++b) {
      for (int a = 0; a < K; ++a) {
        double v = G[static_cast<size_t>(a) * K + b];
        for (int l = 0; l < a; ++l) v -= Ch[static_cast<size_t>(a) * K + l] * y[l];
        y[a] = v / Ch[static_cast<size_t>(a) * K + a];
      }
      for (int a = K - 1; a >= 0; --a) {
        double v = y[a];
        for (int l = a + 1; l < K; ++l) v -= Ch[static_cast<size_t>(l) * K + a] * y[l];
        y[a] = v / Ch[static_cast<size_t>(a) * K + a];
      }
      tr += y[b];
    }
    trP[q] = 2.0 * tr;
  }
  return Status::ok();
}

// SLQ with P_LRAC: probes z = L eps_k + W^{-1/2} eps_n, CG on Sigma~ + W^{-1};
// returns log det M (= sum log W + log det P) on the host.
Status lrac_slq(Model& M, const vl_opts& o, double* logdet_fixed, const int* forced,
                bool keep_z0) {
  const int64_t n = M.n;
  const int t = o.num_probes;
  const int K = M.lrac_K;
  VL_TRY(lrac_factor(M, M.W.p));
  const int ldp = (t + 15) / 16 * 16;
  VL_TRY(M.lrac_S.reserve(static_cast<size_t>(K) * ldp));
  hipLaunchKernelGGL(lrac_probe_k_kernel, dim3(blocks_for((int64_t)K * ldp)), dim3(256), 0,
                     M.stream, K, M.lrac_k, t, ldp, o.seed, M.lrac_S.p);
  VL_TRY(M.rhs_blk.reserve(static_cast<size_t>(n) * t));
  const int64_t tiles = ((n + 15) / 16) * ((t + 15) / 16);
  hipLaunchKernelGGL(panel_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, M.stream, n,
                     K, M.lrac_L.p, M.lrac_S.p, ldp, t, 1, M.W.p, nullptr, o.seed,
                     M.rhs_blk.p);
  VL_TRY(check_launch("lrac probes"));
  double ld = 0.0;
  VL_HIP(hipMemcpyAsync(&ld, M.lrac_M.p + K * K, sizeof(double), hipMemcpyDeviceToHost,
                        M.stream));
  CgOps ops = lrac_ops(M.W.p);
  VL_TRY(cg_solve(M, M.cg, ops, t, M.rhs_blk.p, o.cg_tol, o.max_cg, keep_z0, forced));
  *logdet_fixed = ld;
  return Status::ok();
}

}  // namespace vl
