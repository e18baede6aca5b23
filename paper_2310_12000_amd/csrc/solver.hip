// Block preconditioned CG with Lanczos coefficients (appendix algorithm
// "Preconditioned conjugate gradient algorithm with Lanczos tridiagonal
// matrix"), run independently on each of t columns, for the systems
//   (W + B^T D^{-1} B) u = rhs       preconditioned with
//   P_VADU = B^T (W + D^{-1}) B      (eqs. pcls1, P_VADU; Sec. 3.1.1),
// plus the tridiagonal quadrature e_1^T log(T~) e_1 of eq. (def_SLQ) and the
// likelihood terms of eq. (VLA_loss).
//
// Column reductions are deterministic: a fixed grid of row chunks writes one
// partial sum per (chunk, column), and a single block adds the partials of
// each column in chunk order.
#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

// ------------------------------------------------------------ chunk layout
ChunkGrid ChunkGrid::of(int64_t n, int t) {
  ChunkGrid g;
  g.L = Lanes::of(t);
  g.n = n;
  g.t = t;
  const int64_t step = 4LL << g.L.rpw_log;
  int64_t groups = (n + step - 1) / step;
  int64_t want = 2048 / g.L.slices;
  if (want < 1) want = 1;
  if (want > groups) want = groups;
  if (want < 1) want = 1;
  int64_t per = (groups + want - 1) / want;
  g.rpc = per * step;
  g.nchunk = static_cast<int>((n + g.rpc - 1) / g.rpc);
  if (g.nchunk < 1) g.nchunk = 1;
  return g;
}

// Sum of column c's per-chunk partials by one wave: lane k takes chunks
// k, k + 64, ... in order, then a fixed butterfly adds the lanes, so the
// result does not depend on timing.  Every lane returns the sum.
__device__ __forceinline__ double wave_colsum(const double* __restrict__ part, int nchunk, int t,
                                              int c) {
  double s = 0.0;
  for (int k = threadIdx.x & 63; k < nchunk; k += 64) s += part[(int64_t)k * t + c];
  return wave_sum(s);
}

// One wave per column, four columns per block.
static unsigned col_blocks(int t) { return static_cast<unsigned>((t + 3) / 4); }
__device__ __forceinline__ int wave_col() { return blockIdx.x * 4 + (threadIdx.x >> 6); }

__global__ __launch_bounds__(256) void reduce_chunks_kernel(const double* __restrict__ part,
                                                            int nchunk, int t,
                                                            double* __restrict__ out) {
  const int c = wave_col();
  if (c >= t) return;
  const double s = wave_colsum(part, nchunk, t, c);
  if ((threadIdx.x & 63) == 0) out[c] = s;
}

Status reduce_chunks(hipStream_t s, const double* part, int nchunk, int t, double* out) {
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3(col_blocks(t)), dim3(256), 0, s, part, nchunk,
                     t, out);
  return check_launch("reduce_chunks");
}

// ---------------------------------------------------------- CG kernels
// The vector kernels are templated on the storage type T of the n x t blocks
// (double; float in the mixed-precision form); every sum is accumulated in
// double.  Y and Z (the preconditioner's outputs) are pre-filled with the
// sentinel of the sync-free solves when given.


template <typename T>
__global__ __launch_bounds__(256) void cg_init_kernel(ChunkGrid g, const T* __restrict__ rhs,
                                                      T* __restrict__ U, T* __restrict__ R,
                                                      T* __restrict__ Y, T* __restrict__ Z,
                                                      int* counter) {
  CHUNK_LOOP_BEGIN(g)
  const int64_t o = i * g.t + c;
  U[o] = T(0);
  R[o] = rhs[o];
  if (Y) {
    Y[o] = sentinel_of<T>();
    Z[o] = sentinel_of<T>();
  }
  CHUNK_LOOP_END
  if (counter && blockIdx.x == 0 && blockIdx.y == 0) reset_counters(counter);
}

// H = Z (and Z0 = Z); partial sums of r.z
template <typename T>
__global__ __launch_bounds__(256) void cg_init2_kernel(ChunkGrid g, const T* __restrict__ R,
                                                       const T* __restrict__ Z,
                                                       T* __restrict__ H, T* __restrict__ Z0,
                                                       double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  const int64_t o = i * g.t + c;
  const T z = Z[o];
  H[o] = z;
  if (Z0) Z0[o] = z;
  acc += static_cast<double>(R[o]) * static_cast<double>(z);
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

template <typename T>
__global__ __launch_bounds__(256) void dot_kernel(ChunkGrid g, const T* __restrict__ X,
                                                  const T* __restrict__ Y,
                                                  double* __restrict__ part) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  const int64_t o = i * g.t + c;
  acc += static_cast<double>(X[o]) * static_cast<double>(Y[o]);
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
}

// rz = r0z0 = sum of partials, active = 1, iters = 0 (one wave per column)
// forced (optional, t entries): fixed iteration counts replacing the
// tolerance test where >= 0 (replay of another run's counts).
__global__ __launch_bounds__(256) void cg_start_kernel(int t, int nchunk,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ rz,
                                                       double* __restrict__ r0z0,
                                                       int* __restrict__ active,
                                                       int* __restrict__ iters,
                                                       int* __restrict__ num_active,
                                                       const int* __restrict__ forced) {
  if (blockIdx.x == 0 && threadIdx.x == 0) num_active[0] = t;
  const int c = wave_col();
  if (c >= t) return;
  const double s = wave_colsum(part, nchunk, t, c);
  if ((threadIdx.x & 63) != 0) return;
  rz[c] = s;
  r0z0[c] = s;
  const int f = forced ? forced[c] : -1;
  // a zero right-hand side is already solved; a replayed count of 0 as well
  active[c] = (f >= 0) ? (f > 0 ? 1 : 0) : ((s > 0.0) ? 1 : 0);
  iters[c] = 0;
}

// alpha = r.z / h.v for active columns; records alpha_{l+1} (one wave per
// column).  Also clears the active-column count that cg_beta_kernel adds to.
__global__ __launch_bounds__(256) void cg_alpha_kernel(int t, int nchunk,
                                                       const double* __restrict__ part,
                                                       const double* __restrict__ rz,
                                                       double* __restrict__ alpha,
                                                       const int* __restrict__ active,
                                                       const int* __restrict__ iters,
                                                       double* __restrict__ hist_a,
                                                       int* __restrict__ num_active,
                                                       int* __restrict__ status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) num_active[0] = 0;
  const int c = wave_col();
  if (c >= t) return;
  const double hv = wave_colsum(part, nchunk, t, c);
  if ((threadIdx.x & 63) != 0) return;
  double a = 0.0;
  if (active[c]) {
    if (!(hv > 0.0) || !isfinite(hv)) {
      raise_error(status, kErrNonfinite);
    } else {
      a = rz[c] / hv;
      hist_a[(int64_t)iters[c] * t + c] = a;
    }
  }
  alpha[c] = a;
}

// u += alpha h, r -= alpha v; partial ||r||^2; pre-fill solve outputs
template <typename T>
__global__ __launch_bounds__(256) void cg_update_ur_kernel(
    ChunkGrid g, const double* __restrict__ alpha, const int* __restrict__ active,
    const T* __restrict__ H, const T* __restrict__ V, T* __restrict__ U, T* __restrict__ R,
    T* __restrict__ Y, T* __restrict__ Z, double* __restrict__ part, int* counter) {
  double acc = 0.0;
  CHUNK_LOOP_BEGIN(g)
  const int64_t o = i * g.t + c;
  T r = R[o];
  if (active[c]) {
    const T a = static_cast<T>(alpha[c]);
    U[o] += a * H[o];
    r -= a * V[o];
    R[o] = r;
  }
  acc += static_cast<double>(r) * static_cast<double>(r);
  if (Y) {
    Y[o] = sentinel_of<T>();
    Z[o] = sentinel_of<T>();
  }
  CHUNK_LOOP_END
  block_colsum(g, acc, part);
  if (counter && blockIdx.x == 0 && blockIdx.y == 0) reset_counters(counter);
}

// beta = r_new.z_new / r.z; records beta; stopping test on ||r||_2 (one
// wave per column); columns still active are counted into num_active.
__global__ __launch_bounds__(256) void cg_beta_kernel(int t, int nchunk,
                                                      const double* __restrict__ part_rz,
                                                      const double* __restrict__ part_rr,
                                                      double tol, int max_iter,
                                                      double* __restrict__ rz,
                                                      double* __restrict__ beta,
                                                      int* __restrict__ active,
                                                      int* __restrict__ iters,
                                                      double* __restrict__ hist_b,
                                                      int* __restrict__ num_active,
                                                      int* __restrict__ status,
                                                      const int* __restrict__ forced) {
  const int c = wave_col();
  if (c >= t) return;
  const bool act = active[c] != 0;
  double rzn = 0.0, rr = 0.0;
  if (act) {
    rzn = wave_colsum(part_rz, nchunk, t, c);
    rr = wave_colsum(part_rr, nchunk, t, c);
  }
  if ((threadIdx.x & 63) != 0) return;
  double b = 0.0;
  if (act) {
    const int it = iters[c];
    b = rzn / rz[c];
    hist_b[(int64_t)it * t + c] = b;
    rz[c] = rzn;
    iters[c] = it + 1;
    if (!isfinite(rr) || !isfinite(b)) raise_error(status, kErrNonfinite);
    const int f = forced ? forced[c] : -1;
    const bool done = (f >= 0) ? (it + 1 >= f) : (sqrt(rr) < tol);
    if (done || it + 1 >= max_iter || !isfinite(rr)) {
      active[c] = 0;
    } else {
      atomicAdd(num_active, 1);
    }
  }
  beta[c] = b;
}

template <typename T>
__global__ __launch_bounds__(256) void cg_update_h_kernel(ChunkGrid g,
                                                          const double* __restrict__ beta,
                                                          const int* __restrict__ active,
                                                          const T* __restrict__ Z,
                                                          T* __restrict__ H) {
  CHUNK_LOOP_BEGIN(g)
  if (active[c]) {
    const int64_t o = i * g.t + c;
    H[o] = Z[o] + static_cast<T>(beta[c]) * H[o];
  }
  CHUNK_LOOP_END
}

// ------------------------------------------------------------ CG driver
static Status cg_reserve(Model& M, CgState& S, int t, int lmax, bool keep_z0) {
  const size_t nt = static_cast<size_t>(M.n) * t;
  VL_TRY(S.U.reserve(nt));
  VL_TRY(S.R.reserve(nt));
  VL_TRY(S.Z.reserve(nt));
  VL_TRY(S.H.reserve(nt));
  VL_TRY(S.V.reserve(nt));
  VL_TRY(S.Tmp.reserve(nt));
  VL_TRY(S.Y.reserve(nt));
  if (keep_z0) VL_TRY(S.Z0.reserve(nt));
  VL_TRY(S.rz.reserve(t));
  VL_TRY(S.rr.reserve(t));
  VL_TRY(S.alpha.reserve(t));
  VL_TRY(S.beta.reserve(t));
  VL_TRY(S.r0z0.reserve(t));
  VL_TRY(S.active.reserve(t));
  VL_TRY(S.iters.reserve(t));
  VL_TRY(S.num_active.reserve(4));
  VL_TRY(S.hist_a.reserve(static_cast<size_t>(lmax) * t));
  VL_TRY(S.hist_b.reserve(static_cast<size_t>(lmax) * t));
  ChunkGrid g = ChunkGrid::of(M.n, t);
  VL_TRY(S.part_a.reserve(static_cast<size_t>(g.nchunk) * t));
  VL_TRY(S.part_b.reserve(static_cast<size_t>(g.nchunk) * t));
  VL_TRY(M.counter.reserve(2 * kSlotInts + 64));
  if (!M.host_pin) VL_HIP(hipHostMalloc(reinterpret_cast<void**>(&M.host_pin), 64 * sizeof(double)));
  S.t = t;
  S.lmax = lmax;
  return Status::ok();
}

static dim3 chunk_dims(const ChunkGrid& g) { return dim3(g.nchunk, g.L.slices); }

// Storage of the n x t blocks of S as T (a block of n t doubles holds n t
// floats).
template <typename T>
static T* blk(DevBuf<double>& b) {
  return reinterpret_cast<T*>(b.p);
}

template <typename T, class Ops>
static Status cg_run(Model& M, CgState& S, const Ops& ops, int t, const T* rhs, double tol,
                     int max_iter, bool keep_z0, bool sentinel_fill, const int* forced_host) {
  if (t <= 0) return Status::invalid("t must be positive");
  if (max_iter < 1) max_iter = 1;
  VL_TRY(cg_reserve(M, S, t, max_iter, keep_z0));
  hipStream_t s = M.stream;
  const int* forced = nullptr;
  if (forced_host) {
    VL_TRY(S.forced.reserve(t));
    VL_HIP(hipMemcpyAsync(S.forced.p, forced_host, sizeof(int) * t, hipMemcpyHostToDevice, s));
    VL_TRY(sync_stream(s));  // the host array may go away after the call
    forced = S.forced.p;
  }
  ChunkGrid g = ChunkGrid::of(M.n, t);
  const dim3 cg_grid = chunk_dims(g);
  int* cnt = sentinel_fill ? M.counter.p : nullptr;
  T *U = blk<T>(S.U), *R = blk<T>(S.R), *Z = blk<T>(S.Z), *H = blk<T>(S.H), *V = blk<T>(S.V),
    *Tmp = blk<T>(S.Tmp), *Y = blk<T>(S.Y);
  T* Yf = sentinel_fill ? Y : nullptr;
  T* Zf = sentinel_fill ? Z : nullptr;
  // u_0 = 0, r_0 = rhs, z_0 = P^{-1} r_0, h_0 = z_0
  hipLaunchKernelGGL(cg_init_kernel<T>, cg_grid, dim3(256), 0, s, g, rhs, U, R, Yf, Zf, cnt);
  VL_TRY(ops.precond(M, R, Z, Y, t));
  hipLaunchKernelGGL(cg_init2_kernel<T>, cg_grid, dim3(256), 0, s, g, R, Z, H,
                     keep_z0 ? blk<T>(S.Z0) : nullptr, S.part_a.p);
  hipLaunchKernelGGL(cg_start_kernel, dim3(col_blocks(t)), dim3(256), 0, s, t, g.nchunk,
                     S.part_a.p, S.rz.p, S.r0z0.p, S.active.p, S.iters.p, S.num_active.p, forced);
  VL_TRY(check_launch("cg start"));
  for (int it = 0; it < max_iter; ++it) {
    VL_TRY(ops.apply(M, H, V, Tmp, t));
    hipLaunchKernelGGL(dot_kernel<T>, cg_grid, dim3(256), 0, s, g, H, V, S.part_a.p);
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(col_blocks(t)), dim3(256), 0, s, t, g.nchunk,
                       S.part_a.p, S.rz.p, S.alpha.p, S.active.p, S.iters.p, S.hist_a.p,
                       S.num_active.p, M.status);
    hipLaunchKernelGGL(cg_update_ur_kernel<T>, cg_grid, dim3(256), 0, s, g, S.alpha.p,
                       S.active.p, H, V, U, R, Yf, Zf, S.part_b.p, cnt);
    VL_TRY(ops.precond(M, R, Z, Y, t));
    hipLaunchKernelGGL(dot_kernel<T>, cg_grid, dim3(256), 0, s, g, R, Z, S.part_a.p);
    hipLaunchKernelGGL(cg_beta_kernel, dim3(col_blocks(t)), dim3(256), 0, s, t, g.nchunk,
                       S.part_a.p, S.part_b.p, tol, max_iter, S.rz.p, S.beta.p, S.active.p,
                       S.iters.p, S.hist_b.p, S.num_active.p, M.status, forced);
    hipLaunchKernelGGL(cg_update_h_kernel<T>, cg_grid, dim3(256), 0, s, g, S.beta.p, S.active.p,
                       Z, H);
    VL_TRY(check_launch("cg iteration"));
    VL_HIP(hipMemcpyAsync(M.host_pin, S.num_active.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VL_TRY(sync_stream(s));
    if (*reinterpret_cast<int*>(M.host_pin) == 0) break;
  }
  S.host_iters.resize(t);
  VL_HIP(hipMemcpyAsync(S.host_iters.data(), S.iters.p, sizeof(int) * t, hipMemcpyDeviceToHost,
                        s));
  VL_TRY(sync_stream(s));
  return read_status(M);
}

Status cg_solve(Model& M, CgState& S, const CgOps& ops, int t, const double* rhs, double tol,
                int max_iter, bool keep_z0, const int* forced_host) {
  const bool fill = ops.needs_fill ? ops.needs_fill(M, t) : true;
  return cg_run<double>(M, S, ops, t, rhs, tol, max_iter, keep_z0, fill, forced_host);
}

// Replayed iteration counts of columns c0..c0+t-1 of a solve (host, -1 = the
// tolerance test), or nullptr when none of them is replayed.
const int* replay_slice(const vl_opts& o, int c0, int t, std::vector<int>& buf) {
  if (!o.replay_cg_iters || o.replay_len <= c0) return nullptr;
  buf.assign(t, -1);
  for (int c = 0; c < t && c0 + c < o.replay_len; ++c) buf[c] = o.replay_cg_iters[c0 + c];
  return buf.data();
}

Status dot_cols(Model& M, const double* X, const double* Y, int t, double* part, double* out) {
  ChunkGrid g = ChunkGrid::of(M.n, t);
  hipLaunchKernelGGL(dot_kernel<double>, chunk_dims(g), dim3(256), 0, M.stream, g, X, Y, part);
  return reduce_chunks(M.stream, part, g.nchunk, t, out);
}

// ------------------------------------------------ tridiagonal quadrature
// For each column: T~ from the CG coefficients (T_11 = 1/a_1, T_jj = 1/a_j +
// b_{j-1}/a_{j-1}, T_{j-1,j} = sqrt(b_{j-1})/a_{j-1}), its eigenvalues by
// implicit QL with shifts, rotating only the first row of the eigenvector
// matrix, and sum_j z_j^2 log(lambda_j) = e_1^T log(T~) e_1.
__global__ void tridiag_logquad_kernel(int t, int lmax, const int* __restrict__ iters,
                                       const double* __restrict__ hist_a,
                                       const double* __restrict__ hist_b,
                                       double* __restrict__ work, double* __restrict__ out,
                                       int* __restrict__ status) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  const int L = iters[c];
  double* d = work + (int64_t)c * 3 * lmax;
  double* e = d + lmax;
  double* z = e + lmax;
  if (L <= 0) {
    out[c] = 0.0;
    return;
  }
  for (int j = 0; j < L; ++j) {
    const double a = hist_a[(int64_t)j * t + c];
    double dj = 1.0 / a;
    if (j > 0) {
      const double ap = hist_a[(int64_t)(j - 1) * t + c];
      const double bp = hist_b[(int64_t)(j - 1) * t + c];
      dj += bp / ap;
      e[j - 1] = sqrt(bp) / ap;
    }
    d[j] = dj;
    z[j] = (j == 0) ? 1.0 : 0.0;
  }
  e[L - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < L; ++l) {
    int sweeps = 0;
    for (;;) {
      int mm = l;
      while (mm < L - 1) {
        const double scale = fabs(d[mm]) + fabs(d[mm + 1]);
        if (fabs(e[mm]) <= eps * scale) break;
        ++mm;
      }
      if (mm == l) break;
      if (++sweeps > 64) {
        raise_error(status, kErrNonfinite);
        out[c] = __longlong_as_double(0x7FF8000000000000ll);
        return;
      }
      // shift from the leading 2 x 2 block at l
      double gq = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double rq = hypot(gq, 1.0);
      gq = d[mm] - d[l] + e[l] / (gq + copysign(rq, gq));
      double sn = 1.0, cs = 1.0, shift = 0.0;
      bool deflated = false;
      for (int i = mm - 1; i >= l; --i) {
        const double f = sn * e[i];
        const double bq = cs * e[i];
        rq = hypot(f, gq);
        e[i + 1] = rq;
        if (rq == 0.0) {
          d[i + 1] -= shift;
          e[mm] = 0.0;
          deflated = true;
          break;
        }
        sn = f / rq;
        cs = gq / rq;
        const double gg = d[i + 1] - shift;
        const double rr = (d[i] - gg) * sn + 2.0 * cs * bq;
        shift = sn * rr;
        d[i + 1] = gg + shift;
        gq = cs * rr - bq;
        const double zf = z[i + 1];
        z[i + 1] = sn * z[i] + cs * zf;
        z[i] = cs * z[i] - sn * zf;
      }
      if (deflated) continue;
      d[l] -= shift;
      e[l] = gq;
      e[mm] = 0.0;
    }
  }
  double acc = 0.0;
  for (int j = 0; j < L; ++j) {
    if (!(d[j] > 0.0)) raise_error(status, kErrNonfinite);
    acc += z[j] * z[j] * log(d[j]);
  }
  out[c] = acc;
}

Status tridiag_quadrature(Model& M, CgState& S, double* out_dev) {
  VL_TRY(S.tri.reserve(static_cast<size_t>(S.t) * 3 * S.lmax));
  const int g = (S.t + 63) / 64;
  hipLaunchKernelGGL(tridiag_logquad_kernel, dim3(g), dim3(64), 0, M.stream, S.t, S.lmax,
                     S.iters.p, S.hist_a.p, S.hist_b.p, S.tri.p, out_dev, M.status);
  return check_launch("tridiag");
}

}  // namespace vl
