// Sparse operations with the Vecchia factor B (unit lower triangular,
// B_{i,N(i)} = -A_i, Sec. 2.1) over blocks of t columns stored row-major
// (n x t, "probe-interleaved"): every neighbour gather reads t contiguous
// values, and a wave maps lanes to columns (64 / lanes_per_row rows per wave
// for t <= 64; 64-column slices for t > 64).
//
//   spmm_b   Y = rs o (X + B_off X)          B in ELL (neighbour lists)
//   spmm_bt  Y = d o v + X + B_off^T X       B^T in CSR (built once per
//                                            neighbour set by counting sort)
//   trsm_b   B Y = rs o X    (forward, rows in index order)
//   trsm_bt  B^T Y = X       (backward, rows in reverse index order)
//
// The triangular solves are sync-free: the output is pre-filled with a
// sentinel NaN, waves take work units from a global counter in topological
// order, and a row waits (bounded spin) until each needed value differs from
// the sentinel.  Values are published with device-coherent relaxed stores, so
// no grid-wide barrier is needed per level of the dependency DAG.  Each row
// sums its terms in a fixed order, so results do not depend on timing.
#include <algorithm>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

static int64_t units_of(int64_t n, int t) { return units_of_hd(n, t, Lanes::of(t)); }

int spmm_nblocks(int64_t n, int t) {
  return static_cast<int>((units_of(n, t) + 3) / 4);
}

// ------------------------------------------------------- input functors
struct InMem {
  const double* X;
  int t;
  __device__ __forceinline__ double operator()(int64_t i, int c) const { return X[i * t + c]; }
};
// The same for an FP32 block (mixed-precision solves), widened on read.
struct InMemF {
  const float* X;
  int t;
  __device__ __forceinline__ double operator()(int64_t i, int c) const {
    return static_cast<double>(X[i * t + c]);
  }
};
// s_i * (Rademacher or Gaussian probe (seed, tag, col0 + c, i))
struct InProbe {
  const double* s;
  uint64_t seed;
  uint32_t tag;
  int col0;
  int gauss;
  __device__ __forceinline__ double operator()(int64_t i, int c) const {
    double e = gauss ? gaussian(seed, tag, (uint64_t)(col0 + c), (uint64_t)i)
                     : rademacher(seed, tag, (uint64_t)(col0 + c), (uint64_t)i);
    return s ? s[i] * e : e;
  }
};

// ------------------------------------------------------------- transpose
__global__ void bt_count(const int* __restrict__ nbr, int64_t n, int m, int* __restrict__ cnt) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  int j = nbr[e];
  if (j >= 0) atomicAdd(&cnt[j], 1);
}

__global__ void bt_fill(const int* __restrict__ nbr, int64_t n, int m,
                        const int* __restrict__ ptr, int* __restrict__ cursor,
                        int* __restrict__ col, int* __restrict__ src) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  int j = nbr[e];
  if (j < 0) return;
  int pos = ptr[j] + atomicAdd(&cursor[j], 1);
  col[pos] = static_cast<int>(e / m);
  src[pos] = static_cast<int>(e);
}

// sort each row of B^T by column (= row index of B), carrying the source slot
__global__ void bt_sort_rows(int64_t n, const int* __restrict__ ptr, int* __restrict__ col,
                             int* __restrict__ src) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  int b = ptr[j], e = ptr[j + 1];
  for (int p = b + 1; p < e; ++p) {
    int c = col[p], s = src[p];
    int q = p - 1;
    while (q >= b && col[q] > c) {
      col[q + 1] = col[q];
      src[q + 1] = src[q];
      --q;
    }
    col[q + 1] = c;
    src[q + 1] = s;
  }
}

__global__ void bt_gather_vals(int64_t nnz, const int* __restrict__ src,
                               const double* __restrict__ bval, double* __restrict__ out) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nnz) out[e] = bval[src[e]];
}

Status build_transpose(Model& M) {
  const int64_t n = M.n;
  const int m = M.m;
  hipStream_t s = M.stream;
  VL_TRY(M.bt_ptr.alloc(n + 1));
  DevBuf<int> cnt;
  VL_TRY(cnt.alloc(n + 1));
  VL_TRY(fill_int(cnt.p, 0, n + 1, s));
  const int tb = 256;
  const int64_t nm = n * m;
  if (nm > 0) {
    hipLaunchKernelGGL(bt_count, dim3((unsigned)((nm + tb - 1) / tb)), dim3(tb), 0, s,
                       M.nbr.p, n, m, cnt.p);
  }
  VL_TRY(exclusive_scan_int(cnt.p, M.bt_ptr.p, n + 1, s));
  int nnz_i = 0;
  VL_HIP(hipMemcpyAsync(&nnz_i, M.bt_ptr.p + n, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  M.nnz = nnz_i;
  VL_TRY(M.bt_col.alloc(M.nnz));
  VL_TRY(M.bt_src.alloc(M.nnz));
  VL_TRY(M.bt_val.alloc(M.nnz));
  VL_TRY(fill_int(cnt.p, 0, n + 1, s));
  if (nm > 0) {
    hipLaunchKernelGGL(bt_fill, dim3((unsigned)((nm + tb - 1) / tb)), dim3(tb), 0, s, M.nbr.p,
                       n, m, M.bt_ptr.p, cnt.p, M.bt_col.p, M.bt_src.p);
  }
  hipLaunchKernelGGL(bt_sort_rows, dim3((unsigned)((n + tb - 1) / tb)), dim3(tb), 0, s, n,
                     M.bt_ptr.p, M.bt_col.p, M.bt_src.p);
  VL_TRY(check_launch("transpose"));
  VL_TRY(sync_stream(s));
  return Status::ok();
}

Status transpose_pattern(Model& M, const int* nbr, int64_t rows, int m, int64_t cols,
                         DevBuf<int>& ptr, DevBuf<int>& col, DevBuf<int>& src, int* nnz_out) {
  hipStream_t s = M.stream;
  VL_TRY(ptr.reserve(cols + 1));
  DevBuf<int> cnt;
  VL_TRY(cnt.alloc(cols + 1));
  VL_TRY(fill_int(cnt.p, 0, cols + 1, s));
  const int tb = 256;
  const int64_t nm = rows * m;
  if (nm > 0)
    hipLaunchKernelGGL(bt_count, dim3((unsigned)((nm + tb - 1) / tb)), dim3(tb), 0, s, nbr,
                       rows, m, cnt.p);
  VL_TRY(exclusive_scan_int(cnt.p, ptr.p, cols + 1, s));
  int nnz = 0;
  VL_HIP(hipMemcpyAsync(&nnz, ptr.p + cols, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  VL_TRY(col.reserve(nnz > 0 ? nnz : 1));
  VL_TRY(src.reserve(nnz > 0 ? nnz : 1));
  VL_TRY(fill_int(cnt.p, 0, cols + 1, s));
  if (nm > 0)
    hipLaunchKernelGGL(bt_fill, dim3((unsigned)((nm + tb - 1) / tb)), dim3(tb), 0, s, nbr, rows,
                       m, ptr.p, cnt.p, col.p, src.p);
  hipLaunchKernelGGL(bt_sort_rows, dim3((unsigned)((cols + tb - 1) / tb)), dim3(tb), 0, s, cols,
                     ptr.p, col.p, src.p);
  VL_TRY(check_launch("transpose pattern"));
  VL_TRY(sync_stream(s));  // cnt is released on return
  *nnz_out = nnz;
  return Status::ok();
}

// Copies of the B values after a factor: B^T, and B's rows with their slots
// in the forward tail's consumption order (tail_slots_kernel).
Status refresh_transpose_values(Model& M) {
  if (M.nnz == 0) return Status::ok();
  const int tb = 256;
  hipLaunchKernelGGL(bt_gather_vals, dim3((unsigned)((M.nnz + tb - 1) / tb)), dim3(tb), 0,
                     M.stream, M.nnz, M.bt_src.p, M.bval.p, M.bt_val.p);
  const int64_t nm = M.n * static_cast<int64_t>(M.m);
  if (M.tsrc.p && nm > 0)
    hipLaunchKernelGGL(bt_gather_vals, dim3((unsigned)((nm + tb - 1) / tb)), dim3(tb), 0,
                       M.stream, nm, M.tsrc.p, M.bval.p, M.tval.p);
  return check_launch("transpose values");
}

// ------------------------------------------------------------------ SpMM
// Work unit -> (row, column).  For t > 64 units are slice-major (all rows of
// slice 0, then slice 1, ...), so one 64-column slice of the operand is the
// working set at a time.  `order` (optional) maps the unit's row position to
// a row index (spatial order for products; topological order is required
// for solves, which pass nullptr and use index order).
struct UnitPos {
  int64_t i;
  int c;
  bool valid;
};
__device__ __forceinline__ UnitPos unit_pos(int64_t unit, int lane, Lanes L, int64_t n, int t,
                                            bool reverse, const int* __restrict__ order) {
  const int64_t rgs = (n + (1 << L.rpw_log) - 1) >> L.rpw_log;
  const int64_t slice = unit / rgs;
  const int64_t rg = unit - slice * rgs;
  const int sub = lane >> L.lpr_log;
  const int c = static_cast<int>(slice) * 64 + (lane & ((1 << L.lpr_log) - 1));
  const int64_t r = (rg << L.rpw_log) + sub;
  UnitPos p;
  p.valid = (r < n) && (c < t);
  int64_t rr = reverse ? (n - 1 - r) : r;
  if (order && p.valid) rr = order[rr];
  p.i = rr;
  p.c = c;
  return p;
}

// Y_i = rs_i * (unit * X_i + sum_k vals[i,k] X_{nbr[i,k]}) over the W >= m
// neighbour slots (empty slots add zero).
template <int W, class In>
__global__ __launch_bounds__(256) void spmm_ell_kernel(int64_t n, int m, int t, Lanes L,
                                                       const int* __restrict__ order,
                                                       const int* __restrict__ nbr,
                                                       const double* __restrict__ vals, In x,
                                                       const double* __restrict__ rs,
                                                       int unit_diag, double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (unit >= units_of_hd(n, t, L)) return;
  UnitPos p = unit_pos(unit, lane, L, n, t, false, order);
  if (!p.valid) return;
  const int* nb = nbr + p.i * m;
  const double* vb = vals + p.i * m;
  double acc = unit_diag ? x(p.i, p.c) : 0.0;
  // neighbour slots in chunks of 8: a chunk's gathers are in flight together
  // and the register footprint stays small enough for full occupancy
#pragma unroll 1
  for (int k0 = 0; k0 < W && k0 < m; k0 += 8) {
    int js[8];
    double vv[8], xs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      js[k] = (k0 + k < m) ? nb[k0 + k] : -1;
      vv[k] = (k0 + k < m) ? vb[k0 + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[k] = (js[k] >= 0) ? x(js[k], p.c) : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += vv[k] * xs[k];
  }
  if (rs) acc *= rs[p.i];
  Y[p.i * t + p.c] = acc;
}

// Y_j = d_j * v_j + X_j + sum_e btval[e] X_{btcol[e]}; entries in batches of 8
template <class In, class Dv>
__global__ __launch_bounds__(256) void spmm_csr_t_kernel(
    int64_t n, int t, Lanes L, const int* __restrict__ order, const int* __restrict__ ptr,
    const int* __restrict__ col, const double* __restrict__ val, In x,
    const double* __restrict__ d, Dv v, double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (unit >= units_of_hd(n, t, L)) return;
  UnitPos p = unit_pos(unit, lane, L, n, t, false, order);
  if (!p.valid) return;
  double acc = x(p.i, p.c);
  const int b = ptr[p.i], e = ptr[p.i + 1];
  for (int q = b; q < e; q += 8) {
    int cs[8];
    double vs[8], xs[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cs[k] = (q + k < e) ? col[q + k] : -1;
      vs[k] = (q + k < e) ? val[q + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) xs[k] = (cs[k] >= 0) ? x(cs[k], p.c) : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += vs[k] * xs[k];
  }
  if (d) acc += d[p.i] * v(p.i, p.c);
  Y[p.i * t + p.c] = acc;
}

// Wide blocks (t > 64): block (r, s) computes row order[r] for the 256 VEC
// columns of slice s; the row's indices and values are uniform over the block
// (scalar loads), and each thread gathers VEC consecutive columns of every
// neighbour row at once.  The sums run in the same order as the kernels
// above (unit diagonal first, then the entries in stored order).
template <int VEC>
struct VecT;
template <>
struct VecT<1> {
  typedef double T;
};
template <>
struct VecT<2> {
  typedef double2 T;
};

template <int VEC>
__device__ __forceinline__ void vload(const double* p, double* v) {
  if (VEC == 2) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    v[0] = q.x;
    v[1] = q.y;
  } else {
    v[0] = p[0];
  }
}
template <int VEC>
__device__ __forceinline__ void vstore(double* p, const double* v) {
  if (VEC == 2) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  } else {
    p[0] = v[0];
  }
}

template <int VEC>
__global__ __launch_bounds__(256) void spmm_ell_wide_kernel(int64_t n, int m, int t,
                                                            const int* __restrict__ order,
                                                            const int* __restrict__ nbr,
                                                            const double* __restrict__ vals,
                                                            const double* __restrict__ X,
                                                            const double* __restrict__ rs,
                                                            int unit_diag, double* __restrict__ Y) {
  const int64_t r = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = order ? order[r] : r;
  const int c = (blockIdx.y * 256 + threadIdx.x) * VEC;
  if (c >= t) return;
  double acc[VEC];
  if (unit_diag) {
    vload<VEC>(X + i * t + c, acc);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
  }
  const int* nb = nbr + i * m;
  const double* vb = vals + i * m;
  for (int k0 = 0; k0 < m; k0 += 8) {
    int js[8];
    double vv[8], xs[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      js[k] = (k0 + k < m) ? nb[k0 + k] : -1;
      vv[k] = (k0 + k < m) ? vb[k0 + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (js[k] >= 0) {
        vload<VEC>(X + (int64_t)js[k] * t + c, xs[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) xs[k][v] = 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += vv[k] * xs[k][v];
  }
  if (rs) {
    const double s = rs[i];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] *= s;
  }
  vstore<VEC>(Y + i * t + c, acc);
}

template <int VEC, bool DIAG>
__global__ __launch_bounds__(256) void spmm_csr_t_wide_kernel(
    int64_t n, int t, const int* __restrict__ order, const int* __restrict__ ptr,
    const int* __restrict__ col, const double* __restrict__ val, const double* __restrict__ X,
    const double* __restrict__ d, const double* __restrict__ V, double* __restrict__ Y) {
  const int64_t r = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = order ? order[r] : r;
  const int c = (blockIdx.y * 256 + threadIdx.x) * VEC;
  if (c >= t) return;
  double acc[VEC];
  vload<VEC>(X + i * t + c, acc);
  const int b = ptr[i], e = ptr[i + 1];
  for (int q = b; q < e; q += 8) {
    int cs[8];
    double vs[8], xs[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cs[k] = (q + k < e) ? col[q + k] : -1;
      vs[k] = (q + k < e) ? val[q + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cs[k] >= 0) {
        vload<VEC>(X + (int64_t)cs[k] * t + c, xs[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) xs[k][v] = 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += vs[k] * xs[k][v];
  }
  if (DIAG) {
    double vv[VEC];
    vload<VEC>(V + i * t + c, vv);
    const double di = d[i];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += di * vv[v];
  }
  vstore<VEC>(Y + i * t + c, acc);
}

// double2 accesses need even t and 16-byte aligned blocks
static bool vec2_ok(int t, const void* a, const void* b, const void* c = nullptr) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
  return t % 2 == 0 && al(a) && al(b) && (c == nullptr || al(c));
}

static dim3 wide_grid(int64_t n, int t, int vec) {
  const int cols = 256 * vec;
  return dim3(static_cast<unsigned>(n), static_cast<unsigned>((t + cols - 1) / cols));
}

struct InNone {
  __device__ __forceinline__ double operator()(int64_t, int) const { return 0.0; }
};

static const int* spatial_order(Model& M) { return static_cast<const int*>(M.grid_pts); }

#define VL_ELL_LAUNCH(W, ...)                                                                   \
  hipLaunchKernelGGL((spmm_ell_kernel<W, InMem>), dim3(nb), dim3(256), 0, M.stream, __VA_ARGS__)

// Algorithmic bytes of one product: nonzeros (8-byte value + 4-byte index),
// the operand read once, the result written once, plus per-row vectors.
static double spmm_bytes(const Model& M, int t, bool rowscale) {
  return 12.0 * M.nnz + 16.0 * M.n * t + (rowscale ? 8.0 * M.n : 0.0);
}

static Status launch_ell(Model& M, const double* vals, const double* X, double* Y, int t,
                         const double* rowscale, int unit_diag) {
  TimedLaunch tl(M, kTimeSpmmB, spmm_bytes(M, t, rowscale != nullptr));
  if (unit_diag && vals == M.bval.p && group_spmm_ok(M, t))
    return spmm_group_b(M, X, Y, t, rowscale);
  if (t > 64) {
    const int* ord = spatial_order(M);
    if (vec2_ok(t, X, Y)) {
      hipLaunchKernelGGL(spmm_ell_wide_kernel<2>, wide_grid(M.n, t, 2), dim3(256), 0, M.stream,
                         M.n, M.m, t, ord, M.nbr.p, vals, X, rowscale, unit_diag, Y);
    } else {
      hipLaunchKernelGGL(spmm_ell_wide_kernel<1>, wide_grid(M.n, t, 1), dim3(256), 0, M.stream,
                         M.n, M.m, t, ord, M.nbr.p, vals, X, rowscale, unit_diag, Y);
    }
    return check_launch("spmm_ell wide");
  }
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  const int* ord = spatial_order(M);
  if (M.m <= 8) {
    VL_ELL_LAUNCH(8, M.n, M.m, t, L, ord, M.nbr.p, vals, InMem{X, t}, rowscale, unit_diag, Y);
  } else if (M.m <= 16) {
    VL_ELL_LAUNCH(16, M.n, M.m, t, L, ord, M.nbr.p, vals, InMem{X, t}, rowscale, unit_diag, Y);
  } else {
    VL_ELL_LAUNCH(32, M.n, M.m, t, L, ord, M.nbr.p, vals, InMem{X, t}, rowscale, unit_diag, Y);
  }
  return check_launch("spmm_ell");
}

Status spmm_b(Model& M, const double* X, double* Y, int t, const double* rowscale) {
  return launch_ell(M, M.bval.p, X, Y, t, rowscale, 1);
}

Status spmm_ell_vals(Model& M, const double* vals, const double* X, double* Y, int t,
                     const double* rowscale, bool unit_diag) {
  return launch_ell(M, vals, X, Y, t, rowscale, unit_diag ? 1 : 0);
}

Status spmm_bt(Model& M, const double* X, double* Y, int t, const double* diag,
               const double* diagvec) {
  TimedLaunch tl(M, kTimeSpmmBt,
                 spmm_bytes(M, t, false) + 4.0 * (M.n + 1) +
                     (diag ? 8.0 * M.n + 8.0 * M.n * t : 0.0));
  if (group_spmm_ok(M, t)) return spmm_group_bt(M, X, Y, t, diag, diagvec);
  if (t > 64) {
    const int* ord = spatial_order(M);
    const int vec = vec2_ok(t, X, Y, diag ? diagvec : nullptr) ? 2 : 1;
    const dim3 gw = wide_grid(M.n, t, vec);
    if (vec == 2 && diag) {
      hipLaunchKernelGGL((spmm_csr_t_wide_kernel<2, true>), gw, dim3(256), 0, M.stream, M.n, t,
                         ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, diag, diagvec, Y);
    } else if (vec == 2) {
      hipLaunchKernelGGL((spmm_csr_t_wide_kernel<2, false>), gw, dim3(256), 0, M.stream, M.n, t,
                         ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, nullptr, nullptr, Y);
    } else if (diag) {
      hipLaunchKernelGGL((spmm_csr_t_wide_kernel<1, true>), gw, dim3(256), 0, M.stream, M.n, t,
                         ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, diag, diagvec, Y);
    } else {
      hipLaunchKernelGGL((spmm_csr_t_wide_kernel<1, false>), gw, dim3(256), 0, M.stream, M.n, t,
                         ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, nullptr, nullptr, Y);
    }
    return check_launch("spmm_bt wide");
  }
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  const int* ord = spatial_order(M);
  if (diag) {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InMem, InMem>), dim3(nb), dim3(256), 0, M.stream, M.n,
                       t, L, ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, InMem{X, t}, diag,
                       InMem{diagvec, t}, Y);
  } else {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InMem, InNone>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, InMem{X, t}, nullptr,
                       InNone{}, Y);
  }
  return check_launch("spmm_bt");
}

// out[i, c] = p(i, c) for an n x t block (probe values written once).
__global__ void probe_fill_kernel(int64_t n, int t, InProbe p, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * t;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = p(e / t, static_cast<int>(e % t));
}

Status probe_fill(Model& M, double* Y, int t, const double* s, uint64_t seed, uint32_t tag,
                  int col0) {
  const int64_t nt = M.n * static_cast<int64_t>(t);
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((nt + 255) / 256, 8192));
  hipLaunchKernelGGL(probe_fill_kernel, dim3(g), dim3(256), 0, M.stream, M.n, t,
                     InProbe{s, seed, tag, col0, 0}, Y);
  return check_launch("probe fill");
}

// Y = d o probe1 + B^T (s o probe2).  Narrow blocks generate the probes in
// place; wider ones (tmp1, tmp2: n x t scratch, given) write them once and
// take the wide product, where regenerating them per gathered neighbour row
// would cost 21 generator calls per value.  Both sum in the same order.
Status spmm_bt_probe(Model& M, double* Y, int t, const double* s, uint64_t seed, uint32_t tag2,
                     int col0, int gauss2, const double* d, uint32_t tag1, int gauss1,
                     double* tmp1, double* tmp2) {
  if (t > 64 && tmp1 && tmp2) {
    const int64_t nt = M.n * static_cast<int64_t>(t);
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((nt + 255) / 256, 8192));
    hipLaunchKernelGGL(probe_fill_kernel, dim3(g), dim3(256), 0, M.stream, M.n, t,
                       InProbe{s, seed, tag2, col0, gauss2}, tmp2);
    if (d)
      hipLaunchKernelGGL(probe_fill_kernel, dim3(g), dim3(256), 0, M.stream, M.n, t,
                         InProbe{nullptr, seed, tag1, col0, gauss1}, tmp1);
    VL_TRY(check_launch("probe fill"));
    return spmm_bt(M, tmp2, Y, t, d, d ? tmp1 : nullptr);
  }
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  const int* ord = spatial_order(M);
  InProbe x{s, seed, tag2, col0, gauss2};
  if (d) {
    InProbe v{nullptr, seed, tag1, col0, gauss1};
    hipLaunchKernelGGL((spmm_csr_t_kernel<InProbe, InProbe>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, x, d, v, Y);
  } else {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InProbe, InNone>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, ord, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, x, nullptr, InNone{},
                       Y);
  }
  return check_launch("spmm_bt_probe");
}

// --------------------------------------------------------- sync-free TRSM
constexpr int kSpinLimit = 1 << 22;    // poll rounds before a wave gives up

__device__ __forceinline__ int64_t grab(int* counter, int lane, int chunk) {
  int v = 0;
  if (lane == 0) v = atomicAdd(counter, 1);
  return static_cast<int64_t>(__shfl(v, 0)) * chunk;
}

// Work streams: units u = s + S k belong to stream s = blockIdx mod S, each
// stream with its own counter (own cache line) handing its units out in
// increasing order.  Every stream follows the global topological order, so
// the smallest unfinished unit can always be taken or finished: no deadlock,
// and S counters spread the atomic traffic.
__device__ __forceinline__ int64_t grab_stream(int* counters, int lane, int nstreams) {
  const int s = blockIdx.x % nstreams;
  int v = 0;
  if (lane == 0) v = atomicAdd(&counters[s * kCounterStride], 1);
  v = __shfl(v, 0);
  return static_cast<int64_t>(s) + static_cast<int64_t>(nstreams) * v;
}

// In-order consumption of a window whose entries k < k0 are already taken:
// applies acc -= v[k] y[k] while y[k] is ready and returns the first position
// still waiting (W once the window is done).  Empty slots hold v = y = 0,
// never the sentinel, and consumed entries are never reloaded, so the first
// sentinel in the window is the first entry still missing.
// A round in which no lane of the wave moves skips the updates.
template <int W, typename TY>
__device__ __forceinline__ int consume_window(const double* vb, const TY* yv, int k0,
                                              double& acc) {
  int fm = W;
#pragma unroll
  for (int k = W - 1; k >= 0; --k) fm = is_sentinel(yv[k]) ? k : fm;
  if (__any(fm > k0)) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double nx = acc - vb[k] * static_cast<double>(yv[k]);
      acc = (k >= k0 && k < fm) ? nx : acc;
    }
  }
  return fm;
}

// One row of a triangular solve, consumed in windows of W entries:
//   Y_i = rs_i X_i - sum_q vals[q] Y_{idx[q]},  q in [q0, e) (idx < 0 ends the row).
// A window's coefficients and the byte offsets of its Y entries are loaded
// once; its Y entries are read first through the caches (a cached copy can
// only be a stale sentinel, since every entry changes once, from the sentinel
// to its final value) and then only the still-missing ones are polled
// device-coherently.  Entries are consumed in a fixed order (windows
// ascending for B, descending for B^T; ascending inside a window), so the sum
// order is fixed.  Rows r0..n-1 are solved, taken in the topological order
// `order` (level by level) when given, else ascending (lower) / descending
// (upper); rows below r0 must be final.  The caller guarantees that every
// byte offset n * t * sizeof(TY) fits in 32 bits.
template <int W, bool LOWER, class In, typename TY = double>
__global__ __launch_bounds__(256) void trsm_kernel(int64_t n, int64_t r0, int m, int t, Lanes L,
                                                   const int* __restrict__ order,
                                                   const int* __restrict__ ptr,
                                                   const int* __restrict__ idx,
                                                   const double* __restrict__ vals, In x,
                                                   const double* __restrict__ rs, TY* Y,
                                                   int nstreams, int* counter, int* abort_flag,
                                                   int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t nt = n - r0;
  const int64_t total = units_of_hd(nt, t, L);
  char* const ybase = reinterpret_cast<char*>(Y);
  for (;;) {
    const int64_t unit = grab_stream(counter, lane, nstreams);
    if (unit >= total) return;
    {
      const int64_t rg = unit / L.slices;
      const int slice = static_cast<int>(unit - rg * L.slices);
      const int64_t r = (rg << L.rpw_log) + (lane >> L.lpr_log);
      const int c = slice * 64 + (lane & ((1 << L.lpr_log) - 1));
      const bool valid = (r < nt) && (c < t);
      int64_t i = LOWER ? (r0 + r) : (n - 1 - r);
      if (order && r < nt) i = order[r];
      bool pending = valid;
      double acc = 0.0;
      int q = 0, e = 0, wb = 0;  // row entries [q, e); current window [wb, wb + W)
      if (valid) {
        acc = x(i, c);
        if (rs) acc *= rs[i];
        if (LOWER) {
          q = static_cast<int>(i * m);
          e = q + m;
        } else {
          q = ptr[i];
          e = ptr[i + 1];
        }
        // The last window consumed is a full one: a row's slowest entry is
        // then likely in it, and no window load follows the last arrival.
        // Lower rows run forward with the remainder in the first window (sum
        // order unchanged).  B^T rows (children in ascending index) run from
        // their last window back: the latest children are solved first in
        // the backward order, so the last window holds the slowest entries.
        wb = LOWER ? e - W * ((e - q + W - 1) / W) : e - W;
        if (q >= e) {
          publish(&Y[i * t + c], static_cast<TY>(acc));
          pending = false;
        }
      }
      uint32_t bo[W];  // byte offset of each entry's Y value
      double vb[W];
      TY yv[W];
      int kk = W;  // cursor in the current window; W = no window loaded
      int rounds = 0;
      while (__any(pending)) {
        bool progressed = false;
        if (pending) {
          if (kk == W) {
            int jw[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
              const bool in = (wb + k >= q) && (wb + k < e);
              jw[k] = in ? idx[wb + k] : -1;
              vb[k] = in ? vals[wb + k] : 0.0;  // 0 in padding slots
              bo[k] = (static_cast<uint32_t>(jw[k]) * static_cast<uint32_t>(t) +
                       static_cast<uint32_t>(c)) * static_cast<uint32_t>(sizeof(TY));
            }
#pragma unroll
            for (int k = 0; k < W; ++k)
              yv[k] = (jw[k] >= 0) ? *reinterpret_cast<const TY*>(ybase + bo[k]) : TY(0);
            kk = 0;
          } else {
#pragma unroll
            for (int k = 0; k < W; ++k)
              if (is_sentinel(yv[k]))
                yv[k] = poll_load(reinterpret_cast<const TY*>(ybase + bo[k]));
          }
          const int fm = consume_window<W>(vb, yv, kk, acc);
          progressed = fm > kk;
          kk = fm;
          if (kk == W) {
            if (LOWER ? (wb + W >= e) : (wb <= q)) {  // slots outside the row are empty
              publish(&Y[i * t + c], static_cast<TY>(acc));
              pending = false;
            } else {
              wb += LOWER ? W : -W;  // window consumed: the next round loads the next one
            }
          }
        }
        if (__any(pending) && !__any(progressed)) {
          ++rounds;
          __builtin_amdgcn_s_sleep(1);
          if ((rounds & 63) == 0) {
            if (poll_load(abort_flag) != 0) return;
            if (rounds > kSpinLimit) {
              if (lane == 0) {
                publish(abort_flag, 1);
                raise_error(status, kErrTimeout);
              }
              return;
            }
          }
        }
      }
    }
  }
}

// Fill Y with the sentinel and reset the work counter and abort flag.
template <typename TY>
__global__ void trsm_prefill(TY* __restrict__ Y, int64_t count, int* counter) {
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < kSlotInts; k += blockDim.x) counter[k] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    Y[i] = sentinel_of<TY>();
}

// Level-scheduled solve of one level (wide blocks, t > 64).  All rows a
// level depends on were written by earlier launches on the stream, so plain
// cached loads are safe and nothing waits.  A thread covers VEC adjacent
// columns with 16-byte accesses (VEC = 2) when the width allows, so a wave
// issues one gather instruction per neighbour row for 128 columns; each
// column keeps its own accumulator, so VEC does not change any result.
//
// Forward (B Y = rs o X, ELL): block (k, s) solves row rows[k] for its
// slice of columns, subtracting the terms in slot order, as in the sync-free
// kernel (neighbours form a prefix, so an empty slot ends the row).
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_lower_kernel(
    int t, const int* __restrict__ rows, int m, const int* __restrict__ idx,
    const double* __restrict__ vals, const double* __restrict__ X,
    const double* __restrict__ rs, double* __restrict__ Y) {
  const int c = (blockIdx.y * blockDim.x + threadIdx.x) * VEC;
  const int64_t i = rows[blockIdx.x];
  if (c >= t) return;
  const int* nb = idx + i * m;
  const double* vb = vals + i * m;
  double acc[VEC];
  vld<VEC>(X + i * t + c, acc);
  if (rs) {
    const double s = rs[i];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] *= s;
  }
  for (int q = 0; q < m; q += 8) {
    int cb[8];
    double w[8], y[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cb[k] = (q + k < m) ? nb[q + k] : -1;
      w[k] = (q + k < m) ? vb[q + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] >= 0) {
        vld<VEC>(Y + (int64_t)cb[k] * t + c, y[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) y[k][v] = 0.0;
      }
    }
    bool ended = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] < 0) ended = true;
      if (!ended) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] -= w[k] * y[k][v];
      }
    }
    if (ended) break;
  }
  vst<VEC>(Y + i * t + c, acc);
}

// Backward (B^T Y = X, CSR): the same per row over the entries
// [ptr[i], end_i), end_i = pend[i] if pend is given (the head rows'
// head-internal prefix), else ptr[i + 1].
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_upper_kernel(
    int t, const int* __restrict__ rows, const int* __restrict__ ptr,
    const int* __restrict__ pend, const int* __restrict__ idx, const double* __restrict__ vals,
    const double* __restrict__ X, double* __restrict__ Y) {
  const int c = (blockIdx.y * blockDim.x + threadIdx.x) * VEC;
  const int64_t i = rows[blockIdx.x];
  if (c >= t) return;
  int q = ptr[i];
  const int e = pend ? pend[i] : ptr[i + 1];
  double acc[VEC];
  vld<VEC>(X + i * t + c, acc);
  for (; q < e; q += 8) {
    int cb[8];
    double w[8], y[8][VEC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      cb[k] = (q + k < e) ? idx[q + k] : -1;
      w[k] = (q + k < e) ? vals[q + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (cb[k] >= 0) {
        vld<VEC>(Y + (int64_t)cb[k] * t + c, y[k]);
      } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) y[k][v] = 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (cb[k] >= 0) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] -= w[k] * y[k][v];
      }
  }
  vst<VEC>(Y + i * t + c, acc);
}

// The same for levels of long B^T rows (average length above 16): block
// (k, s) covers 64 * VEC columns of row rows[k] with 4 waves sharing the
// row's entries.  `pend` as above.
template <int VEC>
__global__ __launch_bounds__(256) void trsm_level_split_kernel(int t, const int* __restrict__ rows,
                                                               const int* __restrict__ ptr,
                                                               const int* __restrict__ pend,
                                                               const int* __restrict__ idx,
                                                               const double* __restrict__ vals,
                                                               const double* __restrict__ X,
                                                               double* __restrict__ Y) {
  const int c = (blockIdx.y * 64 + (threadIdx.x & 63)) * VEC;
  const int64_t i = rows[blockIdx.x];
  const int b = ptr[i], e = pend ? pend[i] : ptr[i + 1];
  double tot[VEC];
  if (!split_row_sum<VEC>(t, c, b, e, idx, vals, Y, tot)) return;
  double x[VEC];
  vld<VEC>(X + i * t + c, x);
#pragma unroll
  for (int v = 0; v < VEC; ++v) x[v] -= tot[v];
  vst<VEC>(Y + i * t + c, x);
}

// Fold of the head rows' tail entries (B^T Y = X, after every tail row is
// solved): Xh_j = X_j - sum over the entries [pend[j], ptr[j + 1]) of row j,
// for all head rows j < H in one launch, block (j, s) covering 64 * VEC
// columns.  The head rows then solve against Xh with their head-internal
// entries only, so the long tail part of an early point's row never sits on
// a level's critical path.
template <int VEC, typename TY>
__global__ __launch_bounds__(256) void trsm_fold_kernel(int t, const int* __restrict__ ptr,
                                                        const int* __restrict__ pend,
                                                        const int* __restrict__ idx,
                                                        const TY* __restrict__ vals,
                                                        const double* __restrict__ X,
                                                        const TY* __restrict__ Y,
                                                        double* __restrict__ Xh) {
  const int c = (blockIdx.y * 64 + (threadIdx.x & 63)) * VEC;
  const int64_t j = blockIdx.x;
  double tot[VEC];
  if (!split_row_sum<VEC>(t, c, pend[j], ptr[j + 1], idx, vals, Y, tot)) return;
  double x[VEC];
  vld<VEC>(X + j * t + c, x);
#pragma unroll
  for (int v = 0; v < VEC; ++v) x[v] -= tot[v];
  vst<VEC>(Xh + j * t + c, x);
}

// out_j = base_j - sum over the B^T entries [beg[j], end[j]) of row j, for
// rows j < rows; block (j, s) covers 64 VEC columns with 4 waves sharing the
// row's entries (the wide-block fold before the dense leading rows).
template <int VEC, typename TY>
__global__ __launch_bounds__(256) void range_fold_kernel(int t, const int* __restrict__ beg,
                                                         const int* __restrict__ end,
                                                         const int* __restrict__ idx,
                                                         const TY* __restrict__ vals,
                                                         const double* __restrict__ base,
                                                         const TY* __restrict__ Y,
                                                         double* __restrict__ out) {
  const int c = (blockIdx.y * 64 + (threadIdx.x & 63)) * VEC;
  const int64_t j = blockIdx.x;
  double tot[VEC];
  if (!split_row_sum<VEC>(t, c, beg[j], end[j], idx, vals, Y, tot)) return;
  double x[VEC];
  vld<VEC>(base + j * t + c, x);
#pragma unroll
  for (int v = 0; v < VEC; ++v) x[v] -= tot[v];
  vst<VEC>(out + j * t + c, x);
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Column vector width of the level kernels: 16-byte accesses need t a
// multiple of the width and 16-byte aligned blocks.
int level_vec(int t, int elem_bytes, const void* a, const void* b, const void* c) {
  const bool al = aligned16(a) && aligned16(b) && (c == nullptr || aligned16(c));
  if (!al) return 1;
  const int want = 16 / elem_bytes;  // 2 doubles or 4 floats
  if (t % want == 0) return want;
  if (want == 4 && t % 2 == 0) return 2;
  return 1;
}

Status fold_launch_f32(Model& M, const double* X, const float* Y, double* Xh, int t) {
  const int H = M.head_rows;
  if (H <= 0) return Status::ok();
  TimedLaunch tl(M, kTimeLevelUpperFold, 8.0 * M.fold_nnz + 8.0 * H * t + 8.0 * H * t);
  const int vec = level_vec(t, 4, X, Y, Xh);
  const dim3 grid(H, (t + 64 * vec - 1) / (64 * vec));
  if (vec == 4) {
    hipLaunchKernelGGL((trsm_fold_kernel<4, float>), grid, dim3(256), 0, M.stream, t, M.bt_ptr.p,
                       M.head_split.p, M.bt_col.p, M.bt_val_f.p, X, Y, Xh);
  } else if (vec == 2) {
    hipLaunchKernelGGL((trsm_fold_kernel<2, float>), grid, dim3(256), 0, M.stream, t, M.bt_ptr.p,
                       M.head_split.p, M.bt_col.p, M.bt_val_f.p, X, Y, Xh);
  } else {
    hipLaunchKernelGGL((trsm_fold_kernel<1, float>), grid, dim3(256), 0, M.stream, t, M.bt_ptr.p,
                       M.head_split.p, M.bt_col.p, M.bt_val_f.p, X, Y, Xh);
  }
  return check_launch("trsm fold f32");
}

Status fold_rows(Model& M, int rows, const int* beg, const int* end, const double* base,
                 const double* Y, double* out, int t) {
  if (rows <= 0) return Status::ok();
  const int vec = level_vec(t, 8, base, Y, out);
  const dim3 grid(static_cast<unsigned>(rows), (t + 64 * vec - 1) / (64 * vec));
  if (vec == 2) {
    hipLaunchKernelGGL((range_fold_kernel<2, double>), grid, dim3(256), 0, M.stream, t, beg, end,
                       M.bt_col.p, M.bt_val.p, base, Y, out);
  } else {
    hipLaunchKernelGGL((range_fold_kernel<1, double>), grid, dim3(256), 0, M.stream, t, beg, end,
                       M.bt_col.p, M.bt_val.p, base, Y, out);
  }
  return check_launch("range fold");
}

// The same with Y and the B^T values in FP32 (the mixed-precision solves).
Status fold_rows(Model& M, int rows, const int* beg, const int* end, const double* base,
                 const float* Y, double* out, int t) {
  if (rows <= 0) return Status::ok();
  const int vec = level_vec(t, 4, base, Y, out);
  const dim3 grid(static_cast<unsigned>(rows), (t + 64 * vec - 1) / (64 * vec));
  if (vec == 4) {
    hipLaunchKernelGGL((range_fold_kernel<4, float>), grid, dim3(256), 0, M.stream, t, beg, end,
                       M.bt_col.p, M.bt_val_f.p, base, Y, out);
  } else if (vec == 2) {
    hipLaunchKernelGGL((range_fold_kernel<2, float>), grid, dim3(256), 0, M.stream, t, beg, end,
                       M.bt_col.p, M.bt_val_f.p, base, Y, out);
  } else {
    hipLaunchKernelGGL((range_fold_kernel<1, float>), grid, dim3(256), 0, M.stream, t, beg, end,
                       M.bt_col.p, M.bt_val_f.p, base, Y, out);
  }
  return check_launch("range fold f32");
}

// Levels [lp] of the forward order `order`.
static Status lower_levels(Model& M, const std::vector<int>& lp, const std::vector<int64_t>& lnz,
                           const int* order, const double* X, double* Y, int t,
                           const double* rs) {
  const int tb = t <= 64 ? 64 : 256;  // threads per block
  const int vec = level_vec(t, 8, X, Y, nullptr);
  const unsigned gy = static_cast<unsigned>((t + tb * vec - 1) / (tb * vec));
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    TimedLaunch tl(M, kTimeLevelLower,
                   12.0 * lnz[l] + 16.0 * rows * t + 4.0 * rows + (rs ? 8.0 * rows : 0.0));
    const int* r = order + lp[l];
    if (vec == 2) {
      hipLaunchKernelGGL(trsm_level_lower_kernel<2>, dim3(rows, gy), dim3(tb), 0, M.stream, t, r,
                         M.m, M.nbr.p, M.bval.p, X, rs, Y);
    } else {
      hipLaunchKernelGGL(trsm_level_lower_kernel<1>, dim3(rows, gy), dim3(tb), 0, M.stream, t, r,
                         M.m, M.nbr.p, M.bval.p, X, rs, Y);
    }
  }
  return check_launch("trsm level lower");
}

// Levels [lp] of the rows `order`; entries [ptr[i], pend ? pend[i] : ptr[i+1]).
static Status upper_levels(Model& M, const std::vector<int>& lp, const std::vector<int64_t>& lnz,
                           const int* order, const int* pend, const double* X, double* Y, int t) {
  const int tb = t <= 64 ? 64 : 256;
  const int vec = level_vec(t, 8, X, Y, nullptr);
  const unsigned gy = static_cast<unsigned>((t + tb * vec - 1) / (tb * vec));
  const unsigned gs = static_cast<unsigned>((t + 64 * vec - 1) / (64 * vec));
  for (size_t l = 0; l + 1 < lp.size(); ++l) {
    const int rows = lp[l + 1] - lp[l];
    if (rows <= 0) continue;
    const bool split = lnz[l] > 16LL * rows;
    TimedLaunch tl(M, split ? kTimeLevelUpperSplit : kTimeLevelUpper,
                   12.0 * lnz[l] + 16.0 * rows * t + 8.0 * rows);
    const int* r = order + lp[l];
    if (split && vec == 2) {
      hipLaunchKernelGGL(trsm_level_split_kernel<2>, dim3(rows, gs), dim3(256), 0, M.stream, t, r,
                         M.bt_ptr.p, pend, M.bt_col.p, M.bt_val.p, X, Y);
    } else if (split) {
      hipLaunchKernelGGL(trsm_level_split_kernel<1>, dim3(rows, gs), dim3(256), 0, M.stream, t, r,
                         M.bt_ptr.p, pend, M.bt_col.p, M.bt_val.p, X, Y);
    } else if (vec == 2) {
      hipLaunchKernelGGL(trsm_level_upper_kernel<2>, dim3(rows, gy), dim3(tb), 0, M.stream, t, r,
                         M.bt_ptr.p, pend, M.bt_col.p, M.bt_val.p, X, Y);
    } else {
      hipLaunchKernelGGL(trsm_level_upper_kernel<1>, dim3(rows, gy), dim3(tb), 0, M.stream, t, r,
                         M.bt_ptr.p, pend, M.bt_col.p, M.bt_val.p, X, Y);
    }
  }
  return check_launch("trsm level upper");
}

// One launch per level; each launch is timed on its own when timing is on.
// B Y = rs o X runs the full level order.  B^T Y = X with t > 64 runs in
// three stages: the tail rows by level (they depend on tail rows only), one
// fold of every head row's tail entries into Xh = X - (tail part), then the
// head rows by their head-internal levels against Xh.
static Status trsm_levels(Model& M, bool lower, const double* X, double* Y, int t,
                          const double* rowscale) {
  // wide blocks with the dense leading rows: those first (forward) or last
  // (backward) from G's leading block, the rest by its own levels
  const bool dense = t > 64 && M.dense_wide > 0;
  if (lower) {
    if (dense) {
      if (M.dlvl_ptr_f.size() < 2 || M.dlvl_ptr_f.back() != M.n - M.dense_wide)
        return Status::make(VL_ERR_STATE, "no level schedule");
      VL_TRY(dense_wide_lower(M, X, Y, t, rowscale));
      return lower_levels(M, M.dlvl_ptr_f, M.dlvl_nnz_f, M.dfull_order_f.p, X, Y, t, rowscale);
    }
    if (M.lvl_ptr_f.size() < 2 || M.lvl_ptr_f.back() != M.n)
      return Status::make(VL_ERR_STATE, "no level schedule");
    return lower_levels(M, M.lvl_ptr_f, M.lvl_nnz_f, M.full_order_f.p, X, Y, t, rowscale);
  }
  // Narrow blocks (t <= 64, when the level path is forced): the fold would
  // leave most lanes of its launch idle, so the full level order is used.
  if (t <= 64) {
    if (M.lvl_ptr_b.size() < 2 || M.lvl_ptr_b.back() != M.n)
      return Status::make(VL_ERR_STATE, "no level schedule");
    return upper_levels(M, M.lvl_ptr_b, M.lvl_nnz_b, M.full_order_b.p, nullptr, X, Y, t);
  }
  const int64_t H = M.head_rows;
  if (M.hlv_ptr_b.size() < 2 || M.hlv_ptr_b.back() != H ||
      (M.n > H && (M.tlvl_ptr_b.size() < 2 || M.tlvl_ptr_b.back() != M.n - H)))
    return Status::make(VL_ERR_STATE, "no level schedule");
  if (M.n > H)
    VL_TRY(upper_levels(M, M.tlvl_ptr_b, M.tlvl_nnz_b, M.tail_order_b.p, nullptr, X, Y, t));
  VL_TRY(M.lvl_fold.reserve(static_cast<size_t>(H) * t));
  {
    TimedLaunch tl(M, kTimeLevelUpperFold, 12.0 * M.fold_nnz + 16.0 * H * t);
    const int vec = level_vec(t, 8, X, Y, M.lvl_fold.p);
    const dim3 grid(static_cast<unsigned>(H), (t + 64 * vec - 1) / (64 * vec));
    if (vec == 2) {
      hipLaunchKernelGGL((trsm_fold_kernel<2, double>), grid, dim3(256), 0, M.stream, t,
                         M.bt_ptr.p, M.head_split.p, M.bt_col.p, M.bt_val.p, X, Y, M.lvl_fold.p);
    } else {
      hipLaunchKernelGGL((trsm_fold_kernel<1, double>), grid, dim3(256), 0, M.stream, t,
                         M.bt_ptr.p, M.head_split.p, M.bt_col.p, M.bt_val.p, X, Y, M.lvl_fold.p);
    }
    VL_TRY(check_launch("trsm fold"));
  }
  if (dense) {
    if (M.dhlv_ptr_b.size() < 2 || M.dhlv_ptr_b.back() != H - M.dense_wide)
      return Status::make(VL_ERR_STATE, "no level schedule");
    VL_TRY(upper_levels(M, M.dhlv_ptr_b, M.dhlv_nnz_b, M.dhlv_rows_b.p, M.head_split.p,
                        M.lvl_fold.p, Y, t));
    return dense_wide_upper(M, M.lvl_fold.p, Y, t);
  }
  return upper_levels(M, M.hlv_ptr_b, M.hlv_nnz_b, M.hlv_rows_b.p, M.head_split.p, M.lvl_fold.p,
                      Y, t);
}

static int trsm_grid(int64_t total_units) {
  int64_t blocks = (total_units + 3) / 4;
  const int64_t cap = 256 * 8;  // about eight resident blocks per CU
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return static_cast<int>(blocks);
}

// Grid of a sync-free tail solve whose order spans `levels` dependency
// levels: enough waves for about kTailLookahead levels' worth of units.  More
// waves only add waiting rows, and every waiting row re-polls its missing
// entries each round: at t = 1 (1500 units over ~200 levels at n = 1e5) all
// units in flight made each round 4.7 us of memory traffic, and 32-64 blocks
// instead of 375 took the forward solve from 0.52 to 0.41 ms.  With the
// small windows a lookahead of 32 levels beat 8, 16 and 64 (mode 276 ms
// against 320, 286 and 284).  Wide blocks (t = 50: 96k units) keep the
// resident maximum.
constexpr int64_t kTailLookahead = 32;
static int levels_of(const std::vector<int>& level_ptr) {
  return level_ptr.size() > 1 ? static_cast<int>(level_ptr.size()) - 1 : 0;
}
static int tail_grid(int64_t total_units, int levels) {
  int64_t blocks = (total_units + 3) / 4;
  if (levels > 0) {
    const int64_t want = (kTailLookahead * total_units / levels + 3) / 4;
    blocks = std::min(blocks, std::max<int64_t>(want, 32));
  }
  return trsm_grid(blocks * 4);
}

static int trsm_streams(const Model& M, int blocks) {
  int s = blocks < kCounterStreams ? blocks : kCounterStreams;
  if (s > M.num_cus) s = M.num_cus;
  if (M.max_streams > 0 && s > M.max_streams) s = M.max_streams;
  return s < 1 ? 1 : s;
}

// Counter slots: slot k uses counter[k * kSlotInts ...] (streams and abort
// flag).  Callers that pre-fill the output themselves must also have reset
// the slot.
static int* counter_slot(Model& M, int slot) {
  return M.ext ? M.ext->counter : M.counter.p + slot * kSlotInts;
}

template <typename TY>
static Status trsm_prepare(Model& M, TY* Y, int64_t count, int slot) {
  if (!M.ext) VL_TRY(M.counter.reserve(2 * kSlotInts + 64));
  int g = static_cast<int>((count + 255) / 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(trsm_prefill<TY>, dim3(g), dim3(256), 0, M.stream, Y, count,
                     counter_slot(M, slot));
  return check_launch("trsm prefill");
}

// Blocks wider than 64 columns have ample parallelism inside each level and
// are bandwidth-bound: they take the level-scheduled path (no sentinel fill,
// no polling).  Narrower blocks take the dense leading block and the
// sync-free tail.
static bool use_levels(const Model& M, int t) {
  return (t > 64 || M.force_levels) && M.lvl_ptr_f.size() > 1;
}

// Window widths of the tail solve (see lower_window / upper_window).
constexpr int kLowerWindowNarrow = 8, kLowerWindowWide = 4;  // B's rows, level-sorted
constexpr int kUpperWindowNarrow = 1, kUpperWindowWide = 4;  // B^T rows

// Launch of the sync-free tail solve with window width W.
template <bool LOWER, class In, typename TY>
static Status launch_tail(Model& M, int W, int g, int64_t H, int t, Lanes L, const int* ord,
                          const int* ptr, const int* idx, const double* val, In x,
                          const double* rowscale, TY* Y, int ns, int* cnt) {
  // Entries are addressed by 32-bit byte offsets into Y.
  if (static_cast<uint64_t>(M.n) * static_cast<uint64_t>(t) * sizeof(TY) >= (1ull << 32))
    return Status::invalid("triangular solve block larger than 4 GiB");
  const int m = LOWER ? M.m : 0;
#define VL_TAIL(WW)                                                                          \
  hipLaunchKernelGGL((trsm_kernel<WW, LOWER, In, TY>), dim3(g), dim3(256), 0, M.stream, M.n, \
                     H, m, t, L, ord, ptr, idx, val, x, rowscale, Y, ns, cnt,                \
                     cnt + kAbortOffset, M.status)
  if constexpr (LOWER) {
    if (W == kLowerWindowNarrow) {
      VL_TAIL(kLowerWindowNarrow);
    } else if (W == kLowerWindowWide) {
      VL_TAIL(kLowerWindowWide);
    } else {
      return Status::invalid("forward tail window");
    }
  } else {
    if (W == kUpperWindowNarrow) {
      VL_TAIL(kUpperWindowNarrow);
    } else if (W == kUpperWindowWide) {
      VL_TAIL(kUpperWindowWide);
    } else {
      return Status::invalid("backward tail window");
    }
  }
#undef VL_TAIL
  return check_launch(LOWER ? "trsm_b" : "trsm_bt");
}

// Window widths of the tail solve, measured at n = 1e5, m = 20.  A row is
// consumed window by window with its slowest entries last: forward, B's rows
// in tnbr order (neighbours sorted by forward level, tail_slots_kernel);
// backward, B^T rows from their last window back (children in ascending index
// finish in descending order).  The early windows are then taken while the
// row still waits for its slowest entries, only the last one follows the last
// arrival, and small windows win on registers and on the work of a round.
// Forward, with the level-sorted slots: t = 1 took 0.28 / 0.30 / 0.36 ms with
// 8 / 4 / 20 entries (0.39 ms with 20 in slot order), t = 50 0.38 / 0.35 /
// 0.49 ms with 8 / 4 / 16 (0.56 ms with 16 in slot order; 0.38 ms with 2).
// Backward: t = 1 took 0.28 / 0.34 / 0.35 / 0.39 / 0.48 ms with 1 / 2 / 4 / 8 /
// 16 entries, t = 50 0.48 / 0.46 / 0.48 / 0.57 ms with 2 / 4 / 8 / 16.
static int lower_window(int t) { return t <= 8 ? kLowerWindowNarrow : kLowerWindowWide; }
static int upper_window(int t) { return t <= 8 ? kUpperWindowNarrow : kUpperWindowWide; }
static const int* tail_nbr(const Model& M) { return M.tnbr.p ? M.tnbr.p : M.nbr.p; }
static const double* tail_val(const Model& M) { return M.tval.p ? M.tval.p : M.bval.p; }

// First row of the sync-free tail for narrow blocks, in both directions: the
// rows below come from the dense block.  An LDS head for the rows between
// (one workgroup per column walking their levels in shared memory) was
// measured and removed: it walks a level no faster than the sync-free kernel
// does.  At n = 1e5, m = 20 the forward solve took 0.53 / 0.63 ms at t = 1 / 50
// without it against 0.56 / 0.69 ms with it, and after the backward kernel's
// window changes a backward head of 12288 rows cost 11 ms of mode and 16 ms of
// likelihood per evaluation against none.
static int64_t narrow_tail_start(const Model& M, int t) { return t <= 64 ? M.dense_rows : 0; }

// Entries of B's rows below r (row i has min(i, m) off-diagonal entries).
static double nnz_below(const Model& M, int64_t r) {
  const double m = M.m, rr = static_cast<double>(r);
  return rr <= m ? rr * (rr - 1.0) / 2.0 : rr * m - m * (m + 1.0) / 2.0;
}

Status trsm_b_slot(Model& M, const double* X, double* Y, int t, const double* rowscale,
                   bool prefilled, int slot) {
  if (M.bd_use) return bd_lower(M, X, Y, t, rowscale);
  if (use_levels(M, t)) return trsm_levels(M, true, X, Y, t, rowscale);
  if (!prefilled) VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, slot));
  const int64_t R0 = narrow_tail_start(M, t);
  if (R0 > 0) VL_TRY(dense_lower(M, X, Y, t, rowscale));
  if (R0 >= M.n) return Status::ok();
  Lanes L = Lanes::of(t);
  int g = tail_grid(units_of(M.n - R0, t), R0 ? M.tail_levels_f : levels_of(M.lvl_ptr_f));
  const int ns = trsm_streams(M, g);
  int* cnt = counter_slot(M, slot);
  PollingOrder order(M);
  TimedLaunch tl(M, kTimeTrsmLower,
                 12.0 * (M.nnz - nnz_below(M, R0)) + 16.0 * (M.n - R0) * t +
                     (rowscale ? 8.0 * (M.n - R0) : 0.0));
  return launch_tail<true>(M, lower_window(t), g, R0, t, L,
                           R0 ? M.tail_order_f.p : M.full_order_f.p, nullptr, tail_nbr(M),
                           tail_val(M), InMem{X, t}, rowscale, Y, ns, cnt);
}

Status trsm_bt_slot(Model& M, const double* X, double* Y, int t, bool prefilled, int slot) {
  if (M.bd_use) return bd_upper(M, X, Y, t);
  if (use_levels(M, t)) return trsm_levels(M, false, X, Y, t, nullptr);
  if (!prefilled) VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, slot));
  const int64_t R0 = narrow_tail_start(M, t);  // the backward tail ends at the same row
  if (R0 < M.n) {
    Lanes L = Lanes::of(t);
    int g = tail_grid(units_of(M.n - R0, t), R0 ? M.tail_levels_b : levels_of(M.lvl_ptr_b));
    const int ns = trsm_streams(M, g);
    int* cnt = counter_slot(M, slot);
    PollingOrder order(M);
    TimedLaunch tl(M, kTimeTrsmUpper,
                   12.0 * (M.nnz - (R0 ? M.nnz_bt_dense : 0)) + 4.0 * (M.n - R0) +
                       16.0 * (M.n - R0) * t);
    VL_TRY(launch_tail<false>(M, upper_window(t), g, R0, t, L,
                              R0 ? M.tail_order_bn.p : M.full_order_b.p, M.bt_ptr.p, M.bt_col.p,
                              M.bt_val.p, InMem{X, t}, nullptr, Y, ns, cnt));
  }
  if (R0 > 0) VL_TRY(dense_upper(M, X, Y, t));  // rows 0..K-1, after every later row
  return Status::ok();
}

// FP32-storage narrow solves (t <= 64) of the mixed-precision form: the same
// head and sync-free tail kernels with FP32 right-hand sides and results
// (FP64 B values, FP64 row sums), for the preconditioner of the FP64 PCG.
Status trsm_b_f32_narrow(Model& M, const float* X, float* Y, int t, const double* rowscale) {
  if (t > 64) return Status::invalid("narrow FP32 solve with more than 64 columns");
  VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, 0));
  const int64_t R0 = narrow_tail_start(M, t);
  if (R0 > 0) VL_TRY(dense_lower_f32(M, X, Y, t, rowscale));
  if (R0 >= M.n) return Status::ok();
  Lanes L = Lanes::of(t);
  int g = tail_grid(units_of(M.n - R0, t), R0 ? M.tail_levels_f : levels_of(M.lvl_ptr_f));
  const int ns = trsm_streams(M, g);
  int* cnt = counter_slot(M, 0);
  PollingOrder order(M);
  TimedLaunch tl(M, kTimeTrsmLower,
                 12.0 * (M.nnz - nnz_below(M, R0)) + 8.0 * (M.n - R0) * t +
                     (rowscale ? 8.0 * (M.n - R0) : 0.0));
  return launch_tail<true>(M, lower_window(t), g, R0, t, L,
                           R0 ? M.tail_order_f.p : M.full_order_f.p, nullptr, tail_nbr(M),
                           tail_val(M), InMemF{X, t}, rowscale, Y, ns, cnt);
}

Status trsm_bt_f32_narrow(Model& M, const double* X, float* Y, int t) {
  if (t > 64) return Status::invalid("narrow FP32 solve with more than 64 columns");
  VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, 0));
  const int64_t R0 = narrow_tail_start(M, t);
  if (R0 < M.n) {
    Lanes L = Lanes::of(t);
    int g = tail_grid(units_of(M.n - R0, t), R0 ? M.tail_levels_b : levels_of(M.lvl_ptr_b));
    const int ns = trsm_streams(M, g);
    int* cnt = counter_slot(M, 0);
    PollingOrder order(M);
    TimedLaunch tl(M, kTimeTrsmUpper,
                   12.0 * (M.nnz - (R0 ? M.nnz_bt_dense : 0)) + 4.0 * (M.n - R0) +
                       12.0 * (M.n - R0) * t);
    VL_TRY(launch_tail<false>(M, upper_window(t), g, R0, t, L,
                              R0 ? M.tail_order_bn.p : M.full_order_b.p, M.bt_ptr.p, M.bt_col.p,
                              M.bt_val.p, InMem{X, t}, nullptr, Y, ns, cnt));
  }
  if (R0 > 0) VL_TRY(dense_upper_f32(M, X, Y, t));
  return Status::ok();
}

Status trsm_b(Model& M, const double* X, double* Y, int t, const double* rowscale,
              bool prefilled) {
  return trsm_b_slot(M, X, Y, t, rowscale, prefilled, 0);
}

Status trsm_bt(Model& M, const double* X, double* Y, int t, bool prefilled) {
  return trsm_bt_slot(M, X, Y, t, prefilled, 0);
}

// ------------------------------------------------------ level schedules
// Longest-path level of every row in the dependency DAG of B (lower: over
// N(i); upper: over the rows of B^T), computed once per neighbour set with
// the same sync-free scheme as the solves (sentinel -1, 64 rows per wave).
// Lower: rows below r0 are known (their levels preset, not recomputed).
template <int W, bool LOWER>
__global__ __launch_bounds__(256) void levels_kernel(int64_t n, int64_t r0, int m,
                                                     const int* __restrict__ ptr,
                                                     const int* __restrict__ idx, int* lev,
                                                     int* counter, int* abort_flag,
                                                     int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t total = (n - r0 + 63) >> 6;
  for (;;) {
    const int64_t u = grab(counter, lane, 1);
    if (u >= total) return;
    const int64_t r = r0 + (u << 6) + lane;
    const bool valid = r < n;
    const int64_t i = LOWER ? r : (n - 1 - r);
    bool pending = valid;
    int q = 0, e = 0, acc = 0;
    if (valid) {
      if (LOWER) {
        q = static_cast<int>(i * m);
        e = q + m;
      } else {
        q = ptr[i];
        e = ptr[i + 1];
      }
    }
    int rounds = 0;
    while (__any(pending)) {
      bool progressed = false;
      if (pending) {
        int cb[W], lv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) cb[k] = (q + k < e) ? idx[q + k] : -1;
#pragma unroll
        for (int k = 0; k < W; ++k) lv[k] = (cb[k] >= 0) ? poll_load(&lev[cb[k]]) : 0;
        bool stop = false;
        int adv = 0;
        bool ended = false;
#pragma unroll
        for (int k = 0; k < W; ++k) {
          if (!stop) {
            if (cb[k] < 0) {
              stop = ended = true;
            } else if (lv[k] < 0) {
              stop = true;
            } else {
              acc = max(acc, lv[k] + 1);
              ++adv;
            }
          }
        }
        q += adv;
        progressed = adv > 0;
        if (ended || q >= e) {
          publish(&lev[i], acc);
          pending = false;
        }
      }
      if (__any(pending) && !__any(progressed)) {
        ++rounds;
        __builtin_amdgcn_s_sleep(1);
        if ((rounds & 63) == 0) {
          if (poll_load(abort_flag) != 0) return;
          if (rounds > kSpinLimit) {
            if (lane == 0) {
              publish(abort_flag, 1);
              raise_error(status, kErrTimeout);
            }
            return;
          }
        }
      }
    }
  }
}

// Counting sort of rows >= r0 by level, visiting rows in spatial order so
// rows of one level stay roughly spatially sorted.
__global__ void level_count_kernel(int64_t n, int64_t r0, const int* __restrict__ spatial,
                                   const int* __restrict__ lev, int* __restrict__ cnt) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int r = spatial[k];
  if (r < r0) return;
  const int l = lev[r];
  if (l >= 0) atomicAdd(&cnt[l], 1);
}

// nnz of the rows of each level (lower: entries with idx >= 0 of the ELL
// row; upper: the CSR row length)
__global__ void level_nnz_kernel(int64_t n, int64_t r0, int m, const int* __restrict__ ptr,
                                 const int* __restrict__ idx, const int* __restrict__ lev,
                                 unsigned long long* __restrict__ nnz) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || i < r0) return;
  int c = 0;
  if (ptr) {
    c = ptr[i + 1] - ptr[i];
  } else {
    for (int k = 0; k < m; ++k) c += idx[i * m + k] >= 0 ? 1 : 0;
  }
  const int l = lev[i];
  if (c && l >= 0) atomicAdd(&nnz[l], static_cast<unsigned long long>(c));
}

__global__ void level_scatter_kernel(int64_t n, int64_t r0, const int* __restrict__ spatial,
                                     const int* __restrict__ lev, const int* __restrict__ start,
                                     int* __restrict__ cursor, int* __restrict__ order) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int r = spatial[k];
  if (r < r0) return;
  const int l = lev[r];
  if (l < 0) return;
  order[start[l] + atomicAdd(&cursor[l], 1)] = r;
}

// Slots of every row of B ordered by the forward level of their neighbour
// (ties by slot; padding slots first): the forward tail consumes a row in this
// order, so its last window holds the neighbours solved last.  tnbr holds the
// neighbours, tsrc the source slot of each (for the values, refreshed with
// every factor).
__global__ void tail_slots_kernel(int64_t n, int m, const int* __restrict__ nbr,
                                  const int* __restrict__ lev, int* __restrict__ tnbr,
                                  int* __restrict__ tsrc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int key[32], slot[32];
  for (int k = 0; k < m; ++k) {
    const int j = nbr[i * m + k];
    key[k] = j >= 0 ? lev[j] : -1;
    slot[k] = k;
  }
  for (int a = 1; a < m; ++a) {  // insertion sort, stable
    const int ka = key[a], sa = slot[a];
    int b = a - 1;
    while (b >= 0 && key[b] > ka) {
      key[b + 1] = key[b];
      slot[b + 1] = slot[b];
      --b;
    }
    key[b + 1] = ka;
    slot[b + 1] = sa;
  }
  for (int k = 0; k < m; ++k) {
    tnbr[i * m + k] = nbr[i * m + slot[k]];
    tsrc[i * m + k] = static_cast<int>(i * m + slot[k]);
  }
}

Status build_tail_orders(Model& M) {
  const int64_t n = M.n, H = M.head_rows;
  const int64_t K = H > 0 ? M.dense_rows : 0;  // start of the narrow tails (narrow_tail_start)
  M.nnz_bt_dense = 0;
  if (K > 0) {
    VL_HIP(hipMemcpyAsync(&M.nnz_bt_dense, M.bt_ptr.p + K, sizeof(int), hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
  }
  VL_TRY(M.tail_order_f.alloc(n - K > 0 ? n - K : 1));
  VL_TRY(M.tail_order_bn.alloc(n - K > 0 ? n - K : 1));
  VL_TRY(M.tail_order_b.alloc(n - H > 0 ? n - H : 1));
  VL_TRY(M.full_order_f.alloc(n));
  VL_TRY(M.full_order_b.alloc(n));
  DevBuf<int> lev, cnt, start;
  VL_TRY(lev.alloc(n));
  VL_TRY(cnt.alloc(n + 1));
  VL_TRY(start.alloc(n + 1));
  VL_TRY(M.counter.reserve(2 * kSlotInts + 64));
  const int tb = 256;
  const unsigned gn = static_cast<unsigned>((n + tb - 1) / tb);
  for (int dir = 0; dir < 2; ++dir) {
    VL_TRY(fill_int(lev.p, -1, n, M.stream));
    VL_TRY(fill_int(M.counter.p, 0, 2, M.stream));
    const int64_t units = (n + 63) / 64;
    unsigned g = static_cast<unsigned>(std::min<int64_t>((units + 3) / 4, 2048));
    {
      PollingOrder order(M);
      if (dir == 0) {
        hipLaunchKernelGGL((levels_kernel<32, true>), dim3(g), dim3(256), 0, M.stream, n, 0,
                           M.m, nullptr, M.nbr.p, lev.p, M.counter.p, M.counter.p + 1, M.status);
      } else {
        hipLaunchKernelGGL((levels_kernel<16, false>), dim3(g), dim3(256), 0, M.stream, n, 0, 0,
                           M.bt_ptr.p, M.bt_col.p, lev.p, M.counter.p, M.counter.p + 1,
                           M.status);
      }
    }
    // A wave that reached its wait bound leaves rows without a level (-1):
    // stop before anything indexes by level.
    VL_TRY(check_launch("levels"));
    VL_TRY(read_status(M));
    if (dir == 0 && M.m > 0 && M.m <= 32) {
      const size_t nm = static_cast<size_t>(n) * M.m;
      VL_TRY(M.tnbr.alloc(nm));
      VL_TRY(M.tsrc.alloc(nm));
      VL_TRY(M.tval.alloc(nm));
      hipLaunchKernelGGL(tail_slots_kernel, dim3(gn), dim3(tb), 0, M.stream, n, M.m, M.nbr.p,
                         lev.p, M.tnbr.p, M.tsrc.p);
      VL_TRY(check_launch("tail slots"));
    }
    const int* spatial = static_cast<const int*>(M.grid_pts);
    // per direction: the narrow blocks' tail (rows >= K), the wide backward
    // solve's tail (rows >= H), the full order
    for (int kind = 0; kind < 3; ++kind) {
      if (kind == 1 && dir == 0) continue;
      const bool full = kind == 2;
      const int64_t r0 = kind == 0 ? K : kind == 1 ? H : 0;
      if (n - r0 <= 0) continue;
      int* out = full ? (dir == 0 ? M.full_order_f.p : M.full_order_b.p)
                 : kind == 0 ? (dir == 0 ? M.tail_order_f.p : M.tail_order_bn.p)
                             : M.tail_order_b.p;
      VL_TRY(fill_int(cnt.p, 0, n + 1, M.stream));
      hipLaunchKernelGGL(level_count_kernel, dim3(gn), dim3(tb), 0, M.stream, n, r0, spatial,
                         lev.p, cnt.p);
      VL_TRY(exclusive_scan_int(cnt.p, start.p, n + 1, M.stream));
      VL_TRY(fill_int(cnt.p, 0, n + 1, M.stream));
      hipLaunchKernelGGL(level_scatter_kernel, dim3(gn), dim3(tb), 0, M.stream, n, r0, spatial,
                         lev.p, start.p, cnt.p, out);
      VL_TRY(check_launch("level order"));
      if (kind == 0) {  // dependency levels the narrow tail order spans (sizes its grid)
        std::vector<int> st(n + 1);
        VL_HIP(hipMemcpyAsync(st.data(), start.p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost,
                              M.stream));
        VL_TRY(sync_stream(M.stream));
        int levels = 0;
        for (int64_t l = 0; l < n; ++l) levels += st[l + 1] > st[l];
        (dir == 0 ? M.tail_levels_f : M.tail_levels_b) = levels;
      }
      // level pointers and per-level nnz, to the host: of the full orders
      // (both directions) and of the wide backward tail order
      if (kind != 0) {
        const int64_t cnt_rows = n - r0;
        std::vector<int> st(n + 1);
        VL_HIP(hipMemcpyAsync(st.data(), start.p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost,
                              M.stream));
        VL_TRY(sync_stream(M.stream));
        int64_t L = 0;
        while (L < n && st[L] < cnt_rows) ++L;  // levels 0..L-1 hold the counted rows
        std::vector<int>& lp = full ? (dir == 0 ? M.lvl_ptr_f : M.lvl_ptr_b) : M.tlvl_ptr_b;
        lp.assign(st.begin(), st.begin() + L + 1);
        DevBuf<unsigned long long> lnz;
        VL_TRY(lnz.alloc(L > 0 ? L : 1));
        VL_HIP(hipMemsetAsync(lnz.p, 0, sizeof(unsigned long long) * (L > 0 ? L : 1), M.stream));
        hipLaunchKernelGGL(level_nnz_kernel, dim3(gn), dim3(tb), 0, M.stream, n, r0,
                           dir == 0 ? M.m : 0, dir == 0 ? nullptr : M.bt_ptr.p,
                           dir == 0 ? M.nbr.p : nullptr, lev.p, lnz.p);
        VL_TRY(check_launch("level nnz"));
        std::vector<unsigned long long> hz(L > 0 ? L : 1);
        VL_HIP(hipMemcpyAsync(hz.data(), lnz.p, sizeof(unsigned long long) * hz.size(),
                              hipMemcpyDeviceToHost, M.stream));
        VL_TRY(sync_stream(M.stream));
        std::vector<int64_t>& nz = full ? (dir == 0 ? M.lvl_nnz_f : M.lvl_nnz_b) : M.tlvl_nnz_b;
        nz.assign(hz.begin(), hz.begin() + L);
      }
    }
  }
  // forward order of the rows Kw..n-1 with the rows below Kw known (the wide
  // solves take those from the dense inverse)
  const int64_t Kw = M.dense_wide;
  if (Kw > 0 && n > Kw) {
    VL_TRY(fill_int(lev.p, -1, n, M.stream));
    VL_TRY(fill_int(lev.p, 0, Kw, M.stream));
    VL_TRY(fill_int(M.counter.p, 0, 2, M.stream));
    const int64_t units = (n - Kw + 63) / 64;
    unsigned g = static_cast<unsigned>(std::min<int64_t>((units + 3) / 4, 2048));
    {
      PollingOrder order(M);
      hipLaunchKernelGGL((levels_kernel<32, true>), dim3(g), dim3(256), 0, M.stream, n, Kw, M.m,
                         nullptr, M.nbr.p, lev.p, M.counter.p, M.counter.p + 1, M.status);
    }
    VL_TRY(check_launch("levels"));
    VL_TRY(read_status(M));
    const int* spatial = static_cast<const int*>(M.grid_pts);
    VL_TRY(M.dfull_order_f.alloc(n - Kw));
    VL_TRY(fill_int(cnt.p, 0, n + 1, M.stream));
    hipLaunchKernelGGL(level_count_kernel, dim3(gn), dim3(tb), 0, M.stream, n, Kw, spatial, lev.p,
                       cnt.p);
    VL_TRY(exclusive_scan_int(cnt.p, start.p, n + 1, M.stream));
    VL_TRY(fill_int(cnt.p, 0, n + 1, M.stream));
    hipLaunchKernelGGL(level_scatter_kernel, dim3(gn), dim3(tb), 0, M.stream, n, Kw, spatial,
                       lev.p, start.p, cnt.p, M.dfull_order_f.p);
    VL_TRY(check_launch("dense wide order"));
    std::vector<int> st(n + 1);
    VL_HIP(hipMemcpyAsync(st.data(), start.p, sizeof(int) * (n + 1), hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
    int64_t L = 0;
    while (L < n && st[L] < n - Kw) ++L;
    M.dlvl_ptr_f.assign(st.begin(), st.begin() + L + 1);
    DevBuf<unsigned long long> lnz;
    VL_TRY(lnz.alloc(L > 0 ? L : 1));
    VL_HIP(hipMemsetAsync(lnz.p, 0, sizeof(unsigned long long) * (L > 0 ? L : 1), M.stream));
    hipLaunchKernelGGL(level_nnz_kernel, dim3(gn), dim3(tb), 0, M.stream, n, Kw, M.m, nullptr,
                       M.nbr.p, lev.p, lnz.p);
    VL_TRY(check_launch("level nnz"));
    std::vector<unsigned long long> hz(L > 0 ? L : 1);
    VL_HIP(hipMemcpyAsync(hz.data(), lnz.p, sizeof(unsigned long long) * hz.size(),
                          hipMemcpyDeviceToHost, M.stream));
    VL_TRY(sync_stream(M.stream));
    M.dlvl_nnz_f.assign(hz.begin(), hz.begin() + L);
  }
  VL_TRY(sync_stream(M.stream));
  return read_status(M);
}

}  // namespace vl
