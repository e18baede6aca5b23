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

Status refresh_transpose_values(Model& M) {
  if (M.nnz == 0) return Status::ok();
  const int tb = 256;
  hipLaunchKernelGGL(bt_gather_vals, dim3((unsigned)((M.nnz + tb - 1) / tb)), dim3(tb), 0,
                     M.stream, M.nnz, M.bt_src.p, M.bval.p, M.bt_val.p);
  return check_launch("transpose values");
}

// ------------------------------------------------------------------ SpMM
struct UnitPos {
  int64_t i;
  int c;
  bool valid;
};
__device__ __forceinline__ UnitPos unit_pos(int64_t unit, int lane, Lanes L, int64_t n, int t,
                                            bool reverse) {
  int64_t rg = unit / L.slices;
  int slice = static_cast<int>(unit - rg * L.slices);
  int sub = lane >> L.lpr_log;
  int c = slice * 64 + (lane & ((1 << L.lpr_log) - 1));
  int64_t r = (rg << L.rpw_log) + sub;
  UnitPos p;
  p.i = reverse ? (n - 1 - r) : r;
  p.c = c;
  p.valid = (r < n) && (c < t);
  return p;
}

// Y_i = rs_i * (unit * X_i + sum_k vals[i,k] X_{nbr[i,k]})
template <class In>
__global__ __launch_bounds__(256) void spmm_ell_kernel(int64_t n, int m, int t, Lanes L,
                                                       const int* __restrict__ nbr,
                                                       const double* __restrict__ vals, In x,
                                                       const double* __restrict__ rs,
                                                       int unit_diag, double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (unit >= units_of_hd(n, t, L)) return;
  UnitPos p = unit_pos(unit, lane, L, n, t, false);
  if (!p.valid) return;
  const int* nb = nbr + p.i * m;
  const double* vb = vals + p.i * m;
  double acc = unit_diag ? x(p.i, p.c) : 0.0;
  for (int k = 0; k < m; ++k) {
    int j = nb[k];
    if (j < 0) break;
    acc += vb[k] * x(j, p.c);
  }
  if (rs) acc *= rs[p.i];
  Y[p.i * t + p.c] = acc;
}

// Y_j = d_j * v_j + X_j + sum_e btval[e] X_{btcol[e]}   (v from memory or probe)
template <class In, class Dv>
__global__ __launch_bounds__(256) void spmm_csr_t_kernel(
    int64_t n, int t, Lanes L, const int* __restrict__ ptr, const int* __restrict__ col,
    const double* __restrict__ val, In x, const double* __restrict__ d, Dv v,
    double* __restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int64_t unit = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (unit >= units_of_hd(n, t, L)) return;
  UnitPos p = unit_pos(unit, lane, L, n, t, false);
  if (!p.valid) return;
  double acc = x(p.i, p.c);
  const int b = ptr[p.i], e = ptr[p.i + 1];
  for (int q = b; q < e; ++q) acc += val[q] * x(col[q], p.c);
  if (d) acc += d[p.i] * v(p.i, p.c);
  Y[p.i * t + p.c] = acc;
}

struct InNone {
  __device__ __forceinline__ double operator()(int64_t, int) const { return 0.0; }
};

Status spmm_b(Model& M, const double* X, double* Y, int t, const double* rowscale) {
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  hipLaunchKernelGGL(spmm_ell_kernel<InMem>, dim3(nb), dim3(256), 0, M.stream, M.n, M.m, t, L,
                     M.nbr.p, M.bval.p, InMem{X, t}, rowscale, 1, Y);
  return check_launch("spmm_b");
}

Status spmm_ell_vals(Model& M, const double* vals, const double* X, double* Y, int t,
                     const double* rowscale, bool unit_diag) {
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  hipLaunchKernelGGL(spmm_ell_kernel<InMem>, dim3(nb), dim3(256), 0, M.stream, M.n, M.m, t, L,
                     M.nbr.p, vals, InMem{X, t}, rowscale, unit_diag ? 1 : 0, Y);
  return check_launch("spmm_ell");
}

Status spmm_bt(Model& M, const double* X, double* Y, int t, const double* diag,
               const double* diagvec) {
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  if (diag) {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InMem, InMem>), dim3(nb), dim3(256), 0, M.stream, M.n,
                       t, L, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, InMem{X, t}, diag,
                       InMem{diagvec, t}, Y);
  } else {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InMem, InNone>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, InMem{X, t}, nullptr,
                       InNone{}, Y);
  }
  return check_launch("spmm_bt");
}

// Y = d o probe1 + B^T (s o probe2), probes generated in place
Status spmm_bt_probe(Model& M, double* Y, int t, const double* s, uint64_t seed, uint32_t tag2,
                     int col0, int gauss2, const double* d, uint32_t tag1, int gauss1) {
  Lanes L = Lanes::of(t);
  int nb = spmm_nblocks(M.n, t);
  InProbe x{s, seed, tag2, col0, gauss2};
  if (d) {
    InProbe v{nullptr, seed, tag1, col0, gauss1};
    hipLaunchKernelGGL((spmm_csr_t_kernel<InProbe, InProbe>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, x, d, v, Y);
  } else {
    hipLaunchKernelGGL((spmm_csr_t_kernel<InProbe, InNone>), dim3(nb), dim3(256), 0, M.stream,
                       M.n, t, L, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, x, nullptr, InNone{}, Y);
  }
  return check_launch("spmm_bt_probe");
}

// --------------------------------------------------------- sync-free TRSM
constexpr int kTrsmChunk = 4;          // work units taken per counter increment
constexpr int kSpinLimit = 1 << 22;    // poll rounds before a wave gives up

__device__ __forceinline__ int64_t grab(int* counter, int lane) {
  int v = 0;
  if (lane == 0) v = atomicAdd(counter, 1);
  return static_cast<int64_t>(__shfl(v, 0)) * kTrsmChunk;
}

// Lower solve: Y_i = rs_i * X_i - sum_k vals[i,k] Y_{nbr[i,k]}   (B Y = rs o X)
template <class In>
__global__ __launch_bounds__(256) void trsm_lower_kernel(
    int64_t n, int m, int t, Lanes L, const int* __restrict__ nbr,
    const double* __restrict__ vals, In x, const double* __restrict__ rs, double* Y,
    int* counter, int* abort_flag, int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t total = units_of_hd(n, t, L);
  for (;;) {
    const int64_t u0 = grab(counter, lane);
    if (u0 >= total) return;
    for (int64_t unit = u0; unit < u0 + kTrsmChunk && unit < total; ++unit) {
      UnitPos p = unit_pos(unit, lane, L, n, t, false);
      bool pending = p.valid;
      double acc = 0.0;
      int k = 0;
      const int* nb = nbr + (p.valid ? p.i * m : 0);
      const double* vb = vals + (p.valid ? p.i * m : 0);
      if (p.valid) {
        acc = x(p.i, p.c);
        if (rs) acc *= rs[p.i];
      }
      int rounds = 0;
      while (__any(pending)) {
        if (pending) {
          for (; k < m; ++k) {
            const int j = nb[k];
            if (j < 0) {
              k = m;
              break;
            }
            const double v = poll_load(&Y[(int64_t)j * t + p.c]);
            if (is_sentinel(v)) break;
            acc -= vb[k] * v;
          }
          if (k >= m) {
            publish(&Y[p.i * t + p.c], acc);
            pending = false;
          }
        }
        if (__any(pending)) {
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

// Upper solve with B^T rows (CSR): Y_j = X_j - sum_e btval[e] Y_{btcol[e]}
template <class In>
__global__ __launch_bounds__(256) void trsm_upper_kernel(
    int64_t n, int t, Lanes L, const int* __restrict__ ptr, const int* __restrict__ col,
    const double* __restrict__ val, In x, double* Y, int* counter, int* abort_flag,
    int* status) {
  const int lane = threadIdx.x & 63;
  const int64_t total = units_of_hd(n, t, L);
  for (;;) {
    const int64_t u0 = grab(counter, lane);
    if (u0 >= total) return;
    for (int64_t unit = u0; unit < u0 + kTrsmChunk && unit < total; ++unit) {
      UnitPos p = unit_pos(unit, lane, L, n, t, true);
      bool pending = p.valid;
      double acc = 0.0;
      int q = 0, e = 0;
      if (p.valid) {
        acc = x(p.i, p.c);
        q = ptr[p.i];
        e = ptr[p.i + 1];
      }
      int rounds = 0;
      while (__any(pending)) {
        if (pending) {
          for (; q < e; ++q) {
            const double v = poll_load(&Y[(int64_t)col[q] * t + p.c]);
            if (is_sentinel(v)) break;
            acc -= val[q] * v;
          }
          if (q >= e) {
            publish(&Y[p.i * t + p.c], acc);
            pending = false;
          }
        }
        if (__any(pending)) {
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
__global__ void trsm_prefill(double* __restrict__ Y, int64_t count, int* counter) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    counter[0] = 0;
    counter[1] = 0;
  }
  for (; i < count; i += (int64_t)gridDim.x * blockDim.x) Y[i] = sentinel();
}

static int trsm_grid(int64_t total_units) {
  int64_t chunks = (total_units + kTrsmChunk - 1) / kTrsmChunk;
  int64_t blocks = (chunks + 3) / 4;
  const int64_t cap = 256 * 8;  // about eight resident blocks per CU
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return static_cast<int>(blocks);
}

// Counter slots: slot k uses counter[2k] (work units) and counter[2k + 1]
// (abort flag).  Callers that pre-fill the output themselves must also have
// reset the slot.
static Status trsm_prepare(Model& M, double* Y, int64_t count, int slot) {
  VL_TRY(M.counter.reserve(64));
  int g = static_cast<int>((count + 255) / 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(trsm_prefill, dim3(g), dim3(256), 0, M.stream, Y, count,
                     M.counter.p + 2 * slot);
  return check_launch("trsm prefill");
}

Status trsm_b_slot(Model& M, const double* X, double* Y, int t, const double* rowscale,
                   bool prefilled, int slot) {
  if (!prefilled) VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, slot));
  Lanes L = Lanes::of(t);
  int g = trsm_grid(units_of(M.n, t));
  int* cnt = M.counter.p + 2 * slot;
  hipLaunchKernelGGL(trsm_lower_kernel<InMem>, dim3(g), dim3(256), 0, M.stream, M.n, M.m, t, L,
                     M.nbr.p, M.bval.p, InMem{X, t}, rowscale, Y, cnt, cnt + 1, M.status);
  return check_launch("trsm_b");
}

Status trsm_bt_slot(Model& M, const double* X, double* Y, int t, bool prefilled, int slot) {
  if (!prefilled) VL_TRY(trsm_prepare(M, Y, M.n * (int64_t)t, slot));
  Lanes L = Lanes::of(t);
  int g = trsm_grid(units_of(M.n, t));
  int* cnt = M.counter.p + 2 * slot;
  hipLaunchKernelGGL(trsm_upper_kernel<InMem>, dim3(g), dim3(256), 0, M.stream, M.n, t, L,
                     M.bt_ptr.p, M.bt_col.p, M.bt_val.p, InMem{X, t}, Y, cnt, cnt + 1,
                     M.status);
  return check_launch("trsm_bt");
}

Status trsm_b(Model& M, const double* X, double* Y, int t, const double* rowscale,
              bool prefilled) {
  return trsm_b_slot(M, X, Y, t, rowscale, prefilled, 0);
}

Status trsm_bt(Model& M, const double* X, double* Y, int t, bool prefilled) {
  return trsm_bt_slot(M, X, Y, t, prefilled, 0);
}

}  // namespace vl
