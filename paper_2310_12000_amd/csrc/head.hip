// Backward triangular solves with B^T over the "head" rows 0..H-1.
//
// With a random ordering the dependency DAG of B is deep only among early
// rows: for n = 1e5, m = 20 the first 16384 rows already span 214 of the 278
// levels, while the remaining rows add only 68.  The first K rows are solved
// with the dense inverse of B's leading block (dense.hip).  Backward
// (B^T Y = X), the tail rows are solved first (sparse.hip), then rows K..H-1
// (K = 4096, H = 12288 by default) level by level inside one workgroup per
// probe column, with the column's head values in LDS and no barrier between
// levels (rows poll LDS), reading finished tail values from global memory;
// then the dense block.  The early points' B^T rows are long (they are
// neighbours of many later points), which is what the LDS head absorbs.
// Forward (B Y = rs o X) needs no head: the dense block, then the sync-free
// tail from row K.
//
// Level schedules (rows of the head grouped by level, per direction) depend
// only on the neighbour sets and are built once.
#include <algorithm>
#include <cstdlib>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

constexpr int kHeadThreads = 1024;

// Workgroup-scope relaxed accesses to LDS: each read observes the latest
// value written by any wave of the workgroup.
__device__ __forceinline__ double lds_poll(double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------- level schedules
// Longest-path levels of the head rows K..H-1 by repeated relaxation in LDS
// (monotone, so it stops at the fixpoint): forward uses N(i), backward uses
// the rows of B^T restricted to head rows.  Rows below K are solved apart
// (a dense block) and count as known: they get level -1, and forward
// dependencies on them are dropped (backward rows K..H-1 only depend on
// later rows).
__global__ __launch_bounds__(kHeadThreads) void head_levels_kernel(
    int H, int K, int m, const int* __restrict__ nbr, const int* __restrict__ bt_ptr,
    const int* __restrict__ bt_col, int backward, int* __restrict__ level_out) {
  extern __shared__ int s_lev[];
  for (int i = threadIdx.x; i < H; i += kHeadThreads) s_lev[i] = 0;
  __syncthreads();
  for (;;) {
    int changed = 0;
    for (int i = K + threadIdx.x; i < H; i += kHeadThreads) {
      int l = 0;
      if (!backward) {
        for (int k = 0; k < m; ++k) {
          const int j = nbr[(int64_t)i * m + k];
          if (j < 0) break;
          if (j >= K) l = max(l, s_lev[j] + 1);
        }
      } else {
        const int b = bt_ptr[i], e = bt_ptr[i + 1];
        for (int q = b; q < e; ++q) {
          const int j = bt_col[q];
          if (j >= H) break;  // entries sorted ascending; tail rows are not head deps
          l = max(l, s_lev[j] + 1);
        }
      }
      if (l > s_lev[i]) {
        s_lev[i] = l;
        changed = 1;
      }
    }
    if (!__syncthreads_or(changed)) break;
  }
  for (int i = threadIdx.x; i < H; i += kHeadThreads) level_out[i] = i < K ? -1 : s_lev[i];
}

// Counting sort of head rows by level: ptr[L] = first position of level L;
// rows with level -1 get no position.
__global__ __launch_bounds__(kHeadThreads) void head_sort_kernel(int H,
                                                                  const int* __restrict__ level,
                                                                  int* __restrict__ ptr,
                                                                  int* __restrict__ rows,
                                                                  int* __restrict__ nlev_out) {
  extern __shared__ int s_cnt[];  // H + 1 counters
  for (int i = threadIdx.x; i <= H; i += kHeadThreads) s_cnt[i] = 0;
  __syncthreads();
  int mx = 0;
  int any = 0;
  for (int i = threadIdx.x; i < H; i += kHeadThreads) {
    const int l = level[i];
    if (l < 0) continue;
    atomicAdd(&s_cnt[l], 1);
    mx = max(mx, l);
    any = 1;
  }
  __shared__ int s_max;
  if (threadIdx.x == 0) s_max = -1;
  __syncthreads();
  if (any) atomicMax(&s_max, mx);
  __syncthreads();
  const int nlev = s_max + 1;
  if (threadIdx.x == 0) {
    int run = 0;
    for (int l = 0; l < nlev; ++l) {
      const int c = s_cnt[l];
      ptr[l] = run;
      s_cnt[l] = run;
      run += c;
    }
    ptr[nlev] = run;
    *nlev_out = nlev;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H; i += kHeadThreads) {
    if (level[i] < 0) continue;
    const int pos = atomicAdd(&s_cnt[level[i]], 1);
    rows[pos] = i;
  }
}

// ------------------------------------------------------------ head solves

// Upper: the right-hand side of head row j arrives in Y already reduced by its
// tail dependents (head_upper_pre).  The head rows are cut into index ranges
// [H/4, H), [H/16, H/4), ... (the earliest points of the ordering are
// neighbours of very many later points, so their B^T rows are long); the
// ranges are solved one after another, latest first.  For a range, each B^T
// row first subtracts its entries that point into ranges already solved
// (all final: a fully parallel phase over the range's rows), then the rows
// are solved in level order polling LDS, over the entries inside the range,
// which are few.  Entries are stored per position in descending child
// index, so the entries into solved ranges are a prefix ([pptr, split)) and
// the in-range ones follow ([split, pptr + 1)), their first kWin also in the
// padded wcol/wval.  In-range rows with at most 2 kWin entries are solved by
// one lane in windows of kWin; longer ones (only in the first range) by the
// whole wave in passes of 64 kCoop entries, combined by a fixed butterfly.
struct HeadRanges {
  int n;
  int start[10];  // positions [start[k], start[k + 1]) hold range k
};

template <int NT, typename TY = double>
__global__ __launch_bounds__(NT) void head_upper_kernel(
    int H, int K, int t, HeadRanges R, const int* __restrict__ prow, const int* __restrict__ pptr,
    const int* __restrict__ psplit, const int* __restrict__ pcol,
    const double* __restrict__ pval, const int* __restrict__ wcol,
    const double* __restrict__ wval, TY* Y) {
  extern __shared__ double s_y[];
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  constexpr int kWaves = NT / 64;
  constexpr int kWin = 16;
  constexpr int kCoop = 4;
  constexpr int kPass = 64 * kCoop;
  for (int i = tid; i < H; i += NT) s_y[i] = sentinel();
  __syncthreads();
  for (int r = 0; r < R.n; ++r) {
    const int p0 = R.start[r], p1 = R.start[r + 1];
    // entries into solved ranges: all final, fully parallel
    if (r > 0) {
      for (int p = p0 + tid; p < p1; p += NT) {
        const int j = prow[p];
        double acc = static_cast<double>(Y[(int64_t)j * t + c]);
        const int e = psplit[p];
        for (int q = pptr[p]; q < e; q += 8) {
          int cb[8];
          double vb[8], yv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            cb[k] = (q + k < e) ? pcol[q + k] : -1;
            vb[k] = (q + k < e) ? pval[q + k] : 0.0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) yv[k] = cb[k] >= 0 ? s_y[cb[k]] : 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k) acc -= vb[k] * yv[k];
        }
        Y[(int64_t)j * t + c] = static_cast<TY>(acc);
      }
      __syncthreads();  // the folded right-hand sides are visible to the block
    }
    int a_row = -1, a_q = 0, a_e = 0;          // stage A: two batches ahead
    int nrow = -1, nq = 0, ne = 0, ncb[kWin];   // stage B: one batch ahead
    double nvb[kWin], nacc = 0.0;
    auto stage_a = [&](int p) {
      const bool in = p < p1;
      a_row = in ? prow[p] : -1;
      a_q = in ? psplit[p] : 0;
      a_e = in ? pptr[p + 1] : 0;
    };
    auto stage_b = [&](int p) {
      const bool in = p < p1;
      nrow = a_row;
      nq = a_q;
      ne = a_e;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        ncb[k] = in ? wcol[(int64_t)p * kWin + k] : -1;
        nvb[k] = in ? wval[(int64_t)p * kWin + k] : 0.0;
      }
      nacc = (nrow >= 0) ? static_cast<double>(Y[(int64_t)nrow * t + c]) : 0.0;
    };
    int batch = tid >> 6;
    stage_a(p0 + batch * 64 + lane);
    stage_b(p0 + batch * 64 + lane);
    stage_a(p0 + (batch + kWaves) * 64 + lane);
    int cb[kWin];
    double vb[kWin];
    while (p0 + batch * 64 < p1) {
      const int j = nrow;
      int q = nq;
      const int e = ne;
#pragma unroll
      for (int k = 0; k < kWin; ++k) {
        cb[k] = ncb[k];
        vb[k] = nvb[k];
      }
      double acc = nacc;
      stage_b(p0 + (batch + kWaves) * 64 + lane);
      stage_a(p0 + (batch + 2 * kWaves) * 64 + lane);
      const bool is_long = j >= 0 && e - q > 2 * kWin;
      bool pending = j >= 0 && !is_long;
      uint64_t long_mask = __ballot(is_long);
      int kk = 0;
      while (__any(pending) || long_mask) {
        if (pending) {
          if (kk == kWin) {  // second window of a row
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
              const bool in = q + k < e;
              cb[k] = in ? pcol[q + k] : -1;
              vb[k] = in ? pval[q + k] : 0.0;
            }
            kk = 0;
          }
          double lv[kWin];
#pragma unroll
          for (int k = 0; k < kWin; ++k)
            lv[k] = (k >= kk && cb[k] >= 0) ? lds_poll(&s_y[cb[k]]) : 0.0;
          kk = consume_ready<kWin>(cb, vb, lv, kk, acc);
          if (kk == kWin) {
            if (q + kWin >= e) {
              lds_publish(&s_y[j], acc);
              pending = false;
            } else {
              q += kWin;  // the next round loads the next window
            }
          }
        }
        if (long_mask) {  // the wave's first unfinished long row, pass by pass
          const int owner = __builtin_ctzll(long_mask);
          const int lq = __shfl(q, owner), le = __shfl(e, owner);
          double part = 0.0;
          bool ready = true;
          for (int pos = lq; pos < le && ready; pos += kPass) {
            int xb[kCoop];
            double xv[kCoop], lv[kCoop];
#pragma unroll
            for (int k = 0; k < kCoop; ++k) {
              const int qq = pos + lane + 64 * k;
              xb[k] = qq < le ? pcol[qq] : -1;
              xv[k] = qq < le ? pval[qq] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kCoop; ++k) {
              lv[k] = xb[k] >= 0 ? lds_poll(&s_y[xb[k]]) : 0.0;
              if (xb[k] >= 0 && is_sentinel(lv[k])) ready = false;
            }
            ready = __all(ready);
            if (ready) {
#pragma unroll
              for (int k = 0; k < kCoop; ++k) part += xv[k] * lv[k];
            }
          }
          if (ready) {
            double sum = part;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) sum += __shfl_xor(sum, o);
            if (lane == owner) {
              acc -= sum;
              lds_publish(&s_y[j], acc);
            }
            long_mask &= long_mask - 1;
          }
        }
      }
      batch += kWaves;
    }
    __syncthreads();  // the range is solved before the next one folds it in
  }
  // rows below K are solved afterwards (the dense block) from Y's folded values
  for (int i = K + tid; i < H; i += NT) Y[(int64_t)i * t + c] = static_cast<TY>(s_y[i]);
}

// y_j <- x_j - sum over the tail entries of the B^T row of head row j (all
// finished), for every head row and column; fully parallel.
template <typename TY = double>
__global__ void head_upper_pre_kernel(int H, int t, const int* __restrict__ split,
                                      const int* __restrict__ bt_ptr,
                                      const int* __restrict__ bt_col,
                                      const double* __restrict__ bt_val,
                                      const double* __restrict__ X, TY* Y) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)H * t) return;
  const int j = static_cast<int>(g / t), c = static_cast<int>(g % t);
  double acc = X[(int64_t)j * t + c];
  const int e = bt_ptr[j + 1];
  for (int q = split[j]; q < e; ++q)
    acc -= bt_val[q] * static_cast<double>(Y[(int64_t)bt_col[q] * t + c]);
  Y[(int64_t)j * t + c] = static_cast<TY>(acc);
}

Status head_upper(Model& M, const double* X, double* Y, int t) {
  const int H = M.head_rows;
  if (H == 0) return Status::ok();
  const int K = M.dense_rows, P = M.head_pos;
  const int64_t work = (int64_t)H * t;
  hipLaunchKernelGGL(head_upper_pre_kernel<double>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                     M.stream, H, t, M.head_split.p, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, Y);
  if (P > 0) {
    const size_t lds = sizeof(double) * H;
    TimedLaunch tl(M, kTimeHeadUpper, 12.0 * M.head_nnz_b + 4.0 * H + 16.0 * H * t);
    HeadRanges R{};
    R.n = static_cast<int>(M.hb_blocks.size()) - 1;
    for (int k = 0; k <= R.n; ++k) R.start[k] = M.hb_blocks[k];
    hipLaunchKernelGGL(head_upper_kernel<512>, dim3(t), dim3(512), lds, M.stream, H, K, t, R,
                       M.hb_rows.p, M.hb_pptr.p, M.hb_split.p, M.hb_col.p, M.hb_val.p,
                       M.hb_wcol.p, M.hb_wval.p, Y);
    VL_TRY(check_launch("head upper"));
  }
  if (K > 0) VL_TRY(dense_upper(M, Y, t));  // rows 0..K-1, after every later row
  return check_launch("head upper");
}

// FP32-storage forms of the head solves for the mixed-precision narrow
// blocks: the same kernels with FP32 right-hand sides / results (LDS and
// every sum stay FP64).
Status head_upper_f32(Model& M, const double* X, float* Y, int t) {
  const int H = M.head_rows;
  if (H == 0) return Status::ok();
  const int K = M.dense_rows, P = M.head_pos;
  const int64_t work = (int64_t)H * t;
  hipLaunchKernelGGL(head_upper_pre_kernel<float>, dim3((unsigned)((work + 255) / 256)), dim3(256),
                     0, M.stream, H, t, M.head_split.p, M.bt_ptr.p, M.bt_col.p, M.bt_val.p, X, Y);
  if (P > 0) {
    const size_t lds = sizeof(double) * H;
    TimedLaunch tl(M, kTimeHeadUpper, 12.0 * M.head_nnz_b + 4.0 * H + 8.0 * H * t);
    HeadRanges R{};
    R.n = static_cast<int>(M.hb_blocks.size()) - 1;
    for (int k = 0; k <= R.n; ++k) R.start[k] = M.hb_blocks[k];
    hipLaunchKernelGGL((head_upper_kernel<512, float>), dim3(t), dim3(512), lds, M.stream, H, K,
                       t, R, M.hb_rows.p, M.hb_pptr.p, M.hb_split.p, M.hb_col.p, M.hb_val.p,
                       M.hb_wcol.p, M.hb_wval.p, Y);
    VL_TRY(check_launch("head upper f32"));
  }
  if (K > 0) VL_TRY(dense_upper_f32(M, Y, t));
  return check_launch("head upper f32");
}

// ---- position-ordered copies of the head's rows of B^T

// Rows of B^T are sorted by column, so a head row's head-internal entries
// (columns < H) form a prefix; split[j] is where its tail entries begin.
// Lengths are taken for the P positions; split (optional) is written for
// their rows.
__global__ void head_len_bwd_kernel(int H, int P, const int* __restrict__ prow,
                                    const int* __restrict__ bt_ptr,
                                    const int* __restrict__ bt_col, int* __restrict__ len,
                                    int* __restrict__ split) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) {
    const int j = prow[p];
    int q = bt_ptr[j];
    const int e = bt_ptr[j + 1];
    while (q < e && bt_col[q] < H) ++q;
    len[p] = q - bt_ptr[j];
    if (split) split[j] = q;
  }
  if (p == P) len[p] = 0;
}

__global__ void head_copy_bwd_kernel(int H, const int* __restrict__ prow,
                                     const int* __restrict__ bt_ptr,
                                     const int* __restrict__ bt_col,
                                     const int* __restrict__ bt_src,
                                     const int* __restrict__ pptr, int* __restrict__ pcol,
                                     int* __restrict__ psrc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H) return;
  const int j = prow[p];
  const int b = bt_ptr[j], e = b + (pptr[p + 1] - pptr[p]), o = pptr[p];
  // descending child index: the children that finish first (the latest
  // points) come first, so a row's later windows are loaded while it still
  // waits for its last children
  for (int q = b; q < e; ++q) {
    pcol[o + (e - 1 - q)] = bt_col[q];
    psrc[o + (e - 1 - q)] = bt_src[q];
  }
}

__global__ void head_vals_kernel(const double* __restrict__ bval, int nb,
                                 const int* __restrict__ psrc, double* __restrict__ pval_b) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nb) pval_b[e] = bval[psrc[e]];
}

// First kWin entries of every position of the B^T head rows, padded with -1
// (columns) and 0 (values), so that a batch's first windows load without
// waiting for the row pointers.
__global__ void head_window_kernel(int H, const int* __restrict__ pptr,
                                   const int* __restrict__ psplit,
                                   const int* __restrict__ pcol, const double* __restrict__ pval,
                                   int* __restrict__ wcol, double* __restrict__ wval) {
  constexpr int kWin = 16;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)H * kWin) return;
  const int p = static_cast<int>(g / kWin), k = static_cast<int>(g % kWin);
  const int q = psplit[p] + k;
  const bool in = q < pptr[p + 1];
  if (wcol) wcol[g] = in ? pcol[q] : -1;
  wval[g] = in ? pval[q] : 0.0;
}

Status refresh_head_values(Model& M) {
  const int P = M.head_pos;
  if (M.head_rows == 0 || P == 0) return Status::ok();
  const int64_t work = M.head_nnz_b;
  if (work == 0) return Status::ok();
  hipLaunchKernelGGL(head_vals_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0,
                     M.stream, M.bval.p, static_cast<int>(M.head_nnz_b), M.hb_src.p, M.hb_val.p);
  hipLaunchKernelGGL(head_window_kernel, dim3((unsigned)(((int64_t)P * 16 + 255) / 256)),
                     dim3(256), 0, M.stream, P, M.hb_pptr.p, M.hb_split.p, M.hb_col.p,
                     M.hb_val.p, nullptr, M.hb_wval.p);
  return check_launch("head values");
}

template <class K>
static void allow_lds(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  (void)hipGetLastError();
}

// Reorder the P backward head positions by index range of their rows
// (latest range first, level order kept inside a range) and record, per
// position, where the entries into the row's own range start.  Runs on the
// host (H <= kHeadRows).
static Status order_head_ranges(Model& M, int H, int P, int nnzb) {
  std::vector<int> rows(P > 0 ? P : 1), ptr(P + 1), col(nnzb > 0 ? nnzb : 1),
      src(nnzb > 0 ? nnzb : 1);
  VL_HIP(hipMemcpyAsync(rows.data(), M.hb_rows.p, sizeof(int) * P, hipMemcpyDeviceToHost,
                        M.stream));
  VL_HIP(hipMemcpyAsync(ptr.data(), M.hb_pptr.p, sizeof(int) * (P + 1), hipMemcpyDeviceToHost,
                        M.stream));
  if (nnzb > 0) {
    VL_HIP(hipMemcpyAsync(col.data(), M.hb_col.p, sizeof(int) * nnzb, hipMemcpyDeviceToHost,
                          M.stream));
    VL_HIP(hipMemcpyAsync(src.data(), M.hb_src.p, sizeof(int) * nnzb, hipMemcpyDeviceToHost,
                          M.stream));
  }
  VL_TRY(sync_stream(M.stream));
  // range bounds H > H/4 > H/16 > ... (the last range starts at 0)
  std::vector<int> lo;
  for (int b = H / 4; b >= 256; b /= 4) lo.push_back(b);
  lo.push_back(0);
  std::vector<int> nrows, nptr(1, 0), ncol, nsrc, nsplit, blocks(1, 0);
  nrows.reserve(P);
  nsplit.reserve(P);
  ncol.reserve(nnzb);
  nsrc.reserve(nnzb);
  int hi = H;
  for (int b : lo) {
    for (int p = 0; p < P; ++p) {
      const int j = rows[p];
      if (j < b || j >= hi) continue;
      nrows.push_back(j);
      int split = nptr.back();
      for (int q = ptr[p]; q < ptr[p + 1]; ++q) {
        ncol.push_back(col[q]);
        nsrc.push_back(src[q]);
        if (col[q] >= hi) ++split;  // descending: entries into solved ranges first
      }
      nsplit.push_back(split);
      nptr.push_back(static_cast<int>(ncol.size()));
    }
    blocks.push_back(static_cast<int>(nrows.size()));
    hi = b;
  }
  if (static_cast<int>(nrows.size()) != P || static_cast<int>(ncol.size()) != nnzb ||
      blocks.size() > 10)
    return Status::make(VL_ERR_STATE, "head range reordering failed");
  M.hb_blocks = blocks;
  VL_TRY(M.hb_split.alloc(P > 0 ? P : 1));
  if (P > 0) {
    VL_HIP(hipMemcpyAsync(M.hb_rows.p, nrows.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                          M.stream));
    VL_HIP(hipMemcpyAsync(M.hb_split.p, nsplit.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                          M.stream));
  }
  VL_HIP(hipMemcpyAsync(M.hb_pptr.p, nptr.data(), sizeof(int) * (P + 1), hipMemcpyHostToDevice,
                        M.stream));
  if (nnzb > 0) {
    VL_HIP(hipMemcpyAsync(M.hb_col.p, ncol.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice,
                          M.stream));
    VL_HIP(hipMemcpyAsync(M.hb_src.p, nsrc.data(), sizeof(int) * nnzb, hipMemcpyHostToDevice,
                          M.stream));
  }
  return sync_stream(M.stream);
}

// Level order (by head-internal levels with rows below K known) of the head
// rows K..H-1 in one direction: ptr (level pointers) and rows; returns the
// number of levels.
static Status head_order(Model& M, int H, int K, int dir, int* ptr, int* rows, int* nlev) {
  DevBuf<int> lev, dn;
  VL_TRY(lev.alloc(H));
  VL_TRY(dn.alloc(1));
  const size_t lds = sizeof(int) * (H + 1);
  hipLaunchKernelGGL(head_levels_kernel, dim3(1), dim3(kHeadThreads), lds, M.stream, H, K, M.m,
                     M.nbr.p, M.bt_ptr.p, M.bt_col.p, dir, lev.p);
  hipLaunchKernelGGL(head_sort_kernel, dim3(1), dim3(kHeadThreads), lds, M.stream, H, lev.p, ptr,
                     rows, dn.p);
  VL_TRY(check_launch("head schedule"));
  VL_HIP(hipMemcpyAsync(nlev, dn.p, sizeof(int), hipMemcpyDeviceToHost, M.stream));
  return sync_stream(M.stream);  // temporaries are released on return
}

Status build_head_schedule(Model& M) {
  int max_lds = 0;
  VL_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, M.device));
  int64_t cap = (static_cast<int64_t>(max_lds) - 1024) / static_cast<int64_t>(sizeof(double));
  int64_t want = kHeadRows;
  if (const char* env = std::getenv("VL_HEAD_ROWS")) want = std::atoll(env);  // tuning knob
  if (want < 0) want = 0;
  if (cap > want) cap = want;
  if (cap < 0) cap = 0;
  int64_t H = M.n < cap ? M.n : cap;
  // the kernels' LDS limit is a property of the kernel, shared by every model
  // in the process: always raise it to the largest head, so that a model
  // built later with a smaller head never lowers it under another's launches
  const size_t bytes = sizeof(double) * static_cast<size_t>(cap);
  allow_lds(head_upper_kernel<512>, bytes);
  M.head_rows = static_cast<int>(H);
  if (M.dense_rows > H) M.dense_rows = static_cast<int>(H);
  const int K = M.dense_rows;
  M.head_pos = static_cast<int>(H) - K;
  const int P = M.head_pos;
  if (H == 0) return Status::ok();
  const int m = M.m;
  // ---- the level-scheduled B^T solves (wide blocks): all head rows by their
  // head-internal levels, and where each head row's tail entries begin
  {
    DevBuf<int> ptr, rows, len, pptr;
    VL_TRY(ptr.alloc(H + 1));
    VL_TRY(rows.alloc(H));
    int nl = 0;
    VL_TRY(head_order(M, static_cast<int>(H), 0, 1, ptr.p, rows.p, &nl));
    VL_TRY(len.alloc(H + 1));
    VL_TRY(pptr.alloc(H + 1));
    VL_TRY(M.head_split.alloc(H));
    hipLaunchKernelGGL(head_len_bwd_kernel, dim3((unsigned)((H + 256) / 256)), dim3(256), 0,
                       M.stream, static_cast<int>(H), static_cast<int>(H), rows.p, M.bt_ptr.p,
                       M.bt_col.p, len.p, M.head_split.p);
    VL_TRY(exclusive_scan_int(len.p, pptr.p, H + 1, M.stream));
    VL_TRY(M.hlv_rows_b.alloc(H));
    VL_TRY(copy_d2d(M.hlv_rows_b.p, rows.p, sizeof(int) * H, M.stream));
    std::vector<int> lp(nl + 1), pp(H + 1);
    VL_HIP(hipMemcpyAsync(lp.data(), ptr.p, sizeof(int) * lp.size(), hipMemcpyDeviceToHost,
                          M.stream));
    VL_HIP(hipMemcpyAsync(pp.data(), pptr.p, sizeof(int) * (H + 1), hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
    M.hlv_ptr_b = lp;
    M.hlv_nnz_b.assign(nl, 0);
    for (int l = 0; l < nl; ++l) M.hlv_nnz_b[l] = pp[lp[l + 1]] - pp[lp[l]];
    int bt_head = 0;
    VL_HIP(hipMemcpyAsync(&bt_head, M.bt_ptr.p + H, sizeof(int), hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
    M.nnz_head_bt = bt_head;
    M.fold_nnz = static_cast<int64_t>(bt_head) - pp[H];
  }
  // ---- the wide B^T solves with the dense leading rows: head rows Kw..H-1
  // by their head-internal levels
  M.dense_wide = std::min<int>(K, kDenseWide);
  if (M.dense_wide > 0 && M.dense_wide < H) {
    const int Kw = M.dense_wide;
    DevBuf<int> ptr, len, pptr;
    VL_TRY(ptr.alloc(H + 1));
    VL_TRY(M.dhlv_rows_b.alloc(H));
    int nl = 0;
    VL_TRY(head_order(M, static_cast<int>(H), Kw, 1, ptr.p, M.dhlv_rows_b.p, &nl));
    const int Pw = static_cast<int>(H) - Kw;
    VL_TRY(len.alloc(Pw + 1));
    VL_TRY(pptr.alloc(Pw + 1));
    hipLaunchKernelGGL(head_len_bwd_kernel, dim3((unsigned)((Pw + 256) / 256)), dim3(256), 0,
                       M.stream, static_cast<int>(H), Pw, M.dhlv_rows_b.p, M.bt_ptr.p,
                       M.bt_col.p, len.p, nullptr);
    VL_TRY(exclusive_scan_int(len.p, pptr.p, Pw + 1, M.stream));
    std::vector<int> lp(nl + 1), pp(Pw + 1);
    VL_HIP(hipMemcpyAsync(lp.data(), ptr.p, sizeof(int) * lp.size(), hipMemcpyDeviceToHost,
                          M.stream));
    VL_HIP(hipMemcpyAsync(pp.data(), pptr.p, sizeof(int) * (Pw + 1), hipMemcpyDeviceToHost,
                          M.stream));
    VL_TRY(sync_stream(M.stream));
    M.dhlv_ptr_b = lp;
    M.dhlv_nnz_b.assign(nl, 0);
    for (int l = 0; l < nl; ++l) M.dhlv_nnz_b[l] = pp[lp[l + 1]] - pp[lp[l]];
  } else {
    M.dense_wide = 0;
  }
  // ---- the LDS head solve of B^T (t <= 64): rows K..H-1 in P positions
  VL_TRY(M.hb_ptr.alloc(H + 1));
  VL_TRY(M.hb_rows.alloc(H));
  VL_TRY(head_order(M, static_cast<int>(H), K, 1, M.hb_ptr.p, M.hb_rows.p, &M.head_nlev_b));
  // position-ordered copies (structure; values follow in refresh_head_values)
  DevBuf<int> len;
  VL_TRY(len.alloc(P + 1));
  VL_TRY(M.hb_pptr.alloc(P + 1));
  hipLaunchKernelGGL(head_len_bwd_kernel, dim3((unsigned)((P + 256) / 256)), dim3(256), 0,
                     M.stream, static_cast<int>(H), P, M.hb_rows.p, M.bt_ptr.p, M.bt_col.p,
                     len.p, nullptr);
  VL_TRY(exclusive_scan_int(len.p, M.hb_pptr.p, P + 1, M.stream));
  int nnzb = 0;
  VL_HIP(hipMemcpyAsync(&nnzb, M.hb_pptr.p + P, sizeof(int), hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  M.head_nnz_b = nnzb;
  VL_TRY(M.hb_col.alloc(nnzb));
  VL_TRY(M.hb_src.alloc(nnzb));
  VL_TRY(M.hb_val.alloc(nnzb));
  if (P > 0)
    hipLaunchKernelGGL(head_copy_bwd_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0,
                       M.stream, P, M.hb_rows.p, M.bt_ptr.p, M.bt_col.p, M.bt_src.p, M.hb_pptr.p,
                       M.hb_col.p, M.hb_src.p);
  VL_TRY(check_launch("head copies"));
  VL_TRY(order_head_ranges(M, static_cast<int>(H), P, nnzb));
  VL_TRY(M.hb_wcol.alloc((size_t)(P > 0 ? P : 1) * 16));
  VL_TRY(M.hb_wval.alloc((size_t)(P > 0 ? P : 1) * 16));
  if (P > 0)
    hipLaunchKernelGGL(head_window_kernel, dim3((unsigned)(((int64_t)P * 16 + 255) / 256)),
                       dim3(256), 0, M.stream, P, M.hb_pptr.p, M.hb_split.p, M.hb_col.p,
                       M.hb_val.p, M.hb_wcol.p, M.hb_wval.p);
  VL_TRY(check_launch("head copies"));
  VL_TRY(sync_stream(M.stream));
  return build_dense(M);
}

}  // namespace vl
