// Grouped products with B and B^T for blocks of 32 to 64 columns: the two
// sparse products of the operator W + B^T D^{-1} B (Sec. 3.1) inside the
// block PCG of the stochastic trace and log-determinant estimates (Sec. 3.2),
// whose probe blocks have this width.
//
// Rows are cut into groups of kGroupRows = 4 consecutive positions of the
// spatial order of the neighbour-search grid (Morton-numbered cells).  The
// rows of a group are close in space, so their neighbour sets overlap: at
// n = 1e5, m = 20 the union of the columns that a group touches holds 12.2
// columns per row for B and 13.2 for B^T, against 21 when every row gathers
// its own.  A wave computes one group over 64 columns.  It loads each union
// row of the operand once and accumulates it into every row of the group
// with the group's dense weight column (zero where a row does not touch the
// column), so an operand row crosses the L2 once per group instead of once
// per row.  The weights are uniform over the wave and are read as scalars.
// Measured at n = 1e5 this takes 87 / 111 us for B / B^T at 50 columns
// against 149 / 168 us row by row; at 256 columns and more the row-by-row
// wide kernels are faster (the dense weights cost 4 FMAs per useful one), and
// below 32 columns most lanes of a wave would idle.
//
// A group's union columns are sorted ascending, so each row sums its own
// entries (the unit diagonal included) in ascending column order, with exact
// zeros in between: the result does not depend on how rows are grouped.  A
// non-finite operand entry, multiplied by a zero weight, makes every row of
// its group non-finite.
#include <climits>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

constexpr int kGroupPad = 8;      // union lengths are padded to a multiple of this
constexpr int kGroupCand = 8192;  // candidate columns of one group (sorted in LDS)

// ------------------------------------------------------------ structure
__global__ void grp_inverse_kernel(int64_t n, const int* __restrict__ order,
                                   int* __restrict__ pos_of) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) pos_of[order[p]] = static_cast<int>(p);
}

// Number of stored neighbours of row i (they form a prefix of its slots).
__device__ __forceinline__ int ell_len(const int* __restrict__ nbr, int64_t i, int m) {
  int len = 0;
  while (len < m && nbr[i * m + len] >= 0) ++len;
  return len;
}

// Candidate counts per group: each row contributes itself and its entries.
__global__ void grp_count_kernel(int64_t n, int64_t ng, int m, const int* __restrict__ order,
                                 const int* __restrict__ nbr, const int* __restrict__ bt_ptr,
                                 int* __restrict__ kb, int* __restrict__ kt) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ng) return;
  int cb = 0, ct = 0;
  for (int r = 0; r < kGroupRows; ++r) {
    const int64_t p = g * kGroupRows + r;
    if (p >= n) break;
    const int64_t i = order[p];
    cb += 1 + ell_len(nbr, i, m);
    ct += 1 + bt_ptr[i + 1] - bt_ptr[i];
  }
  kb[g] = cb;
  kt[g] = ct;
}

// Sorted distinct columns of group g: the candidates go to LDS, a bitonic
// network sorts them, and wave 0 keeps the first of each run of equal
// values.  Writes them at cand[kptr[g]...] and their number to ucnt[g]; a
// group with more than kGroupCand candidates sets *err instead.
template <bool TRANS>
__global__ __launch_bounds__(256) void grp_union_kernel(
    int64_t n, int m, const int* __restrict__ order, const int* __restrict__ nbr,
    const int* __restrict__ bt_ptr, const int* __restrict__ bt_col, const int* __restrict__ kptr,
    int* __restrict__ cand, int* __restrict__ ucnt, int* __restrict__ err) {
  __shared__ int s[kGroupCand];
  __shared__ int s_off[kGroupRows + 1];
  const int64_t g = blockIdx.x;
  const int tid = threadIdx.x;
  const int K = kptr[g + 1] - kptr[g];
  if (K > kGroupCand) {
    if (tid == 0) {
      ucnt[g] = 0;
      atomicOr(err, 1);
    }
    return;
  }
  if (tid == 0) {
    int o = 0;
    for (int r = 0; r < kGroupRows; ++r) {
      s_off[r] = o;
      const int64_t p = g * kGroupRows + r;
      if (p < n) {
        const int64_t i = order[p];
        o += 1 + (TRANS ? bt_ptr[i + 1] - bt_ptr[i] : ell_len(nbr, i, m));
      }
    }
    s_off[kGroupRows] = o;
  }
  __syncthreads();
  if (s_off[kGroupRows] != K) {  // counts disagree with this pass: structure error
    if (tid == 0) {
      ucnt[g] = 0;
      atomicOr(err, 2);
    }
    return;
  }
  for (int r = 0; r < kGroupRows; ++r) {
    const int64_t p = g * kGroupRows + r;
    if (p >= n) break;
    const int64_t i = order[p];
    const int base = s_off[r];
    const int len = s_off[r + 1] - base;  // the row itself, then its entries
    for (int k = tid; k < len; k += 256) {
      int v;
      if (k == 0) {
        v = static_cast<int>(i);
      } else {
        v = TRANS ? bt_col[bt_ptr[i] + k - 1] : nbr[i * m + k - 1];
      }
      s[base + k] = v;
    }
  }
  int P = 2;
  while (P < K) P <<= 1;
  for (int k = K + tid; k < P; k += 256) s[k] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int q = tid; q < (P >> 1); q += 256) {
        const int a = 2 * q - (q & (stride - 1));
        const int b = a + stride;
        const bool up = (a & size) == 0;
        const int va = s[a], vb = s[b];
        if ((va > vb) == up) {
          s[a] = vb;
          s[b] = va;
        }
      }
      __syncthreads();
    }
  }
  if (tid < 64) {
    const int lane = tid;
    int cnt = 0;
    for (int base = 0; base < K; base += 64) {
      const int k = base + lane;
      const bool keep = k < K && (k == 0 || s[k] != s[k - 1]);
      const uint64_t mask = __ballot(keep);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      if (keep) cand[kptr[g] + cnt + before] = s[k];
      cnt += __popcll(mask);
    }
    if (lane == 0) ucnt[g] = cnt;
  }
}

__global__ void grp_pad_kernel(int64_t ng, const int* __restrict__ ucnt, int* __restrict__ upad) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < ng) upad[g] = (ucnt[g] + kGroupPad - 1) / kGroupPad * kGroupPad;
}

// Union columns at their padded offsets; padding repeats the last column
// (its weights stay zero).
__global__ void grp_place_kernel(const int* __restrict__ kptr, const int* __restrict__ cand,
                                 const int* __restrict__ ucnt, const int* __restrict__ uptr,
                                 int* __restrict__ ucol) {
  const int64_t g = blockIdx.x;
  const int cnt = ucnt[g];
  const int base = uptr[g], len = uptr[g + 1] - base;
  for (int k = threadIdx.x; k < len; k += blockDim.x)
    ucol[base + k] = cand[kptr[g] + (k < cnt ? k : cnt - 1)];
}

__device__ __forceinline__ int lower_bound_int(const int* __restrict__ a, int len, int v) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v) {
      lo = mid + 1;
    } else {
      hi = mid;
    }
  }
  return lo;
}

// Index into a group matrix of (row at position p, column j); -1 when j is
// not in the group's union (a structure error).
__device__ __forceinline__ int64_t grp_index(int p, int j, const int* __restrict__ uptr,
                                             const int* __restrict__ ucol,
                                             const int* __restrict__ ucnt) {
  const int g = p / kGroupRows, r = p - g * kGroupRows;
  const int base = uptr[g], cnt = ucnt[g];
  const int u = lower_bound_int(ucol + base, cnt, j);
  if (u >= cnt || ucol[base + u] != j) return -1;
  return static_cast<int64_t>(base + u) * kGroupRows + r;
}

// Entry (i, k) of B (column j = nbr[i, k]) sits in row i of B's group matrix
// and in row j, column i of B^T's.
__global__ void grp_pos_kernel(int64_t n, int m, const int* __restrict__ nbr,
                               const int* __restrict__ pos_of, const int* __restrict__ bptr,
                               const int* __restrict__ bcol, const int* __restrict__ bcnt,
                               const int* __restrict__ tptr, const int* __restrict__ tcol,
                               const int* __restrict__ tcnt, int* __restrict__ posb,
                               int* __restrict__ post, int* __restrict__ err) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m;
  const int j = nbr[e];
  if (j < 0) {
    posb[e] = -1;
    post[e] = -1;
    return;
  }
  const int64_t qb = grp_index(pos_of[i], j, bptr, bcol, bcnt);
  const int64_t qt = grp_index(pos_of[j], static_cast<int>(i), tptr, tcol, tcnt);
  if (qb < 0 || qt < 0) {
    atomicOr(err, 4);
    posb[e] = -1;
    post[e] = -1;
    return;
  }
  posb[e] = static_cast<int>(qb);
  post[e] = static_cast<int>(qt);
}

// The unit diagonal of both matrices (written once; values refreshes never
// touch these positions).
__global__ void grp_diag_kernel(int64_t n, const int* __restrict__ pos_of,
                                const int* __restrict__ bptr, const int* __restrict__ bcol,
                                const int* __restrict__ bcnt, const int* __restrict__ tptr,
                                const int* __restrict__ tcol, const int* __restrict__ tcnt,
                                double* __restrict__ wb, double* __restrict__ wt,
                                int* __restrict__ err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = pos_of[i];
  const int64_t qb = grp_index(p, static_cast<int>(i), bptr, bcol, bcnt);
  const int64_t qt = grp_index(p, static_cast<int>(i), tptr, tcol, tcnt);
  if (qb < 0 || qt < 0) {
    atomicOr(err, 8);
    return;
  }
  wb[qb] = 1.0;
  wt[qt] = 1.0;
}

__global__ void grp_refresh_kernel(int64_t nm, const int* __restrict__ posb,
                                   const int* __restrict__ post, const double* __restrict__ bval,
                                   double* __restrict__ wb, double* __restrict__ wt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= nm) return;
  const int pb = posb[e];
  if (pb < 0) return;
  const double v = bval[e];
  wb[pb] = v;
  wt[post[e]] = v;
}

static unsigned blocks_of(int64_t count, int tb) {
  return static_cast<unsigned>((count + tb - 1) / tb);
}

// Union of one matrix: counts `k` (ng + 1 entries, last one zero) ->
// op.ptr / op.col / op.cnt; returns the error flags in *err_host.
static Status build_union(Model& M, bool trans, int* k, int* err, GroupOp& op) {
  hipStream_t s = M.stream;
  const int64_t ng = M.grp_count;
  DevBuf<int> kptr, cand, upad;
  VL_TRY(kptr.alloc(ng + 1));
  VL_TRY(exclusive_scan_int(k, kptr.p, ng + 1, s));
  int total = 0;
  VL_HIP(hipMemcpyAsync(&total, kptr.p + ng, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  VL_TRY(cand.alloc(total));
  VL_TRY(op.cnt.alloc(ng));
  const int* nbr = M.nbr.p;
  if (trans) {
    hipLaunchKernelGGL(grp_union_kernel<true>, dim3(static_cast<unsigned>(ng)), dim3(256), 0, s,
                       M.n, M.m, static_cast<const int*>(M.grid_pts), nbr, M.bt_ptr.p,
                       M.bt_col.p, kptr.p, cand.p, op.cnt.p, err);
  } else {
    hipLaunchKernelGGL(grp_union_kernel<false>, dim3(static_cast<unsigned>(ng)), dim3(256), 0, s,
                       M.n, M.m, static_cast<const int*>(M.grid_pts), nbr, M.bt_ptr.p,
                       M.bt_col.p, kptr.p, cand.p, op.cnt.p, err);
  }
  VL_TRY(upad.alloc(ng + 1));
  VL_TRY(fill_int(upad.p + ng, 0, 1, s));
  hipLaunchKernelGGL(grp_pad_kernel, dim3(blocks_of(ng, 256)), dim3(256), 0, s, ng, op.cnt.p,
                     upad.p);
  VL_TRY(op.ptr.alloc(ng + 1));
  VL_TRY(exclusive_scan_int(upad.p, op.ptr.p, ng + 1, s));
  int ucols = 0;
  VL_HIP(hipMemcpyAsync(&ucols, op.ptr.p + ng, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  op.cols = ucols;
  VL_TRY(op.col.alloc(ucols));
  hipLaunchKernelGGL(grp_place_kernel, dim3(static_cast<unsigned>(ng)), dim3(64), 0, s, kptr.p,
                     cand.p, op.cnt.p, op.ptr.p, op.col.p);
  VL_TRY(check_launch("group union"));
  return sync_stream(s);  // temporaries are released on return
}

Status build_groups(Model& M) {
  M.grp_ok = false;
  const int64_t n = M.n;
  if (M.m < 1 || n < 1) return Status::ok();
  const int64_t ng = (n + kGroupRows - 1) / kGroupRows;
  M.grp_count = ng;
  hipStream_t s = M.stream;
  const int* order = static_cast<const int*>(M.grid_pts);
  DevBuf<int> pos_of, kb, kt, err;
  VL_TRY(pos_of.alloc(n));
  VL_TRY(kb.alloc(ng + 1));
  VL_TRY(kt.alloc(ng + 1));
  VL_TRY(err.alloc(1));
  VL_TRY(fill_int(err.p, 0, 1, s));
  VL_TRY(fill_int(kb.p + ng, 0, 1, s));
  VL_TRY(fill_int(kt.p + ng, 0, 1, s));
  hipLaunchKernelGGL(grp_inverse_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, n, order,
                     pos_of.p);
  hipLaunchKernelGGL(grp_count_kernel, dim3(blocks_of(ng, 256)), dim3(256), 0, s, n, ng, M.m,
                     order, M.nbr.p, M.bt_ptr.p, kb.p, kt.p);
  VL_TRY(check_launch("group count"));
  VL_TRY(build_union(M, false, kb.p, err.p, M.grp_b));
  VL_TRY(build_union(M, true, kt.p, err.p, M.grp_bt));
  int e = 0;
  VL_HIP(hipMemcpyAsync(&e, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  if (e & 2) return Status::make(VL_ERR_STATE, "group structure: inconsistent counts");
  if (e & 1) {  // a group gathers too many columns: keep the per-row products
    M.grp_b.reset();
    M.grp_bt.reset();
    return Status::ok();
  }
  const int64_t nm = n * M.m;
  VL_TRY(M.grp_b.pos.alloc(nm));
  VL_TRY(M.grp_bt.pos.alloc(nm));
  VL_TRY(M.grp_b.w.alloc(static_cast<size_t>(M.grp_b.cols) * kGroupRows));
  VL_TRY(M.grp_bt.w.alloc(static_cast<size_t>(M.grp_bt.cols) * kGroupRows));
  VL_TRY(fill_double(M.grp_b.w.p, 0.0, static_cast<int64_t>(M.grp_b.cols) * kGroupRows, s));
  VL_TRY(fill_double(M.grp_bt.w.p, 0.0, static_cast<int64_t>(M.grp_bt.cols) * kGroupRows, s));
  hipLaunchKernelGGL(grp_pos_kernel, dim3(blocks_of(nm, 256)), dim3(256), 0, s, n, M.m,
                     M.nbr.p, pos_of.p, M.grp_b.ptr.p, M.grp_b.col.p, M.grp_b.cnt.p,
                     M.grp_bt.ptr.p, M.grp_bt.col.p, M.grp_bt.cnt.p, M.grp_b.pos.p,
                     M.grp_bt.pos.p, err.p);
  hipLaunchKernelGGL(grp_diag_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, s, n, pos_of.p,
                     M.grp_b.ptr.p, M.grp_b.col.p, M.grp_b.cnt.p, M.grp_bt.ptr.p,
                     M.grp_bt.col.p, M.grp_bt.cnt.p, M.grp_b.w.p, M.grp_bt.w.p, err.p);
  VL_TRY(check_launch("group positions"));
  VL_HIP(hipMemcpyAsync(&e, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  VL_TRY(sync_stream(s));
  if (e != 0) return Status::make(VL_ERR_STATE, "group structure: entry outside its union");
  M.grp_ok = true;
  return Status::ok();
}

Status refresh_group_values(Model& M) {
  if (!M.grp_ok) return Status::ok();
  const int64_t nm = M.n * M.m;
  hipLaunchKernelGGL(grp_refresh_kernel, dim3(blocks_of(nm, 256)), dim3(256), 0, M.stream, nm,
                     M.grp_b.pos.p, M.grp_bt.pos.p, M.bval.p, M.grp_b.w.p, M.grp_bt.w.p);
  return check_launch("group values");
}

// ------------------------------------------------------------- products
// Wave (g, s): rows g*G .. g*G+G-1 of the spatial order, column
// c = 64 s + lane.  acc[r] = sum over the union u of w[u][r] * X[col[u], c];
// then Y_i = rs_i acc[r] (ROWSCALE) or acc[r] + d_i V_i (DIAG).  Waves of a
// block take consecutive units (group-major).
template <bool ROWSCALE, bool DIAG>
__global__ __launch_bounds__(256) void spmm_group_kernel(
    int64_t n, int t, int64_t ng, int nslices, const int* __restrict__ order,
    const int* __restrict__ uptr, const int* __restrict__ ucol, const double* __restrict__ w,
    const double* __restrict__ X, const double* __restrict__ rs, const double* __restrict__ d,
    const double* __restrict__ V, double* __restrict__ Y) {
  constexpr int G = kGroupRows;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t unit = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
  if (unit >= ng * nslices) return;
  const int64_t g = unit / nslices;
  const int c = static_cast<int>(unit - g * nslices) * 64 + (threadIdx.x & 63);
  const bool act = c < t;
  const int u0 = uptr[g], u1 = uptr[g + 1];
  double acc[G];
#pragma unroll
  for (int r = 0; r < G; ++r) acc[r] = 0.0;
  // Union entries in chunks of KC, two chunks in flight: the gathers of the
  // next chunk are issued before the current one is accumulated.  Union
  // lengths are multiples of kGroupPad = 2 KC.
  constexpr int KC = kGroupPad / 2;
  double xa[KC], xb[KC];
  auto gather = [&](int u, double* x) {
#pragma unroll
    for (int k = 0; k < KC; ++k) x[k] = act ? X[static_cast<int64_t>(ucol[u + k]) * t + c] : 0.0;
  };
  auto accumulate = [&](int u, const double* x) {
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const double* wk = w + static_cast<int64_t>(u + k) * G;
#pragma unroll
      for (int r = 0; r < G; ++r) acc[r] = fma(wk[r], x[k], acc[r]);
    }
  };
  gather(u0, xa);
  for (int u = u0; u < u1; u += 2 * KC) {
    gather(u + KC, xb);
    accumulate(u, xa);
    if (u + 2 * KC < u1) gather(u + 2 * KC, xa);
    accumulate(u + KC, xb);
  }
  if (!act) return;
#pragma unroll
  for (int r = 0; r < G; ++r) {
    const int64_t p = g * G + r;
    if (p >= n) break;
    const int64_t i = order[p];
    double y = acc[r];
    if (ROWSCALE) y *= rs[i];
    if (DIAG) y += d[i] * V[i * t + c];
    Y[i * t + c] = y;
  }
}

bool group_spmm_ok(const Model& M, int t) {
  return M.grp_ok && t >= kGroupMinT && t <= kGroupMaxT;
}

template <bool ROWSCALE, bool DIAG>
static void launch_group(Model& M, const GroupOp& op, const double* X, double* Y, int t,
                         const double* rs, const double* d, const double* V) {
  const int nslices = (t + 63) / 64;
  const int64_t units = M.grp_count * nslices;
  hipLaunchKernelGGL((spmm_group_kernel<ROWSCALE, DIAG>), dim3(blocks_of(units, 4)), dim3(256), 0,
                     M.stream, M.n, t, M.grp_count, nslices,
                     static_cast<const int*>(M.grid_pts), op.ptr.p, op.col.p, op.w.p, X, rs, d,
                     V, Y);
}

Status spmm_group_b(Model& M, const double* X, double* Y, int t, const double* rs) {
  if (rs) {
    launch_group<true, false>(M, M.grp_b, X, Y, t, rs, nullptr, nullptr);
  } else {
    launch_group<false, false>(M, M.grp_b, X, Y, t, nullptr, nullptr, nullptr);
  }
  return check_launch("spmm_b grouped");
}

Status spmm_group_bt(Model& M, const double* X, double* Y, int t, const double* d,
                     const double* V) {
  if (d) {
    launch_group<false, true>(M, M.grp_bt, X, Y, t, nullptr, d, V);
  } else {
    launch_group<false, false>(M, M.grp_bt, X, Y, t, nullptr, nullptr, nullptr);
  }
  return check_launch("spmm_bt grouped");
}

}  // namespace vl
