// Head schedules of the wide (t > 64) backward solves with B^T.
//
// With a random ordering the dependency DAG of B is deep only among early
// rows: for n = 1e5, m = 20 the first 16384 rows already span 214 of the 278
// levels, while the remaining rows add only 68.  The first rows are solved
// with the dense inverse of B's leading block (dense.hip).  A wide B^T solve
// (sparse.hip) takes the tail rows >= H level by level, folds every head
// row's tail entries in one launch, then the head rows by their
// head-internal levels (K = 4096, H = 12288 by default), then the dense
// block.  This file builds those head-internal level schedules; they depend
// only on the neighbour sets and are built once.  Narrow blocks need no head
// schedule: the sync-free tail runs from the dense block in both directions.
#include <algorithm>
#include <cstdlib>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

constexpr int kHeadThreads = 1024;

// ------------------------------------------------------- level schedules
// Backward longest-path levels of the head rows K..H-1 by repeated
// relaxation in LDS (monotone, so it stops at the fixpoint), over the rows of
// B^T restricted to head rows (backward rows K..H-1 only depend on later
// rows).  Rows below K are solved apart (a dense block): they get level -1.
__global__ __launch_bounds__(kHeadThreads) void head_levels_kernel(
    int H, int K, const int* __restrict__ bt_ptr, const int* __restrict__ bt_col,
    int* __restrict__ level_out) {
  extern __shared__ int s_lev[];
  for (int i = threadIdx.x; i < H; i += kHeadThreads) s_lev[i] = 0;
  __syncthreads();
  for (;;) {
    int changed = 0;
    for (int i = K + threadIdx.x; i < H; i += kHeadThreads) {
      int l = 0;
      const int b = bt_ptr[i], e = bt_ptr[i + 1];
      for (int q = b; q < e; ++q) {
        const int j = bt_col[q];
        if (j >= H) break;  // entries sorted ascending; tail rows are not head deps
        l = max(l, s_lev[j] + 1);
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

// ---- where the head rows' tail entries begin

// Rows of B^T are sorted by column, so a head row's head-internal entries
// (columns < H) form a prefix; split[j] is where its tail entries begin.
// Lengths are taken for the P rows prow[0..P-1]; split (optional) is written
// for those rows.
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

template <class K>
static void allow_lds(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  (void)hipGetLastError();
}

// Backward level order (by head-internal levels with rows below K known) of
// the head rows K..H-1: ptr (level pointers) and rows; returns the number of
// levels.
static Status head_order(Model& M, int H, int K, int* ptr, int* rows, int* nlev) {
  DevBuf<int> lev, dn;
  VL_TRY(lev.alloc(H));
  VL_TRY(dn.alloc(1));
  const size_t lds = sizeof(int) * (H + 1);
  hipLaunchKernelGGL(head_levels_kernel, dim3(1), dim3(kHeadThreads), lds, M.stream, H, K,
                     M.bt_ptr.p, M.bt_col.p, lev.p);
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
  const size_t bytes = sizeof(int) * static_cast<size_t>(cap + 1);
  allow_lds(head_levels_kernel, bytes);
  allow_lds(head_sort_kernel, bytes);
  M.head_rows = static_cast<int>(H);
  if (M.dense_rows > H) M.dense_rows = static_cast<int>(H);
  const int K = M.dense_rows;
  if (H == 0) return Status::ok();
  // ---- the level-scheduled B^T solves (wide blocks): all head rows by their
  // head-internal levels, and where each head row's tail entries begin
  {
    DevBuf<int> ptr, rows, len, pptr;
    VL_TRY(ptr.alloc(H + 1));
    VL_TRY(rows.alloc(H));
    int nl = 0;
    VL_TRY(head_order(M, static_cast<int>(H), 0, ptr.p, rows.p, &nl));
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
    VL_TRY(head_order(M, static_cast<int>(H), Kw, ptr.p, M.dhlv_rows_b.p, &nl));
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
  return build_dense(M);
}

}  // namespace vl
