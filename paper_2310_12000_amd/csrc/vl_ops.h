// Work layouts shared by the kernels, and the operator interface of the CG
// driver.
#pragma once

#include <functional>
#include <vector>

#include "vl_internal.h"

namespace vl {

// Lanes of a wave over an n x t row-major block: lanes_per_row =
// min(64, next power of two >= t); a wave covers 64 / lanes_per_row rows;
// for t > 64 each row is split into 64-column slices.
struct Lanes {
  int lpr_log, rpw_log, slices;
  __host__ __device__ static Lanes of(int t) {
    Lanes L;
    if (t > 64) {
      L.lpr_log = 6;
      L.rpw_log = 0;
      L.slices = (t + 63) / 64;
    } else {
      int lg = 0;
      while ((1 << lg) < t) ++lg;
      L.lpr_log = lg;
      L.rpw_log = 6 - lg;
      L.slices = 1;
    }
    return L;
  }
};

// Work units = (row group of 2^rpw_log rows, slice).
__host__ __device__ __forceinline__ int64_t units_of_hd(int64_t n, int t, Lanes L) {
  (void)t;
  int64_t rg = (n + (1 << L.rpw_log) - 1) >> L.rpw_log;
  return rg * L.slices;
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip; remap so
// that each XCD works on one contiguous range of units (spatially ordered
// rows), keeping neighbour gathers inside that XCD's L2.
__host__ __device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  // XCD x = b mod 8 holds blocks x, x + 8, ...: count q + (x < rem); it gets
  // the contiguous range starting at x q + min(x, rem).  A bijection of [0, nb).
  const int64_t q = nb >> 3, rem = nb & 7;
  const int64_t x = b & 7, local = b >> 3;
  return x * q + (x < rem ? x : rem) + local;
}

// Work counters of the sync-free solves: one slot per concurrently prepared
// solve, each with kCounterStreams counters 64 bytes apart and an abort flag.
// Stream s is served by blocks s, s + S, ...; progress needs every stream to
// have a resident wave, so S must not exceed the number of blocks that are
// resident at once.  One 256-thread block of these kernels always fits on a
// CU, so S <= number of CUs (256 on MI355X) is safe.
constexpr int kCounterStreams = 256;
constexpr int kCounterStride = 16;
constexpr int kSlotInts = kCounterStreams * kCounterStride + 16;
constexpr int kAbortOffset = kCounterStreams * kCounterStride;

// Zero the counters and abort flags of both slots (one block calls it).
__device__ __forceinline__ void reset_counters(int* counter) {
  for (int k = threadIdx.x; k < 2 * kSlotInts; k += blockDim.x) counter[k] = 0;
}

// Deterministic chunked grid: gridDim = (nchunk, slices), 256 threads; block
// (k, s) covers rows [k * rpc, (k + 1) * rpc) and columns of slice s.
struct ChunkGrid {
  Lanes L;
  int64_t n;
  int t;
  int nchunk;
  int64_t rpc;
  static ChunkGrid of(int64_t n, int t);
};

// Loop over the (row i, column c) pairs of this lane within the block's chunk.
#define CHUNK_LOOP_BEGIN(g)                                                        \
  {                                                                                \
    const int _lane = threadIdx.x & 63;                                            \
    const int _w = threadIdx.x >> 6;                                               \
    const int _sub = _lane >> (g).L.lpr_log;                                       \
    const int c = blockIdx.y * 64 + (_lane & ((1 << (g).L.lpr_log) - 1));          \
    const int64_t _r0 = (int64_t)blockIdx.x * (g).rpc;                             \
    int64_t _r1 = _r0 + (g).rpc;                                                   \
    if (_r1 > (g).n) _r1 = (g).n;                                                  \
    const int64_t _step = 4LL << (g).L.rpw_log;                                    \
    if (c < (g).t) {                                                               \
      for (int64_t _b = _r0 + ((int64_t)_w << (g).L.rpw_log); _b < _r1; _b += _step) { \
        const int64_t i = _b + _sub;                                               \
        if (i >= _r1) continue;

#define CHUNK_LOOP_END \
  }                    \
  }                    \
  }

// Add a per-lane value over all rows of the block, per column, and store the
// block's column sums at part[blockIdx.x * t + column].  All threads of the
// block must call it.
__device__ __forceinline__ void block_colsum(const ChunkGrid& g, double v,
                                             double* __restrict__ part) {
  __shared__ double s[4][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int lpr = 1 << g.L.lpr_log;
  for (int o = 32; o >= lpr; o >>= 1) v += __shfl_xor(v, o);
  if (lane < lpr) s[w][lane] = v;
  __syncthreads();
  const int c = blockIdx.y * 64 + lane;
  if (w == 0 && lane < lpr && c < g.t)
    part[(int64_t)blockIdx.x * g.t + c] = s[0][lane] + s[1][lane] + s[2][lane] + s[3][lane];
  __syncthreads();
}

Status reduce_chunks(hipStream_t s, const double* part, int nchunk, int t, double* out);

// Row chunks given by a table (the batching form): block (k, s) covers rows
// [r0[k], r1[k]) of the problem prob[k] and columns of slice s, visited in
// the same lane pattern as CHUNK_LOOP.
struct SegArgs {
  Lanes L;
  int t;
  const int* prob;
  const int* r0;
  const int* r1;
};

// Rows (i, column c) of this lane in the block's chunk, in the same pattern
// as a solo run's chunk (so sums come out in the same order).
#define SEG_LOOP_BEGIN(a)                                                            \
  {                                                                                  \
    const int _lane = threadIdx.x & 63;                                              \
    const int _w = threadIdx.x >> 6;                                                 \
    const int _sub = _lane >> (a).L.lpr_log;                                         \
    const int c = blockIdx.y * 64 + (_lane & ((1 << (a).L.lpr_log) - 1));            \
    const int64_t _r0 = (a).r0[blockIdx.x];                                          \
    const int64_t _r1 = (a).r1[blockIdx.x];                                          \
    const int64_t _step = 4LL << (a).L.rpw_log;                                      \
    if (c < (a).t) {                                                                 \
      for (int64_t _b = _r0 + ((int64_t)_w << (a).L.rpw_log); _b < _r1; _b += _step) { \
        const int64_t i = _b + _sub;                                                 \
        if (i >= _r1) continue;

#define SEG_LOOP_END \
  }                  \
  }                  \
  }

__device__ __forceinline__ void seg_colsum(const SegArgs& a, double v, double* part) {
  ChunkGrid g;
  g.L = a.L;
  g.t = a.t;
  block_colsum(g, v, part);
}

// Per chunk of the table (t = 1): log p(y | F + b), D^{-1} (B b)^2, log D,
// log(W + D^{-1}) as four partial arrays of nchunk entries (laplace.hip).
Status seg_terms_launch(Model& M, SegArgs a, int nchunk, const double* b, const double* Bb,
                        const double* W, double* part);

// Operator pair of one CG solve.
struct CgOps {
  // V = A H over t columns (Tmp: n x t scratch)
  std::function<Status(Model&, const double* H, double* V, double* Tmp, int t)> apply;
  // Z = P^{-1} R; Z and Y (n x t scratch) arrive filled with the sentinel and
  // the work counters reset when needs_fill says so (no needs_fill: always)
  std::function<Status(Model&, const double* R, double* Z, double* Y, int t)> precond;
  std::function<bool(const Model&, int t)> needs_fill;
};

Status cg_solve(Model& M, CgState& S, const CgOps& ops, int t, const double* rhs, double tol,
                int max_iter, bool keep_z0, const int* forced_host = nullptr);
const int* replay_slice(const vl_opts& o, int c0, int t, std::vector<int>& buf);

// Mixed-precision form (mixed.hip): the VADU operator in FP64 and the
// preconditioner solves in FP32 (FP64 sums).
CgOps vadu_ops_mixed(const double* W, const double* sdiag);
// Relative deviation of the FP32 preconditioner from the FP64 one on the first
// column of X (n x t), for the mixed form's error estimate.
Status precond_f32_deviation(Model& M, const double* sdiag, const double* X, int t, double* dev);
Status to_f32(Model& M, const double* x, float* y, int64_t count);
// Xh = X - (tail entries of the head rows of B^T) applied to the FP32 block Y
// (sparse.hip; the fold stage of the level-scheduled B^T solve).
Status fold_launch_f32(Model& M, const double* X, const float* Y, double* Xh, int t);

Status dot_cols(Model& M, const double* X, const double* Y, int t, double* part, double* out);

// sparse kernels with explicit value arrays / probe inputs
Status spmm_ell_vals(Model& M, const double* vals, const double* X, double* Y, int t,
                     const double* rowscale, bool unit_diag);
// Y = d o probe1 + B^T (s o probe2); tmp1, tmp2 (n x t scratch, or null) let
// blocks wider than 64 columns write the probes once and take the wide product.
Status spmm_bt_probe(Model& M, double* Y, int t, const double* s, uint64_t seed, uint32_t tag2,
                     int col0, int gauss2, const double* d, uint32_t tag1, int gauss1,
                     double* tmp1, double* tmp2);
// CSR of the transpose of a rows x cols pattern given as rows x m column
// indices (-1 = none): row j of the result lists the (row index, source slot
// r * m + k) pairs with nbr[r * m + k] = j, sorted by row index.
Status transpose_pattern(Model& M, const int* nbr, int64_t rows, int m, int64_t cols,
                         DevBuf<int>& ptr, DevBuf<int>& col, DevBuf<int>& src, int* nnz_out);
// Y[i, c] = s_i eps_ic (Rademacher probes of columns col0 .. col0 + t - 1)
Status probe_fill(Model& M, double* Y, int t, const double* s, uint64_t seed, uint32_t tag,
                  int col0);
// FP32-storage narrow solves (t <= 64, mixed-precision form): B Y = rs o X
// with X and Y FP32, and B^T Y = X with X FP64 and Y FP32.
Status trsm_b_f32_narrow(Model& M, const float* X, float* Y, int t, const double* rowscale);
Status trsm_bt_f32_narrow(Model& M, const double* X, float* Y, int t);
Status trsm_b_slot(Model& M, const double* X, double* Y, int t, const double* rowscale,
                   bool prefilled, int slot);
Status trsm_bt_slot(Model& M, const double* X, double* Y, int t, bool prefilled, int slot);

}  // namespace vl
