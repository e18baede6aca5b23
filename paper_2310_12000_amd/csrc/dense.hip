// The leading K x K block of B as an explicit dense inverse, for the
// triangular solves of narrow blocks (t <= 64).
//
// B is unit lower triangular and row i < K only involves columns < K, so the
// first K unknowns of B y = x are y_K = G x_K with G = B_KK^{-1}, and those
// of B^T y = x are y_K = G^T (x_K - B_RK^T y_R), where R are the rows
// K..n-1, solved first.  With a random ordering the earliest points carry
// most of the dependency depth of the head: at n = 1e5, m = 20 the first
// 16384 rows span 214 levels, the rows 2048..16383 on their own 71 and the
// rows 4096..16383 49.  Taking the first K = 4096 rows out of the
// latency-bound level-by-level solve and applying G instead (67 MB of FP64
// per application, read at bandwidth by the whole chip) took the t = 1 head
// solves of the time (an LDS solve of rows below 16384) from 488 / 915 us to
// 298 / 321 us (forward / backward); K = 2048 gave 320 / 462 us.  Narrow
// blocks now take every row from K on in the sync-free tail.
//
// G is computed once per factor (Sec. 2.1: B changes with the covariance
// parameters) by forward substitution of B_KK G = I, column by column, and
// kept in both orientations: Gf[c K + i] = G_ic (columns contiguous) for
// G x, Gb[i K + c] = G_ic (rows contiguous) for G^T x.
#include <algorithm>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

// Columns of G per workgroup of the inverse: as many as 128 KB of LDS hold
// (8 at K = 2048), a power of two, at most 32.
static int dense_cols(int K) {
  int c = 1;
  while (c < 32 && static_cast<int64_t>(2 * c) * K * 8 <= 131072) c *= 2;
  return c;
}

// Columns c0..c0+C-1 of G in LDS; lane = (column cl, part q) with
// Q = 64 / C parts per column.  Part q sums the slots q, q + Q, ... of row
// i; the parts meet by a butterfly, and row i is final before row i + 1
// reads it (one wave: its LDS accesses complete in order).  Slot data does
// not depend on G and is fetched one row ahead.
// Batched form (tab_p given): block b inverts columns tab_c0[b].. of the
// leading block of problem tab_p[b] of a packed block-diagonal system, whose
// rows start[p]..start[p + 1]-1 are the whole problem (neighbour indices are
// packed, so they are shifted to the problem); its G goes to gofs[p].
template <int C>
__global__ __launch_bounds__(64) void dense_inverse_kernel(int K, int m,
                                                            const int* __restrict__ nbr,
                                                            const double* __restrict__ bval,
                                                            double* __restrict__ Gf,
                                                            double* __restrict__ Gb,
                                                            const int* __restrict__ tab_p,
                                                            const int* __restrict__ tab_c0,
                                                            const int* __restrict__ start,
                                                            const int64_t* __restrict__ gofs) {
  extern __shared__ double s_g[];  // C x K
  constexpr int Q = 64 / C;
  const int lane = threadIdx.x, cl = lane / Q, q = lane % Q;
  int c0 = blockIdx.x * C;
  int64_t s0 = 0;  // first packed row of the problem
  if (tab_p) {
    const int pp = tab_p[blockIdx.x];
    c0 = tab_c0[blockIdx.x];
    s0 = start[pp];
    K = start[pp + 1] - start[pp];
    Gf += gofs[pp];
    Gb += gofs[pp];
  }
  const int c = c0 + cl;
  for (int k = lane; k < C * K; k += 64) s_g[k] = 0.0;
  __syncthreads();
  double* g = s_g + cl * K;
  constexpr int kSlots = C / 2 > 0 ? C / 2 : 1;  // m <= 31: at most 32 / Q slots per part
  int nj[kSlots];
  double nw[kSlots];
  const int per = (m + Q - 1) / Q;
  auto fetch = [&](int i) {
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const int k = q + Q * u;
      const bool in = u < per && i < K && k < m;
      const int j = in ? nbr[(s0 + i) * m + k] : -1;
      nj[u] = j >= 0 ? static_cast<int>(j - s0) : -1;
      nw[u] = in ? bval[(s0 + i) * m + k] : 0.0;
    }
  };
  fetch(c0);
  for (int i = c0; i < K; ++i) {
    int cj[kSlots];
    double cw[kSlots];
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      cj[u] = nj[u];
      cw[u] = nw[u];
    }
    fetch(i + 1);
    // g_j = 0 for j < c (never written), so earlier columns add nothing
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kSlots; ++u)
      if (cj[u] >= 0) s += cw[u] * g[cj[u]];
#pragma unroll
    for (int o = 1; o < Q; o <<= 1) s += __shfl_xor(s, o);
    if (q == 0 && c < K && i >= c) g[i] = (i == c ? 1.0 : 0.0) - s;
  }
  __syncthreads();
  for (int k = lane; k < C * K; k += 64) {
    const int cc = c0 + k / K, i = k % K;
    if (cc < K) Gf[(int64_t)cc * K + i] = s_g[k];
  }
  for (int k = lane; k < C * K; k += 64) {
    const int i = k / C, u = k % C;
    if (c0 + u < K) Gb[(int64_t)i * K + c0 + u] = s_g[u * K + i];
  }
}

// out[r, c] = sum_s A[s K + r] v(s, c), v(s, c) = V[s t + c] (times rs[s]
// when given).  A is zero outside the triangle, so for the 64 rows of a row
// chunk the sum runs over s < end of the chunk (LOWER: A = Gf, out = G v) or
// s >= start of the chunk (A = Gb, out = G^T v).  The s range is cut into
// segments of kSeg: block (chunk x, segment y, column chunk z) stages its
// segment of v in LDS, its 8 waves take 32 steps each (16 loads of A in
// flight for one column, 8 for eight), meet in LDS in wave order and write
// one partial; a second kernel adds the partials of a chunk in segment
// order.  Every value of A is read once per column chunk, and the sums are
// deterministic.
constexpr int kSeg = 256;
constexpr int kApplyWaves = 8;

__host__ __device__ __forceinline__ int seg_lo(int chunk, bool lower) {
  return lower ? 0 : (chunk * 64) / kSeg;
}
__host__ __device__ __forceinline__ int seg_hi(int chunk, int K, bool lower) {
  const int end = lower ? min(K, chunk * 64 + 64) : K;
  return (end + kSeg - 1) / kSeg;
}

// Batched form (tab_p given): block x takes entry x of the tables, a (problem,
// row chunk, segment) triple of a packed block-diagonal system; the problem's
// G sits at gofs[p], its rows at start[p], its partials at pofs[p] t.
template <int TC, bool LOWER, typename TV = double>
__global__ __launch_bounds__(64 * kApplyWaves) void dense_part_kernel(
    int K, int t, const double* __restrict__ A, const TV* __restrict__ V,
    const double* __restrict__ rs, double* __restrict__ part, const int* __restrict__ tab_p,
    const int* __restrict__ tab_chunk, const int* __restrict__ tab_seg,
    const int* __restrict__ start, const int64_t* __restrict__ gofs,
    const int64_t* __restrict__ pofs) {
  __shared__ double s_v[kSeg][TC];
  __shared__ double s_red[kApplyWaves][TC][64];
  int chunk = blockIdx.x, g = blockIdx.y;
  if (tab_p) {
    const int pp = tab_p[blockIdx.x];
    chunk = tab_chunk[blockIdx.x];
    g = tab_seg[blockIdx.x];
    K = start[pp + 1] - start[pp];
    A += gofs[pp];
    V += static_cast<int64_t>(start[pp]) * t;
    if (rs) rs += start[pp];
    part += pofs[pp] * t;
  }
  if (g < seg_lo(chunk, LOWER) || g >= seg_hi(chunk, K, LOWER)) return;  // uniform
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = chunk * 64 + lane;
  const int c0 = blockIdx.z * TC;
  const int s_lo = max(g * kSeg, LOWER ? 0 : chunk * 64);
  const int s_hi = min((g + 1) * kSeg, LOWER ? min(K, chunk * 64 + 64) : K);
  for (int e = threadIdx.x; e < kSeg * TC; e += 64 * kApplyWaves) {
    const int s = g * kSeg + e / TC, c = c0 + e % TC;
    double v = 0.0;
    if (s >= s_lo && s < s_hi && c < t)
      v = static_cast<double>(V[(int64_t)s * t + c]) * (rs ? rs[s] : 1.0);
    s_v[e / TC][e % TC] = v;
  }
  __syncthreads();
  double acc[TC];
#pragma unroll
  for (int cc = 0; cc < TC; ++cc) acc[cc] = 0.0;
  constexpr int kStep = kSeg / kApplyWaves;  // 32
  constexpr int kU = TC == 1 ? 16 : 8;  // loads in flight (registers for 8 columns)
  const int sa = g * kSeg + wave * kStep;
#pragma unroll 1
  for (int h = 0; h < kStep; h += kU) {
    double a[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int s = sa + h + u;
      a[u] = (s >= s_lo && s < s_hi && r < K) ? A[(int64_t)s * K + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int sl = wave * kStep + h + u;
#pragma unroll
      for (int cc = 0; cc < TC; ++cc) acc[cc] += a[u] * s_v[sl][cc];
    }
  }
#pragma unroll
  for (int cc = 0; cc < TC; ++cc) s_red[wave][cc][lane] = acc[cc];
  __syncthreads();
  if (wave == 0 && r < K) {
#pragma unroll
    for (int cc = 0; cc < TC; ++cc) {
      if (c0 + cc >= t) break;
      double v = s_red[0][cc][lane];
      for (int w = 1; w < kApplyWaves; ++w) v += s_red[w][cc][lane];
      part[((int64_t)g * K + r) * t + c0 + cc] = v;
    }
  }
}

template <bool LOWER, typename TO = double>
__global__ void dense_reduce_kernel(int K, int t, const double* __restrict__ part,
                                    TO* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)K * t) return;
  const int r = static_cast<int>(e / t);
  const int chunk = r / 64;
  double v = 0.0;
  for (int g = seg_lo(chunk, LOWER); g < seg_hi(chunk, K, LOWER); ++g)
    v += part[(int64_t)g * K * t + e];
  out[e] = static_cast<TO>(v);
}

// Wide blocks (t > 64): out[r, c] = sum_s A[s lda + r] v(s, c) for the
// leading Kd rows, on the FP64 matrix cores.  Block (x, y) computes rows
// R x.. and columns 64 y..; its R / 16 waves own 32 x 32 pieces (2 x 2 tiles
// of v_mfma_f64_16x16x4f64), R / 32 down by 2 across.  The contraction runs
// over the triangle in steps of 16: the block stages 16 x R of A and 16 x 64
// of v in LDS (the next 16 are loaded into registers meanwhile), then each
// wave takes 4 MFMA steps per tile.  A taller block reuses each staged v
// tile for more rows (R = 128 for wide right-hand sides); R = 64 keeps the
// grid large enough to fill the chip when t is small.  Entries of A outside
// the triangle are stored zeros, so the step range of a block may overrun
// the triangle without changing any sum.  Operand layout of one MFMA step,
// lane l = 16 q + i: A[i][q] and B[q][i] in, D[q + 4 r][i] (r = 0..3) out.
// v and out are FP64 or, for the mixed-precision solves, FP32 (A and the
// accumulation stay FP64); outd, if given, receives out widened to FP64.
typedef double v4d __attribute__((ext_vector_type(4)));

template <bool LOWER, int R, typename TV, typename TO>
__global__ __launch_bounds__(R * 4) void dense_gemm_kernel(int Kd, int lda, int t,
                                                           const double* __restrict__ A,
                                                           const TV* __restrict__ V,
                                                           const double* __restrict__ rs,
                                                           TO* __restrict__ out,
                                                           double* __restrict__ outd) {
  static_assert(R == 64 || R == 128, "block height");
  constexpr int kTps = R / 4;     // staging threads per step
  constexpr int kCols = 64 / kTps;  // v columns each staging thread loads
  __shared__ double sA[16][R];    // [s][row]
  __shared__ double sB[16][64];   // [s][column]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = blockIdx.x * R, c0 = blockIdx.y * 64;
  const int s_lo = LOWER ? 0 : r0;
  const int s_hi = LOWER ? min(Kd, r0 + R) : Kd;
  const int wr = wave >> 1, wc = wave & 1;
  const int q = lane >> 4, i = lane & 15;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  // staging: thread -> one s, four rows of A, kCols columns of v
  const int sl = tid / kTps, xa = (tid % kTps) * 4, xb = (tid % kTps) * kCols;
  double ra[4], rb[kCols];  // the next tile, loaded while the current one is used
  auto fetch = [&](int s0) {
    const int s = s0 + sl;
    const bool in_s = s < s_hi;
    const double sc = (in_s && rs) ? rs[s] : 1.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = r0 + xa + u;
      ra[u] = (in_s && rr < Kd) ? A[(int64_t)s * lda + rr] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kCols; ++u) {
      const int cc = c0 + xb + u;
      rb[u] = (in_s && cc < t) ? static_cast<double>(V[(int64_t)s * t + cc]) * sc : 0.0;
    }
  };
  if (s_lo < s_hi) fetch(s_lo);
  for (int s0 = s_lo; s0 < s_hi; s0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sA[sl][xa + u] = ra[u];
#pragma unroll
    for (int u = 0; u < kCols; ++u) sB[sl][xb + u] = rb[u];
    __syncthreads();
    if (s0 + 16 < s_hi) fetch(s0 + 16);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sA[kk * 4 + q][wr * 32 + a * 16 + i];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sB[kk * 4 + q][wc * 32 + b * 16 + i];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = r0 + wr * 32 + a * 16 + q + 4 * rr;
        const int col = c0 + wc * 32 + b * 16 + i;
        if (row < Kd && col < t) {
          const TO o = static_cast<TO>(acc[a][b][rr]);
          out[(int64_t)row * t + col] = o;
          if (outd) outd[(int64_t)row * t + col] = static_cast<double>(o);
        }
      }
}

// xp[j, c] = base[j, c] - sum of the B^T entries of row j < K whose child is
// K or later (entries [lo[j], end[j]), end = the row ends), with the
// children's values from Y.  One wave per row, lanes over entries, a fixed
// butterfly per column.
template <typename TB, typename TY>
__global__ __launch_bounds__(256) void dense_fold_kernel(int K, int t, const int* __restrict__ lo,
                                                         const int* __restrict__ split,
                                                         const int* __restrict__ bt_col,
                                                         const double* __restrict__ bt_val,
                                                         const TB* __restrict__ base,
                                                         const TY* __restrict__ Y,
                                                         double* __restrict__ xp) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= K) return;
  const int b = lo[j], e = split[j];
  for (int c = 0; c < t; ++c) {
    double part = 0.0;
    for (int q = b + lane; q < e; q += 64)
      part += bt_val[q] * static_cast<double>(Y[(int64_t)bt_col[q] * t + c]);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) part += __shfl_xor(part, o);
    if (lane == 0) xp[(int64_t)j * t + c] = static_cast<double>(base[(int64_t)j * t + c]) - part;
  }
}

// lo[j] = first B^T entry of row j < K with child >= K.
__global__ void dense_lo_kernel(int K, const int* __restrict__ bt_ptr,
                                const int* __restrict__ bt_col, int* __restrict__ lo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K) return;
  int a = bt_ptr[j], b = bt_ptr[j + 1];
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (bt_col[mid] < K) {
      a = mid + 1;
    } else {
      b = mid;
    }
  }
  lo[j] = a;
}

Status build_dense(Model& M) {
  const int K = M.dense_rows;
  if (K <= 0) return Status::ok();
  const size_t kk = static_cast<size_t>(K) * K;
  VL_TRY(M.dense_gf.alloc(kk));
  VL_TRY(M.dense_gb.alloc(kk));
  VL_TRY(M.dense_lo.alloc(K));
  hipLaunchKernelGGL(dense_lo_kernel, dim3((K + 255) / 256), dim3(256), 0, M.stream, K,
                     M.bt_ptr.p, M.bt_col.p, M.dense_lo.p);
  if (M.dense_wide > 0) {
    VL_TRY(M.dense_lo_w.alloc(M.dense_wide));
    hipLaunchKernelGGL(dense_lo_kernel, dim3((M.dense_wide + 255) / 256), dim3(256), 0, M.stream,
                       M.dense_wide, M.bt_ptr.p, M.bt_col.p, M.dense_lo_w.p);
  }
  const size_t lds = sizeof(double) * dense_cols(K) * K;
  for (const void* f : {reinterpret_cast<const void*>(dense_inverse_kernel<1>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<2>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<4>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<8>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<16>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<32>)})
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
  (void)hipGetLastError();
  VL_TRY(check_launch("dense block"));
  return sync_stream(M.stream);
}

static Status bd_factor(Model& M);

Status dense_factor(Model& M) {
  if (M.bd_ready) VL_TRY(bd_factor(M));
  const int K = M.dense_rows;
  if (K <= 0) return Status::ok();
  const int C = dense_cols(K);
  const size_t lds = sizeof(double) * C * K;
  const dim3 grid((K + C - 1) / C);
#define VL_INVERSE(CC)                                                                          \
  hipLaunchKernelGGL(dense_inverse_kernel<CC>, grid, dim3(64), lds, M.stream, K, M.m, M.nbr.p, \
                     M.bval.p, M.dense_gf.p, M.dense_gb.p, nullptr, nullptr, nullptr, nullptr)
  switch (C) {
    case 1: VL_INVERSE(1); break;
    case 2: VL_INVERSE(2); break;
    case 4: VL_INVERSE(4); break;
    case 8: VL_INVERSE(8); break;
    case 16: VL_INVERSE(16); break;
    default: VL_INVERSE(32); break;
  }
#undef VL_INVERSE
  return check_launch("dense inverse");
}

template <bool LOWER, typename TV = double, typename TO = double>
static Status launch_apply(Model& M, const double* A, const TV* V, const double* rs,
                           TO* out, int t) {
  const int K = M.dense_rows;
  const int nseg = (K + kSeg - 1) / kSeg;
  const size_t need = static_cast<size_t>(nseg) * K * t;
  double* part = nullptr;
  if (M.ext) {
    if (M.ext->part_count < need) return Status::invalid("scratch too small for the dense product");
    part = M.ext->part;
  } else {
    VL_TRY(M.dense_part.reserve(need));
    part = M.dense_part.p;
  }
  const unsigned gx = static_cast<unsigned>((K + 63) / 64);
  if (t == 1) {
    hipLaunchKernelGGL((dense_part_kernel<1, LOWER, TV>), dim3(gx, nseg, 1),
                       dim3(64 * kApplyWaves), 0, M.stream, K, t, A, V, rs, part, nullptr,
                       nullptr, nullptr, nullptr, nullptr, nullptr);
  } else {
    hipLaunchKernelGGL((dense_part_kernel<8, LOWER, TV>), dim3(gx, nseg, (t + 7) / 8),
                       dim3(64 * kApplyWaves), 0, M.stream, K, t, A, V, rs, part,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  }
  const int64_t kt = static_cast<int64_t>(K) * t;
  hipLaunchKernelGGL((dense_reduce_kernel<LOWER, TO>),
                     dim3(static_cast<unsigned>((kt + 255) / 256)), dim3(256), 0, M.stream, K, t,
                     part, out);
  return check_launch("dense apply");
}

static double apply_bytes(const Model& M, int t) {
  const double K = M.dense_rows;
  return 8.0 * K * (K + 1) / 2.0 + 16.0 * K * t;
}

Status dense_lower(Model& M, const double* X, double* Y, int t, const double* rs) {
  TimedLaunch tl(M, kTimeDenseLower, apply_bytes(M, t));
  return launch_apply<true>(M, M.dense_gf.p, X, rs, Y, t);
}

Status dense_upper(Model& M, const double* X, double* Y, int t) {
  const int K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseUpper, apply_bytes(M, t));
  const size_t need = static_cast<size_t>(K) * t;
  double* xp = nullptr;
  if (M.ext) {
    if (M.ext->xp_count < need) return Status::invalid("scratch too small for the dense fold");
    xp = M.ext->xp;
  } else {
    VL_TRY(M.dense_xp.reserve(need));
    xp = M.dense_xp.p;
  }
  hipLaunchKernelGGL((dense_fold_kernel<double, double>), dim3((K + 3) / 4), dim3(256), 0,
                     M.stream, K, t, M.dense_lo.p, M.bt_ptr.p + 1, M.bt_col.p, M.bt_val.p, X, Y,
                     xp);
  return launch_apply<false>(M, M.dense_gb.p, xp, nullptr, Y, t);
}

// FP32-storage forms for the mixed-precision narrow blocks (G, the sums and
// the folded right-hand sides stay FP64).
Status dense_lower_f32(Model& M, const float* X, float* Y, int t, const double* rs) {
  TimedLaunch tl(M, kTimeDenseLower, apply_bytes(M, t) - 8.0 * M.dense_rows * t);
  return launch_apply<true, float, float>(M, M.dense_gf.p, X, rs, Y, t);
}

Status dense_upper_f32(Model& M, const double* X, float* Y, int t) {
  const int K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseUpper, apply_bytes(M, t) - 4.0 * K * t);
  VL_TRY(M.dense_xp.reserve(static_cast<size_t>(K) * t));
  hipLaunchKernelGGL((dense_fold_kernel<double, float>), dim3((K + 3) / 4), dim3(256), 0,
                     M.stream, K, t, M.dense_lo.p, M.bt_ptr.p + 1, M.bt_col.p, M.bt_val.p, X, Y,
                     M.dense_xp.p);
  return launch_apply<false, double, float>(M, M.dense_gb.p, M.dense_xp.p, nullptr, Y, t);
}

// Launches dense_gemm_kernel with 128-row blocks when those alone make a grid
// of at least kGemmTallBlocks blocks (wide t), else with 64-row blocks.
constexpr int kGemmTallBlocks = 256;

template <bool LOWER, typename TV, typename TO>
void launch_gemm(Model& M, int Kd, int lda, int t, const double* A, const TV* V,
                 const double* rs, TO* out, double* outd) {
  const int cols = (t + 63) / 64;
  if (((Kd + 127) / 128) * cols >= kGemmTallBlocks)
    hipLaunchKernelGGL((dense_gemm_kernel<LOWER, 128, TV, TO>), dim3((Kd + 127) / 128, cols),
                       dim3(512), 0, M.stream, Kd, lda, t, A, V, rs, out, outd);
  else
    hipLaunchKernelGGL((dense_gemm_kernel<LOWER, 64, TV, TO>), dim3((Kd + 63) / 64, cols),
                       dim3(256), 0, M.stream, Kd, lda, t, A, V, rs, out, outd);
}

// Wide blocks: the leading Kw rows of G are the inverse of B's leading
// Kw x Kw block (a leading block of a triangular inverse), so the same G
// serves with leading dimension K.
Status dense_wide_lower(Model& M, const double* X, double* Y, int t, const double* rs) {
  const int Kw = M.dense_wide, K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseWide, 4.0 * Kw * (Kw + 1.0) + 16.0 * Kw * t);
  launch_gemm<true>(M, Kw, K, t, M.dense_gf.p, X, rs, Y, static_cast<double*>(nullptr));
  return check_launch("dense wide lower");
}

// The mixed-precision forward solve's leading rows: X, Y in FP32, Yd the FP64
// copy of Y; G and the sums in FP64.
Status dense_wide_lower_f32(Model& M, const float* X, float* Y, double* Yd, int t,
                            const double* rs) {
  const int Kw = M.dense_wide, K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseWide, 4.0 * Kw * (Kw + 1.0) + 16.0 * Kw * t);
  launch_gemm<true>(M, Kw, K, t, M.dense_gf.p, X, rs, Y, Yd);
  return check_launch("dense wide lower f32");
}

// Y_j (j < Kw) = sum_i G_ij x'_i, x'_j = Xh_j - the B^T entries of row j with
// child in Kw..H-1 (Xh: the right-hand side with the tail entries folded).
Status dense_wide_upper(Model& M, const double* Xh, double* Y, int t) {
  const int Kw = M.dense_wide, K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseWide, 4.0 * Kw * (Kw + 1.0) + 16.0 * Kw * t);
  VL_TRY(M.dense_xp.reserve(static_cast<size_t>(Kw) * t));
  VL_TRY(fold_rows(M, Kw, M.dense_lo_w.p, M.head_split.p, Xh, Y, M.dense_xp.p, t));
  launch_gemm<false>(M, Kw, K, t, M.dense_gb.p, M.dense_xp.p, nullptr, Y,
                     static_cast<double*>(nullptr));
  return check_launch("dense wide upper");
}

// The mixed-precision backward solve's leading rows: Xh in FP64 (the folded
// right-hand side), Y in FP32.
Status dense_wide_upper_f32(Model& M, const double* Xh, float* Y, int t) {
  const int Kw = M.dense_wide, K = M.dense_rows;
  TimedLaunch tl(M, kTimeDenseWide, 4.0 * Kw * (Kw + 1.0) + 12.0 * Kw * t);
  VL_TRY(M.dense_xp.reserve(static_cast<size_t>(Kw) * t));
  VL_TRY(fold_rows(M, Kw, M.dense_lo_w.p, M.head_split.p, Xh, Y, M.dense_xp.p, t));
  launch_gemm<false>(M, Kw, K, t, M.dense_gb.p, M.dense_xp.p, nullptr, Y,
                     static_cast<double*>(nullptr));
  return check_launch("dense wide upper f32");
}

// ------------------------------------------------ block-diagonal (batching)
// out[r, c] for every packed row r: the sum of its problem's partials in
// segment order.
template <bool LOWER>
__global__ void bd_reduce_kernel(int64_t n, int t, const int* __restrict__ row_prob,
                                 const int* __restrict__ row_local, const int* __restrict__ start,
                                 const int64_t* __restrict__ pofs, const double* __restrict__ part,
                                 double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * t) return;
  const int64_t r = e / t;
  const int c = static_cast<int>(e - r * t);
  const int pp = row_prob[r], loc = row_local[r];
  const int K = start[pp + 1] - start[pp];
  const int chunk = loc / 64;
  const double* pt = part + pofs[pp] * t;
  double v = 0.0;
  for (int g = seg_lo(chunk, LOWER); g < seg_hi(chunk, K, LOWER); ++g)
    v += pt[((int64_t)g * K + loc) * t + c];
  out[e] = v;
}

template <typename T>
static Status upload(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  VL_TRY(d.alloc(h.size() > 0 ? h.size() : 1));
  if (!h.empty())
    VL_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
  return Status::ok();
}

Status bd_build(Model& M, const std::vector<int64_t>& start, const std::vector<int64_t>& n,
                const int* row_prob, const int* row_local) {
  M.bd_ready = false;
  const int P = static_cast<int>(n.size());
  if (P == 0 || M.m < 1) return Status::ok();
  int64_t kmax = 0;
  double bytes = 0.0;
  for (int64_t k : n) {
    kmax = std::max(kmax, k);
    bytes += 16.0 * static_cast<double>(k) * static_cast<double>(k);
  }
  if (kmax > kDenseRows || bytes > kBdBytesCap) return Status::ok();  // not this form
  const int K = static_cast<int>(kmax);
  const int C = dense_cols(K);
  std::vector<int> st(P + 1), inv_p, inv_c0, lo_p, lo_c, lo_g, up_p, up_c, up_g;
  std::vector<int64_t> gofs(P), pofs(P);
  int64_t g_acc = 0, p_acc = 0;
  for (int p = 0; p < P; ++p) {
    st[p] = static_cast<int>(start[p]);
    const int k = static_cast<int>(n[p]);
    gofs[p] = g_acc;
    pofs[p] = p_acc;
    g_acc += static_cast<int64_t>(k) * k;
    p_acc += static_cast<int64_t>((k + kSeg - 1) / kSeg) * k;
    for (int c0 = 0; c0 < k; c0 += C) {
      inv_p.push_back(p);
      inv_c0.push_back(c0);
    }
    for (int ch = 0; ch < (k + 63) / 64; ++ch) {
      for (int g = seg_lo(ch, true); g < seg_hi(ch, k, true); ++g) {
        lo_p.push_back(p);
        lo_c.push_back(ch);
        lo_g.push_back(g);
      }
      for (int g = seg_lo(ch, false); g < seg_hi(ch, k, false); ++g) {
        up_p.push_back(p);
        up_c.push_back(ch);
        up_g.push_back(g);
      }
    }
  }
  st[P] = static_cast<int>(start[P - 1] + n[P - 1]);
  hipStream_t s = M.stream;
  VL_TRY(upload(M.bd_start, st, s));
  VL_TRY(upload(M.bd_gofs, gofs, s));
  VL_TRY(upload(M.bd_pofs, pofs, s));
  VL_TRY(upload(M.bd_inv_p, inv_p, s));
  VL_TRY(upload(M.bd_inv_c0, inv_c0, s));
  VL_TRY(upload(M.bd_lo_p, lo_p, s));
  VL_TRY(upload(M.bd_lo_chunk, lo_c, s));
  VL_TRY(upload(M.bd_lo_seg, lo_g, s));
  VL_TRY(upload(M.bd_up_p, up_p, s));
  VL_TRY(upload(M.bd_up_chunk, up_c, s));
  VL_TRY(upload(M.bd_up_seg, up_g, s));
  VL_TRY(M.bd_gf.alloc(static_cast<size_t>(g_acc)));
  VL_TRY(M.bd_gb.alloc(static_cast<size_t>(g_acc)));
  VL_TRY(sync_stream(s));
  M.bd_C = C;
  M.bd_kmax = K;
  M.bd_inv_n = static_cast<int>(inv_p.size());
  M.bd_lo_n = static_cast<int>(lo_p.size());
  M.bd_up_n = static_cast<int>(up_p.size());
  M.bd_part_rows = p_acc;
  M.bd_row_prob = row_prob;
  M.bd_row_local = row_local;
  const size_t lds = sizeof(double) * C * K;
  for (const void* f : {reinterpret_cast<const void*>(dense_inverse_kernel<1>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<2>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<4>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<8>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<16>),
                        reinterpret_cast<const void*>(dense_inverse_kernel<32>)})
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
  (void)hipGetLastError();
  M.bd_ready = true;
  return Status::ok();
}

static Status bd_factor(Model& M) {
  const int C = M.bd_C;
  const size_t lds = sizeof(double) * C * M.bd_kmax;
  const dim3 grid(M.bd_inv_n);
#define VL_BD_INVERSE(CC)                                                                  \
  hipLaunchKernelGGL(dense_inverse_kernel<CC>, grid, dim3(64), lds, M.stream, M.bd_kmax, M.m, \
                     M.nbr.p, M.bval.p, M.bd_gf.p, M.bd_gb.p, M.bd_inv_p.p, M.bd_inv_c0.p,   \
                     M.bd_start.p, M.bd_gofs.p)
  switch (C) {
    case 1: VL_BD_INVERSE(1); break;
    case 2: VL_BD_INVERSE(2); break;
    case 4: VL_BD_INVERSE(4); break;
    case 8: VL_BD_INVERSE(8); break;
    case 16: VL_BD_INVERSE(16); break;
    default: VL_BD_INVERSE(32); break;
  }
#undef VL_BD_INVERSE
  return check_launch("block-diagonal inverse");
}

template <bool LOWER>
static Status bd_apply(Model& M, const double* X, double* Y, int t, const double* rs) {
  VL_TRY(M.bd_part.reserve(static_cast<size_t>(M.bd_part_rows) * t));
  const double* A = LOWER ? M.bd_gf.p : M.bd_gb.p;
  const int nb = LOWER ? M.bd_lo_n : M.bd_up_n;
  const int* tp = LOWER ? M.bd_lo_p.p : M.bd_up_p.p;
  const int* tc = LOWER ? M.bd_lo_chunk.p : M.bd_up_chunk.p;
  const int* tg = LOWER ? M.bd_lo_seg.p : M.bd_up_seg.p;
  if (t == 1) {
    hipLaunchKernelGGL((dense_part_kernel<1, LOWER>), dim3(nb, 1, 1), dim3(64 * kApplyWaves), 0,
                       M.stream, M.bd_kmax, t, A, X, rs, M.bd_part.p, tp, tc, tg, M.bd_start.p,
                       M.bd_gofs.p, M.bd_pofs.p);
  } else {
    hipLaunchKernelGGL((dense_part_kernel<8, LOWER>), dim3(nb, 1, (t + 7) / 8),
                       dim3(64 * kApplyWaves), 0, M.stream, M.bd_kmax, t, A, X, rs, M.bd_part.p,
                       tp, tc, tg, M.bd_start.p, M.bd_gofs.p, M.bd_pofs.p);
  }
  const int64_t nt = M.n * static_cast<int64_t>(t);
  hipLaunchKernelGGL(bd_reduce_kernel<LOWER>, dim3(static_cast<unsigned>((nt + 255) / 256)),
                     dim3(256), 0, M.stream, M.n, t, M.bd_row_prob, M.bd_row_local,
                     M.bd_start.p, M.bd_pofs.p, M.bd_part.p, Y);
  return check_launch("block-diagonal product");
}

Status bd_lower(Model& M, const double* X, double* Y, int t, const double* rs) {
  TimedLaunch tl(M, kTimeDenseLower, 16.0 * M.n * t);
  return bd_apply<true>(M, X, Y, t, rs);
}

Status bd_upper(Model& M, const double* X, double* Y, int t) {
  TimedLaunch tl(M, kTimeDenseUpper, 16.0 * M.n * t);
  return bd_apply<false>(M, X, Y, t, nullptr);
}

}  // namespace vl
