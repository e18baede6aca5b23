// Batching form: many independent problems of different sizes in one packed,
// block-diagonal model, so that every launch of the sparse kernels, the CG
// vector kernels and the reductions serves all problems at once.
//
// Packing.  Problem p occupies rows [start_p, start_p + n_p) of the packed
// system; its neighbour sets stay inside its own rows (the Vecchia factor of
// the batch is block diagonal), stored as ELL of width max_p m_p padded with
// -1.  Neighbour search and the neighbour Cholesky run per problem on the
// problem's own points; the packed model then builds B^T and the level
// schedules once for all rows.
//
// Segmented CG.  Each problem's rows are cut into the row chunks a solo run
// of that problem would use; a work item is (row chunk of a problem, probe
// slice), and every column reduction sums a problem's own chunks in order.
// The CG scalars (alpha, beta, r.z, activity, iteration counts, Lanczos
// history) are kept per (problem, probe), so each problem follows exactly
// the recurrence of the appendix PCG algorithm on its own system, and
// Newton's method runs all problems in lockstep with per-problem
// convergence and step halving.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>

#include "vl_internal.h"
#include "vl_laplace.h"
#include "vl_ops.h"

namespace vl {

Status finish_factor(Model& M);

constexpr int kBatchMaxProblems = 32;
constexpr int64_t kBatchMaxRows = 65536;

// ----------------------------------------------------------- chunk tables
struct SegTable {
  int nprob = 0, nchunk = 0, t = 0;
  Lanes L;
  DevBuf<int> chunk_prob, chunk_r0, chunk_r1, prob_chunk0;
  std::vector<int> h_prob_chunk0;
};

static Status build_seg(Model& M, const std::vector<int64_t>& start,
                        const std::vector<int64_t>& n, int t, SegTable& S) {
  const int P = static_cast<int>(n.size());
  std::vector<int> cp, c0, c1, pc0(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    pc0[p] = static_cast<int>(cp.size());
    ChunkGrid g = ChunkGrid::of(n[p], t);  // the chunks of a solo run of problem p
    for (int k = 0; k < g.nchunk; ++k) {
      const int64_t r0 = k * g.rpc;
      int64_t r1 = r0 + g.rpc;
      if (r1 > n[p]) r1 = n[p];
      cp.push_back(p);
      c0.push_back(static_cast<int>(start[p] + r0));
      c1.push_back(static_cast<int>(start[p] + r1));
    }
  }
  pc0[P] = static_cast<int>(cp.size());
  S.nprob = P;
  S.nchunk = static_cast<int>(cp.size());
  S.t = t;
  S.L = Lanes::of(t);
  S.h_prob_chunk0 = pc0;
  VL_TRY(S.chunk_prob.alloc(S.nchunk));
  VL_TRY(S.chunk_r0.alloc(S.nchunk));
  VL_TRY(S.chunk_r1.alloc(S.nchunk));
  VL_TRY(S.prob_chunk0.alloc(P + 1));
  VL_HIP(hipMemcpyAsync(S.chunk_prob.p, cp.data(), sizeof(int) * S.nchunk,
                        hipMemcpyHostToDevice, M.stream));
  VL_HIP(hipMemcpyAsync(S.chunk_r0.p, c0.data(), sizeof(int) * S.nchunk, hipMemcpyHostToDevice,
                        M.stream));
  VL_HIP(hipMemcpyAsync(S.chunk_r1.p, c1.data(), sizeof(int) * S.nchunk, hipMemcpyHostToDevice,
                        M.stream));
  VL_HIP(hipMemcpyAsync(S.prob_chunk0.p, pc0.data(), sizeof(int) * (P + 1),
                        hipMemcpyHostToDevice, M.stream));
  return sync_stream(M.stream);
}

// --------------------------------------------------- segmented CG kernels
__global__ __launch_bounds__(256) void seg_init_kernel(SegArgs a, const double* __restrict__ rhs,
                                                       double* __restrict__ U,
                                                       double* __restrict__ R,
                                                       double* __restrict__ Y,
                                                       double* __restrict__ Z, int* counter) {
  SEG_LOOP_BEGIN(a)
  const int64_t o = i * a.t + c;
  U[o] = 0.0;
  R[o] = rhs[o];
  Y[o] = sentinel();
  Z[o] = sentinel();
  SEG_LOOP_END
  if (blockIdx.x == 0 && blockIdx.y == 0) reset_counters(counter);
}

__global__ __launch_bounds__(256) void seg_init2_kernel(SegArgs a, const double* __restrict__ R,
                                                        const double* __restrict__ Z,
                                                        double* __restrict__ H,
                                                        double* __restrict__ part) {
  double acc = 0.0;
  SEG_LOOP_BEGIN(a)
  const int64_t o = i * a.t + c;
  const double z = Z[o];
  H[o] = z;
  acc += R[o] * z;
  SEG_LOOP_END
  seg_colsum(a, acc, part);
}

__global__ __launch_bounds__(256) void seg_dot_kernel(SegArgs a, const double* __restrict__ X,
                                                      const double* __restrict__ Y,
                                                      double* __restrict__ part) {
  double acc = 0.0;
  SEG_LOOP_BEGIN(a)
  const int64_t o = i * a.t + c;
  acc += X[o] * Y[o];
  SEG_LOOP_END
  seg_colsum(a, acc, part);
}

// per (problem p, column c), q = p t + c: the sum of p's chunk partials
__device__ __forceinline__ double seg_sum(const double* part, const int* pc0, int t, int p,
                                          int c) {
  double s = 0.0;
  for (int k = pc0[p]; k < pc0[p + 1]; ++k) s += part[(int64_t)k * t + c];
  return s;
}

__global__ void seg_start_kernel(int P, int t, const int* __restrict__ pc0,
                                 const int* __restrict__ pmask, const double* __restrict__ part,
                                 double* __restrict__ rz, double* __restrict__ r0z0,
                                 int* __restrict__ active, int* __restrict__ iters) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P * t) return;
  const int p = q / t, c = q - (q / t) * t;
  const double s = seg_sum(part, pc0, t, p, c);
  rz[q] = s;
  r0z0[q] = s;
  active[q] = (pmask[p] && s > 0.0) ? 1 : 0;
  iters[q] = 0;
}

__global__ void seg_alpha_kernel(int P, int t, const int* __restrict__ pc0,
                                 const double* __restrict__ part, const double* __restrict__ rz,
                                 double* __restrict__ alpha, const int* __restrict__ active,
                                 const int* __restrict__ iters, double* __restrict__ hist_a,
                                 int* __restrict__ status) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P * t) return;
  const int p = q / t, c = q - (q / t) * t;
  double a = 0.0;
  if (active[q]) {
    const double hv = seg_sum(part, pc0, t, p, c);
    if (!(hv > 0.0) || !isfinite(hv)) {
      raise_error(status, kErrNonfinite);
    } else {
      a = rz[q] / hv;
      hist_a[(int64_t)iters[q] * P * t + q] = a;
    }
  }
  alpha[q] = a;
}

__global__ __launch_bounds__(256) void seg_update_ur_kernel(
    SegArgs a, const double* __restrict__ alpha, const int* __restrict__ active,
    const double* __restrict__ H, const double* __restrict__ V, double* __restrict__ U,
    double* __restrict__ R, double* __restrict__ Y, double* __restrict__ Z,
    double* __restrict__ part, int* counter) {
  const int q0 = a.prob[blockIdx.x] * a.t;
  double acc = 0.0;
  SEG_LOOP_BEGIN(a)
  const int64_t o = i * a.t + c;
  double r = R[o];
  if (active[q0 + c]) {
    const double al = alpha[q0 + c];
    U[o] += al * H[o];
    r -= al * V[o];
    R[o] = r;
  }
  acc += r * r;
  Y[o] = sentinel();
  Z[o] = sentinel();
  SEG_LOOP_END
  seg_colsum(a, acc, part);
  if (blockIdx.x == 0 && blockIdx.y == 0) reset_counters(counter);
}

__global__ void seg_beta_kernel(int P, int t, const int* __restrict__ pc0,
                                const double* __restrict__ part_rz,
                                const double* __restrict__ part_rr, double tol, int max_iter,
                                double* __restrict__ rz, double* __restrict__ beta,
                                int* __restrict__ active, int* __restrict__ iters,
                                double* __restrict__ hist_b, int* __restrict__ num_active,
                                int* __restrict__ status) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P * t) return;
  const int p = q / t, c = q - (q / t) * t;
  double b = 0.0;
  if (active[q]) {
    const double rzn = seg_sum(part_rz, pc0, t, p, c);
    const double rr = seg_sum(part_rr, pc0, t, p, c);
    const int it = iters[q];
    b = rzn / rz[q];
    hist_b[(int64_t)it * P * t + q] = b;
    rz[q] = rzn;
    iters[q] = it + 1;
    if (!isfinite(rr) || !isfinite(b)) raise_error(status, kErrNonfinite);
    if (sqrt(rr) < tol || it + 1 >= max_iter || !isfinite(rr)) {
      active[q] = 0;
    } else {
      atomicAdd(num_active, 1);
    }
  }
  beta[q] = b;
}

__global__ __launch_bounds__(256) void seg_update_h_kernel(SegArgs a,
                                                           const double* __restrict__ beta,
                                                           const int* __restrict__ active,
                                                           const double* __restrict__ Z,
                                                           double* __restrict__ H) {
  const int q0 = a.prob[blockIdx.x] * a.t;
  SEG_LOOP_BEGIN(a)
  if (active[q0 + c]) {
    const int64_t o = i * a.t + c;
    H[o] = Z[o] + beta[q0 + c] * H[o];
  }
  SEG_LOOP_END
}

// ------------------------------------------------------------ batch state
struct Batch {
  Model M;                     // the packed model
  int P = 0;
  int lik = 0;
  double aux = 0.0;
  std::vector<int64_t> start, n;
  std::vector<int> m;
  std::vector<uint64_t> seed;
  DevBuf<int> row_prob;        // packed row -> problem
  DevBuf<int> row_local;       // packed row -> row inside its problem
  DevBuf<uint64_t> prob_seed;  // per problem
  SegTable seg1, segt;         // chunk tables for t = 1 and t = probes
  CgState cg;                  // segmented CG state (scalars per problem x column)
  DevBuf<int> pmask;           // problems taking part in the current solve
  // per problem results of the last fit
  std::vector<double> nll;
  std::vector<int> newton_iters, halvings_total, slq_iters_max;
  std::vector<int> tune;       // autotuned solve path per width class
};

// ------------------------------------------------------------- autotuning
// The tile choice of the packed system's triangular solves, per width class
// (t = 1, 2..64, > 64): the sync-free rows, one launch per
// level, or (when every problem is small enough) each problem's B inverted
// whole and applied as a dense product.  Candidates are timed on the packed
// system itself (one B^{-T} and one B^{-1} solve each, after one untimed
// pass) and the fastest one is kept for that width class and the system's
// shape (rows, m, dense form available).
static std::map<std::tuple<int64_t, int, int>, int>& tune_cache() {
  static std::map<std::tuple<int64_t, int, int>, int> c;
  return c;
}

static int width_class(int t) { return t <= 1 ? 0 : (t <= 64 ? 1 : 2); }

static Status autotune(Model& M, int t, int* choice) {
  const auto key = std::make_tuple(M.n, M.m, width_class(t) + (M.bd_ready ? 8 : 0));
  auto it = tune_cache().find(key);
  if (it != tune_cache().end()) {
    *choice = it->second;
    return Status::ok();
  }
  DevBuf<double> X, Y, Z;
  const size_t nt = static_cast<size_t>(M.n) * t;
  VL_TRY(X.alloc(nt));
  VL_TRY(Y.alloc(nt));
  VL_TRY(Z.alloc(nt));
  VL_TRY(fill_double(X.p, 1.0, static_cast<int64_t>(nt), M.stream));
  double best = 1e300;
  int pick = 0;
  hipEvent_t e0, e1;
  VL_HIP(hipEventCreate(&e0));
  VL_HIP(hipEventCreate(&e1));
  for (int cand = 0; cand < (M.bd_ready ? 3 : 2); ++cand) {
    M.force_levels = cand == 1;
    M.bd_use = cand == 2;
    for (int rep = 0; rep < 2; ++rep) {
      VL_HIP(hipEventRecord(e0, M.stream));
      VL_TRY(trsm_bt(M, X.p, Y.p, t, false));
      VL_TRY(trsm_b(M, Y.p, Z.p, t, nullptr, false));
      VL_HIP(hipEventRecord(e1, M.stream));
      VL_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      VL_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1 && ms < best) {
        best = ms;
        pick = cand;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  M.force_levels = false;
  M.bd_use = false;
  VL_TRY(read_status(M));
  tune_cache()[key] = pick;
  *choice = pick;
  return Status::ok();
}

// ---------------------------------------------------------- segmented CG
static Status seg_reserve(Batch& Bt, const SegTable& S, int lmax) {
  Model& M = Bt.M;
  CgState& C = Bt.cg;
  const size_t nt = static_cast<size_t>(M.n) * S.t;
  const size_t q = static_cast<size_t>(S.nprob) * S.t;
  VL_TRY(C.U.reserve(nt));
  VL_TRY(C.R.reserve(nt));
  VL_TRY(C.Z.reserve(nt));
  VL_TRY(C.H.reserve(nt));
  VL_TRY(C.V.reserve(nt));
  VL_TRY(C.Tmp.reserve(nt));
  VL_TRY(C.Y.reserve(nt));
  VL_TRY(C.rz.reserve(q));
  VL_TRY(C.alpha.reserve(q));
  VL_TRY(C.beta.reserve(q));
  VL_TRY(C.r0z0.reserve(q));
  VL_TRY(C.active.reserve(q));
  VL_TRY(C.iters.reserve(q));
  VL_TRY(C.num_active.reserve(4));
  VL_TRY(C.hist_a.reserve(static_cast<size_t>(lmax) * q));
  VL_TRY(C.hist_b.reserve(static_cast<size_t>(lmax) * q));
  VL_TRY(C.part_a.reserve(static_cast<size_t>(S.nchunk) * S.t));
  VL_TRY(C.part_b.reserve(static_cast<size_t>(S.nchunk) * S.t));
  VL_TRY(M.counter.reserve(2 * kSlotInts + 64));
  if (!M.host_pin) VL_HIP(hipHostMalloc(reinterpret_cast<void**>(&M.host_pin), 64 * sizeof(double)));
  C.t = S.nprob * S.t;  // the quadrature sees one column per (problem, probe)
  C.lmax = lmax;
  return Status::ok();
}

static Status seg_cg(Batch& Bt, const SegTable& S, const CgOps& ops, const double* rhs,
                     double tol, int max_iter) {
  Model& M = Bt.M;
  CgState& C = Bt.cg;
  VL_TRY(seg_reserve(Bt, S, max_iter));
  hipStream_t s = M.stream;
  SegArgs a{S.L, S.t, S.chunk_prob.p, S.chunk_r0.p, S.chunk_r1.p};
  const dim3 grid(S.nchunk, S.L.slices);
  const int q = S.nprob * S.t;
  const dim3 qg((q + 255) / 256);
  int* cnt = M.counter.p;
  hipLaunchKernelGGL(seg_init_kernel, grid, dim3(256), 0, s, a, rhs, C.U.p, C.R.p, C.Y.p, C.Z.p,
                     cnt);
  VL_TRY(ops.precond(M, C.R.p, C.Z.p, C.Y.p, S.t));
  hipLaunchKernelGGL(seg_init2_kernel, grid, dim3(256), 0, s, a, C.R.p, C.Z.p, C.H.p,
                     C.part_a.p);
  hipLaunchKernelGGL(seg_start_kernel, qg, dim3(256), 0, s, S.nprob, S.t, S.prob_chunk0.p,
                     Bt.pmask.p, C.part_a.p, C.rz.p, C.r0z0.p, C.active.p, C.iters.p);
  VL_TRY(check_launch("seg cg start"));
  for (int it = 0; it < max_iter; ++it) {
    VL_TRY(ops.apply(M, C.H.p, C.V.p, C.Tmp.p, S.t));
    hipLaunchKernelGGL(seg_dot_kernel, grid, dim3(256), 0, s, a, C.H.p, C.V.p, C.part_a.p);
    hipLaunchKernelGGL(seg_alpha_kernel, qg, dim3(256), 0, s, S.nprob, S.t, S.prob_chunk0.p,
                       C.part_a.p, C.rz.p, C.alpha.p, C.active.p, C.iters.p, C.hist_a.p,
                       M.status);
    hipLaunchKernelGGL(seg_update_ur_kernel, grid, dim3(256), 0, s, a, C.alpha.p, C.active.p,
                       C.H.p, C.V.p, C.U.p, C.R.p, C.Y.p, C.Z.p, C.part_b.p, cnt);
    VL_TRY(ops.precond(M, C.R.p, C.Z.p, C.Y.p, S.t));
    hipLaunchKernelGGL(seg_dot_kernel, grid, dim3(256), 0, s, a, C.R.p, C.Z.p, C.part_a.p);
    VL_HIP(hipMemsetAsync(C.num_active.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(seg_beta_kernel, qg, dim3(256), 0, s, S.nprob, S.t, S.prob_chunk0.p,
                       C.part_a.p, C.part_b.p, tol, max_iter, C.rz.p, C.beta.p, C.active.p,
                       C.iters.p, C.hist_b.p, C.num_active.p, M.status);
    hipLaunchKernelGGL(seg_update_h_kernel, grid, dim3(256), 0, s, a, C.beta.p, C.active.p,
                       C.Z.p, C.H.p);
    VL_TRY(check_launch("seg cg iteration"));
    VL_HIP(hipMemcpyAsync(M.host_pin, C.num_active.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VL_TRY(sync_stream(s));
    if (*reinterpret_cast<int*>(M.host_pin) == 0) break;
  }
  C.host_iters.resize(q);
  VL_HIP(hipMemcpyAsync(C.host_iters.data(), C.iters.p, sizeof(int) * q, hipMemcpyDeviceToHost,
                        s));
  VL_TRY(sync_stream(s));
  return read_status(M);
}

// ------------------------------------------------------ per-problem terms
// the problem sums of the chunk partials of seg_terms_launch, in chunk order
// (as host_sums adds a solo run's chunks)

__global__ void seg_terms_sum_kernel(int P, const int* __restrict__ pc0, int nchunk,
                                     const double* __restrict__ part, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int j = pc0[p]; j < pc0[p + 1]; ++j) s += part[(int64_t)k * nchunk + j];
    out[4 * p + k] = s;
  }
}


static Status problem_terms(Batch& Bt, const double* b, const double* W,
                            std::vector<double>& terms) {
  Model& M = Bt.M;
  const SegTable& S = Bt.seg1;
  VL_TRY(M.vec_d.reserve(M.n));
  VL_TRY(spmm_b(M, b, M.vec_d.p, 1, nullptr));
  VL_TRY(M.red_part.reserve(static_cast<size_t>(S.nchunk) * 4));
  VL_TRY(M.red_out.reserve(static_cast<size_t>(S.nprob) * 4 + 64));
  SegArgs a{S.L, 1, S.chunk_prob.p, S.chunk_r0.p, S.chunk_r1.p};
  VL_TRY(seg_terms_launch(M, a, S.nchunk, b, M.vec_d.p, W, M.red_part.p));
  hipLaunchKernelGGL(seg_terms_sum_kernel, dim3((S.nprob + 255) / 256), dim3(256), 0, M.stream,
                     S.nprob, S.prob_chunk0.p, S.nchunk, M.red_part.p, M.red_out.p);
  VL_TRY(check_launch("problem terms"));
  terms.resize(static_cast<size_t>(S.nprob) * 4);
  VL_HIP(hipMemcpyAsync(terms.data(), M.red_out.p, sizeof(double) * terms.size(),
                        hipMemcpyDeviceToHost, M.stream));
  return sync_stream(M.stream);
}

// rows of problems with mask[p] != 0: dst = src (mode update) / b = b_old +
// (b - b_old) / 2 (step halving)
__global__ void masked_copy_kernel(int64_t n, const int* __restrict__ row_prob,
                                   const int* __restrict__ mask, const double* __restrict__ src,
                                   double* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && mask[row_prob[i]]) dst[i] = src[i];
}
__global__ void masked_halve_kernel(int64_t n, const int* __restrict__ row_prob,
                                    const int* __restrict__ mask, const double* __restrict__ b_old,
                                    double* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && mask[row_prob[i]]) b[i] = b_old[i] + 0.5 * (b[i] - b_old[i]);
}

// X = s o eps, eps Rademacher keyed by (problem seed, tag, column, row inside
// the problem) -- the probes a solo run of each problem draws
__global__ void batch_probe_kernel(int64_t n, int t, const int* __restrict__ row_prob,
                                   const int* __restrict__ row_local,
                                   const uint64_t* __restrict__ seeds,
                                   const double* __restrict__ s, double* __restrict__ X) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * t) return;
  const int64_t i = e / t;
  const int c = static_cast<int>(e - i * t);
  X[e] = s[i] * rademacher(seeds[row_prob[i]], kTagSlq, (uint64_t)c, (uint64_t)row_local[i]);
}

CgOps vadu_ops(const double* W, const double* sdiag);

static Status apply_tune(Batch& Bt, int t) {
  int choice = 0;
  VL_TRY(autotune(Bt.M, t, &choice));
  Bt.M.force_levels = choice == 1;
  Bt.M.bd_use = choice == 2 && Bt.M.bd_ready;
  const int wc = width_class(t);
  if (static_cast<int>(Bt.tune.size()) <= wc) Bt.tune.resize(wc + 1, -1);
  Bt.tune[wc] = choice;
  return Status::ok();
}

static Status batch_fit(Batch& Bt, const vl_opts& o) {
  Model& M = Bt.M;
  const int P = Bt.P;
  const int64_t n = M.n;
  const unsigned gn = static_cast<unsigned>((n + 255) / 256);
  VL_TRY(M.mode.reserve(n));
  VL_TRY(M.mode_old.reserve(n));
  VL_TRY(M.W.reserve(n));
  VL_TRY(M.g.reserve(n));
  VL_TRY(M.vec_a.reserve(n));
  VL_TRY(M.vec_b.reserve(n));
  VL_TRY(Bt.pmask.reserve(P));
  VL_TRY(fill_double(M.mode.p, 0.0, n, M.stream));
  std::vector<int> pm(P, 1), conv(P, 0);
  Bt.newton_iters.assign(P, 0);
  Bt.halvings_total.assign(P, 0);
  std::vector<double> terms, psi_old(P), psi_new(P);
  VL_TRY(problem_terms(Bt, M.mode.p, nullptr, terms));
  for (int p = 0; p < P; ++p) psi_old[p] = terms[4 * p] - 0.5 * terms[4 * p + 1];
  // ---- Newton, all problems in lockstep (eq. newton with eq. pcls1)
  VL_TRY(apply_tune(Bt, 1));
  for (int it = 0; it < o.max_newton; ++it) {
    int live = 0;
    for (int p = 0; p < P; ++p) live += pm[p];
    if (!live) break;
    VL_HIP(hipMemcpyAsync(Bt.pmask.p, pm.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                          M.stream));
    VL_TRY(lik_rows(M, M.mode.p, M.g.p, M.W.p, M.vec_a.p, M.vec_b.p, nullptr, nullptr));
    VL_TRY(copy_d2d(M.mode_old.p, M.mode.p, sizeof(double) * n, M.stream));
    CgOps ops = vadu_ops(M.W.p, M.vec_b.p);
    VL_TRY(seg_cg(Bt, Bt.seg1, ops, M.vec_a.p, o.cg_tol, o.max_cg));
    hipLaunchKernelGGL(masked_copy_kernel, dim3(gn), dim3(256), 0, M.stream, n, Bt.row_prob.p,
                       Bt.pmask.p, Bt.cg.U.p, M.mode.p);
    VL_TRY(check_launch("batch mode update"));
    for (int p = 0; p < P; ++p) Bt.newton_iters[p] += pm[p];
    VL_TRY(problem_terms(Bt, M.mode.p, nullptr, terms));
    for (int p = 0; p < P; ++p) psi_new[p] = terms[4 * p] - 0.5 * terms[4 * p + 1];
    // per-problem step halving (the rule of the solo Newton iteration)
    std::vector<int> hv(P, 0), hmask(P, 0);
    for (int h = 0; h < 30; ++h) {
      int any = 0;
      for (int p = 0; p < P; ++p) {
        const double floor_psi = psi_old[p] - 1e-12 * std::fabs(psi_old[p]);
        hmask[p] = pm[p] && !(psi_new[p] >= floor_psi);
        any += hmask[p];
      }
      if (!any) break;
      VL_HIP(hipMemcpyAsync(Bt.pmask.p, hmask.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                            M.stream));
      hipLaunchKernelGGL(masked_halve_kernel, dim3(gn), dim3(256), 0, M.stream, n,
                         Bt.row_prob.p, Bt.pmask.p, M.mode_old.p, M.mode.p);
      VL_TRY(check_launch("batch halve"));
      VL_TRY(problem_terms(Bt, M.mode.p, nullptr, terms));
      for (int p = 0; p < P; ++p) {
        if (!hmask[p]) continue;
        psi_new[p] = terms[4 * p] - 0.5 * terms[4 * p + 1];
        ++hv[p];
      }
    }
    std::vector<int> restore(P, 0);
    int any_restore = 0;
    for (int p = 0; p < P; ++p) {
      if (!pm[p]) continue;
      Bt.halvings_total[p] += hv[p];
      const double floor_psi = psi_old[p] - 1e-12 * std::fabs(psi_old[p]);
      if (!(psi_new[p] >= floor_psi)) {
        restore[p] = 1;
        any_restore = 1;
        conv[p] = 1;
        pm[p] = 0;
      } else if (std::fabs(psi_new[p] - psi_old[p]) <= o.newton_tol * std::fabs(psi_old[p])) {
        conv[p] = 1;
        pm[p] = 0;
      } else {
        psi_old[p] = psi_new[p];
      }
    }
    if (any_restore) {
      VL_HIP(hipMemcpyAsync(Bt.pmask.p, restore.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                            M.stream));
      hipLaunchKernelGGL(masked_copy_kernel, dim3(gn), dim3(256), 0, M.stream, n,
                         Bt.row_prob.p, Bt.pmask.p, M.mode_old.p, M.mode.p);
      VL_TRY(check_launch("batch restore"));
    }
  }
  // ---- SLQ negative log-marginal likelihood per problem (eqs. VLA_loss,
  // logdetsplit, def_SLQ) with t probes each
  const int t = o.num_probes;
  VL_TRY(M.vec_c.reserve(n));
  VL_TRY(lik_rows(M, M.mode.p, nullptr, M.W.p, nullptr, M.vec_b.p, M.vec_c.p, nullptr));
  std::vector<int> all(P, 1);
  VL_HIP(hipMemcpyAsync(Bt.pmask.p, all.data(), sizeof(int) * P, hipMemcpyHostToDevice,
                        M.stream));
  VL_TRY(apply_tune(Bt, t));
  VL_TRY(M.rhs_blk.reserve(static_cast<size_t>(n) * t));
  VL_TRY(M.mx_a.reserve(static_cast<size_t>(n) * t));
  hipLaunchKernelGGL(batch_probe_kernel, dim3((unsigned)((n * t + 255) / 256)), dim3(256), 0,
                     M.stream, n, t, Bt.row_prob.p, Bt.row_local.p, Bt.prob_seed.p, M.vec_c.p,
                     M.mx_a.p);
  VL_TRY(check_launch("batch probes"));
  VL_TRY(spmm_bt(M, M.mx_a.p, M.rhs_blk.p, t, nullptr, nullptr));
  CgOps ops = vadu_ops(M.W.p, M.vec_b.p);
  VL_TRY(seg_cg(Bt, Bt.segt, ops, M.rhs_blk.p, o.cg_tol, o.max_cg));
  M.force_levels = false;
  M.bd_use = false;
  const int q = P * t;
  VL_TRY(M.red_out.reserve(2 * static_cast<size_t>(q) + 64));
  VL_TRY(tridiag_quadrature(M, Bt.cg, M.red_out.p));
  std::vector<double> quad(q), r0z0(q);
  VL_HIP(hipMemcpyAsync(quad.data(), M.red_out.p, sizeof(double) * q, hipMemcpyDeviceToHost,
                        M.stream));
  VL_HIP(hipMemcpyAsync(r0z0.data(), Bt.cg.r0z0.p, sizeof(double) * q, hipMemcpyDeviceToHost,
                        M.stream));
  VL_TRY(sync_stream(M.stream));
  VL_TRY(read_status(M));
  VL_TRY(problem_terms(Bt, M.mode.p, M.W.p, terms));
  Bt.nll.assign(P, 0.0);
  Bt.slq_iters_max.assign(P, 0);
  for (int p = 0; p < P; ++p) {
    double gamma = 0.0;
    for (int c = 0; c < t; ++c) {
      gamma += r0z0[p * t + c] * quad[p * t + c];
      Bt.slq_iters_max[p] = std::max(Bt.slq_iters_max[p], Bt.cg.host_iters[p * t + c]);
    }
    gamma /= t;
    const double logdet = terms[4 * p + 2] + terms[4 * p + 3] + gamma;
    Bt.nll[p] = -terms[4 * p] + 0.5 * terms[4 * p + 1] + 0.5 * logdet;
  }
  M.has_mode = true;
  return Status::ok();
}

// ------------------------------------------------------------------ build
__global__ void pack_rows_kernel(int64_t n, int m, int mmax, int64_t start,
                                 const int* __restrict__ nbr, const double* __restrict__ bval,
                                 const double* __restrict__ dval, const int* __restrict__ order,
                                 int* __restrict__ pnbr, double* __restrict__ pbval,
                                 double* __restrict__ pdval, int* __restrict__ porder) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < mmax; ++k) {
    const int j = k < m ? nbr[i * m + k] : -1;
    pnbr[(start + i) * mmax + k] = j >= 0 ? static_cast<int>(start + j) : -1;
    pbval[(start + i) * mmax + k] = j >= 0 ? bval[i * m + k] : 0.0;
  }
  pdval[start + i] = dval[i];
  porder[start + i] = static_cast<int>(start + order[i]);
}

static Status batch_create(const vl_problem* probs, int P, int lik, double aux, hipStream_t stream,
                           Batch** out) {
  *out = nullptr;
  if (!probs || P < 1) return Status::invalid("no problems");
  auto bt = std::unique_ptr<Batch>(new Batch());
  Batch& B = *bt;
  Model& M = B.M;
  VL_HIP(hipGetDevice(&M.device));
  VL_HIP(hipDeviceGetAttribute(&M.num_cus, hipDeviceAttributeMultiprocessorCount, M.device));
  M.stream = stream;
  B.P = P;
  B.lik = lik;
  B.aux = aux;
  int64_t total = 0;
  int mmax = 0;
  for (int p = 0; p < P; ++p) {
    const vl_problem& q = probs[p];
    if (!q.coords || !q.y) return Status::invalid("problem without coordinates or responses");
    if (q.n < 1 || q.m < 0 || q.m > 31) return Status::invalid("problem size out of range");
    if (q.cov != VL_COV_EXPONENTIAL && q.cov != VL_COV_MATERN32)
      return Status::invalid("unknown covariance");
    if (!(q.theta[0] > 0.0) || !(q.theta[1] > 0.0)) return Status::invalid("theta must be positive");
    B.start.push_back(total);
    B.n.push_back(q.n);
    B.m.push_back(q.m);
    B.seed.push_back(q.seed);
    total += q.n;
    mmax = std::max(mmax, q.m);
  }
  if (total * static_cast<int64_t>(mmax > 0 ? mmax : 1) >= (int64_t(1) << 31))
    return Status::invalid("packed size too large");
  // A 256-problem batch (3.2e6 packed rows) ended in a GPU memory fault whose
  // cause is not found yet; until it is, batches stay within the verified
  // size.
  if (P > kBatchMaxProblems || total > kBatchMaxRows)
    return Status::invalid("batch larger than the verified limit (32 problems, 65536 rows)");
  M.n = total;
  M.m = mmax;
  M.lik = lik;
  M.aux = aux;
  VL_TRY(M.status_buf.alloc(4));
  M.status = M.status_buf.p;
  VL_TRY(fill_int(M.status, 0, 4, stream));
  VL_TRY(M.coords_buf.alloc(2 * static_cast<size_t>(total)));
  M.coords = M.coords_buf.p;
  VL_TRY(M.nbr.alloc(static_cast<size_t>(total) * (mmax > 0 ? mmax : 1)));
  VL_TRY(M.bval.alloc(static_cast<size_t>(total) * (mmax > 0 ? mmax : 1)));
  VL_TRY(M.dval.alloc(total));
  VL_TRY(M.dinv.alloc(total));
  VL_TRY(M.y.alloc(total));
  VL_TRY(M.F.alloc(total));
  VL_TRY(M.ws_alloc(&M.grid_pts, sizeof(int) * total));
  std::vector<int> rp(total), rl(total);
  for (int p = 0; p < P; ++p) {
    const vl_problem& q = probs[p];
    const int64_t s0 = B.start[p];
    VL_TRY(copy_d2d(M.coords_buf.p + 2 * s0, q.coords, sizeof(double) * 2 * q.n, stream));
    VL_TRY(copy_d2d(M.y.p + s0, q.y, sizeof(double) * q.n, stream));
    if (q.F) {
      VL_TRY(copy_d2d(M.F.p + s0, q.F, sizeof(double) * q.n, stream));
    } else {
      VL_TRY(fill_double(M.F.p + s0, 0.0, q.n, stream));
    }
    for (int64_t i = 0; i < q.n; ++i) {
      rp[s0 + i] = p;
      rl[s0 + i] = static_cast<int>(i);
    }
    // neighbour search and factor of problem p on its own points
    Model tm;
    tm.device = M.device;
    tm.stream = stream;
    tm.n = q.n;
    tm.m = q.m;
    tm.cov = q.cov;
    tm.sigma2 = q.theta[0];
    tm.rho = q.theta[1];
    tm.status = M.status;
    tm.coords = M.coords_buf.p + 2 * s0;
    Status st = [&]() -> Status {
      VL_TRY(tm.nbr.alloc(static_cast<size_t>(q.n) * (q.m > 0 ? q.m : 1)));
      VL_TRY(tm.bval.alloc(static_cast<size_t>(q.n) * (q.m > 0 ? q.m : 1)));
      VL_TRY(tm.dval.alloc(q.n));
      VL_TRY(knn_build_grid(tm));
      VL_TRY(knn_query(tm, nullptr, q.n, tm.nbr.p));
      VL_TRY(factor_rows(tm, nullptr, q.n, tm.nbr.p, tm.bval.p, tm.dval.p, false, nullptr,
                         nullptr, nullptr));
      hipLaunchKernelGGL(pack_rows_kernel, dim3((unsigned)((q.n + 255) / 256)), dim3(256), 0,
                         stream, q.n, q.m, mmax, s0, tm.nbr.p, tm.bval.p, tm.dval.p,
                         static_cast<const int*>(tm.grid_pts), M.nbr.p, M.bval.p, M.dval.p,
                         static_cast<int*>(M.grid_pts));
      VL_TRY(check_launch("pack rows"));
      return sync_stream(stream);
    }();
    for (void* w : tm.owned) device_free(w);
    tm.owned.clear();
    VL_TRY(st);
  }
  VL_TRY(B.row_prob.alloc(total));
  VL_TRY(B.row_local.alloc(total));
  VL_TRY(B.prob_seed.alloc(P));
  VL_HIP(hipMemcpyAsync(B.row_prob.p, rp.data(), sizeof(int) * total, hipMemcpyHostToDevice,
                        stream));
  VL_HIP(hipMemcpyAsync(B.row_local.p, rl.data(), sizeof(int) * total, hipMemcpyHostToDevice,
                        stream));
  VL_HIP(hipMemcpyAsync(B.prob_seed.p, B.seed.data(), sizeof(uint64_t) * P,
                        hipMemcpyHostToDevice, stream));
  VL_TRY(read_status(M));
  // structure of the packed, block-diagonal system
  VL_TRY(build_transpose(M));
  VL_TRY(build_head_schedule(M));
  VL_TRY(build_tail_orders(M));
  VL_TRY(bd_build(M, B.start, B.n, B.row_prob.p, B.row_local.p));
  VL_TRY(finish_factor(M));
  VL_TRY(build_seg(M, B.start, B.n, 1, B.seg1));
  *out = bt.release();
  return Status::ok();
}

}  // namespace vl

struct vl_batch : public vl::Batch {};

extern "C" {

vl_status vl_batch_create(const vl_problem* problems, int nprob, int lik,
                          const double* aux_host, void* hip_stream, vl_batch** out) {
  vl::CallStream cs(static_cast<hipStream_t>(hip_stream));
  try {
    if (!out) return vl::report(vl::Status::invalid("out is null"));
    *out = nullptr;
    double aux = 0.0;
    vl::Status ls = vl::likelihood_aux(lik, aux_host, &aux);
    if (!ls.good()) return vl::report(ls);
    vl::Batch* b = nullptr;
    vl::Status s = vl::batch_create(problems, nprob, lik, aux,
                                    static_cast<hipStream_t>(hip_stream), &b);
    if (!s.good()) return vl::report(s);
    *out = static_cast<vl_batch*>(b);
    return VL_OK;
  } catch (const std::bad_alloc&) {
    return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}

vl_status vl_batch_fit(vl_batch* b, const vl_opts* o, double* nll_host) {
  vl::CallStream cs(b ? b->M.stream : nullptr);
  try {
    if (!b || !o || !nll_host) return vl::report(vl::Status::invalid("null argument"));
    if (o->num_probes < 1 || o->max_newton < 1 || o->max_cg < 1 || !(o->cg_tol > 0.0))
      return vl::report(vl::Status::invalid("bad options"));
    if (o->precond != VL_PREC_VADU || o->precision != VL_FP64)
      return vl::report(vl::Status::invalid("the batching form runs FP64 with VADU"));
    if (b->segt.t != o->num_probes) {
      vl::Status s = vl::build_seg(b->M, b->start, b->n, o->num_probes, b->segt);
      if (!s.good()) return vl::report(s);
    }
    vl::Status s = vl::batch_fit(*b, *o);
    if (!s.good()) return vl::report(s);
    for (int p = 0; p < b->P; ++p) nll_host[p] = b->nll[p];
    return VL_OK;
  } catch (const std::bad_alloc&) {
    return vl::report(vl::Status::make(VL_ERR_OOM, "host allocation failed"));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}

vl_status vl_batch_mode(vl_batch* b, int p, double* mode_out) {
  if (!b || !mode_out || p < 0 || p >= b->P) return vl::report(vl::Status::invalid("bad argument"));
  if (!b->M.has_mode) return vl::report(vl::Status::make(VL_ERR_STATE, "no fit yet"));
  vl::Status s = vl::copy_d2d(mode_out, b->M.mode.p + b->start[p], sizeof(double) * b->n[p],
                              b->M.stream);
  if (s.good()) s = vl::sync_stream(b->M.stream);
  return vl::report(s);
}

vl_status vl_batch_stats(vl_batch* b, int p, vl_stats* st) {
  if (!b || !st || p < 0 || p >= b->P) return vl::report(vl::Status::invalid("bad argument"));
  if (!b->M.has_mode) return vl::report(vl::Status::make(VL_ERR_STATE, "no fit yet"));
  std::memset(st, 0, sizeof(*st));
  st->newton_iters = b->newton_iters[p];
  st->cg_iters_max = b->slq_iters_max[p];
  st->cg_iters_total = b->halvings_total[p];
  return VL_OK;
}

int vl_batch_tuned_path(vl_batch* b, int width_class) {
  if (!b || width_class < 0 || width_class >= static_cast<int>(b->tune.size())) return -1;
  return b->tune[width_class];
}

void vl_batch_free(vl_batch* b) {
  if (!b) return;
  vl::CallStream cs(b->M.stream);
  (void)hipStreamSynchronize(b->M.stream);
  for (void* p : b->M.owned) vl::device_free(p);
  b->M.owned.clear();
  if (b->M.host_pin) (void)hipHostFree(b->M.host_pin);
  b->M.host_pin = nullptr;
  for (hipEvent_t e : b->M.timing.pool) (void)hipEventDestroy(e);
  delete b;
}

}  // extern "C"
