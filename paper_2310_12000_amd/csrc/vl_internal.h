// Host-side internals of the library: the model handle, status values,
// device buffers and the declarations shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vl.h"
#include "vl_device.h"

namespace vl {

struct Status {
  vl_status code = VL_OK;
  std::string msg;
  static Status ok() { return Status(); }
  static Status make(vl_status c, const std::string& m) {
    Status s;
    s.code = c;
    s.msg = m;
    return s;
  }
  static Status invalid(const std::string& m) { return make(VL_ERR_INVALID_ARG, m); }
  static Status hip(hipError_t e, const char* where) {
    return make(VL_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
  }
  bool good() const { return code == VL_OK; }
};

#define VL_TRY(expr)                          \
  do {                                        \
    ::vl::Status _st = (expr);                \
    if (!_st.good()) return _st;              \
  } while (0)

#define VL_HIP(expr)                                              \
  do {                                                            \
    hipError_t _e = (expr);                                       \
    if (_e != hipSuccess) return ::vl::Status::hip(_e, #expr);    \
  } while (0)

Status check_launch(const char* what);
Status sync_stream(hipStream_t s);
Status device_alloc(void** p, size_t bytes);
void device_free(void* p);
Status set_allocator(vl_alloc_fn a, vl_free_fn f, void* ctx);

// The stream of the entry point in progress on this host thread: default
// allocations are ordered on it, and an installed allocator receives it.
class CallStream {
 public:
  explicit CallStream(hipStream_t s);
  ~CallStream();
  CallStream(const CallStream&) = delete;
  CallStream& operator=(const CallStream&) = delete;

 private:
  hipStream_t prev_;
};

// RAII device buffer for temporaries of one call.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t count = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  Status alloc(size_t n) {
    release();
    if (n == 0) n = 1;
    void* q = nullptr;
    VL_TRY(device_alloc(&q, n * sizeof(T)));
    p = static_cast<T*>(q);
    count = n;
    return Status::ok();
  }
  // grow-only
  Status reserve(size_t n) {
    if (n <= count && p) return Status::ok();
    return alloc(n);
  }
  void release() {
    if (p) device_free(p);
    p = nullptr;
    count = 0;
  }
  void swap(DevBuf& o) {
    T* q = p;
    p = o.p;
    o.p = q;
    const size_t c = count;
    count = o.count;
    o.count = c;
  }
};

struct GridGeom {
  double x0, y0, h, slack;
  int G;
};

// Grouped form of B or B^T for products over blocks of many columns: rows
// in groups of kGroupRows consecutive positions of the spatial order; per
// group the sorted union of the columns its rows touch (padded), and a dense
// kGroupRows-wide weight column per union entry.
#ifndef VL_GROUP_ROWS
#define VL_GROUP_ROWS 4
#endif
constexpr int kGroupRows = VL_GROUP_ROWS;
#ifndef VL_GROUP_MIN_T
#define VL_GROUP_MIN_T 32
#endif
constexpr int kGroupMinT = VL_GROUP_MIN_T;  // block widths that use them
constexpr int kGroupMaxT = 64;
struct GroupOp {
  DevBuf<int> ptr;    // groups + 1 padded union offsets
  DevBuf<int> col;    // union columns, ascending per group
  DevBuf<int> cnt;    // union length per group before padding
  DevBuf<double> w;   // union entries x kGroupRows weights
  DevBuf<int> pos;    // per B entry (i, k): its index in w, -1 for empty slots
  int64_t cols = 0;   // padded union entries in all
  void reset() {
    ptr.release();
    col.release();
    cnt.release();
    w.release();
    pos.release();
    cols = 0;
  }
};

// State of one block CG solve (t columns).
struct CgState {
  int t = 0;
  int lmax = 0;
  DevBuf<double> U, R, Z, H, V, Tmp, Y, Z0;   // n x t each
  DevBuf<double> rz, rr, alpha, beta, r0z0;   // t each
  DevBuf<double> hist_a, hist_b;              // lmax x t
  DevBuf<double> tri;                         // 3 lmax x t (tridiagonal work)
  DevBuf<int> active, iters;                  // t each
  DevBuf<int> forced;                         // t replayed iteration counts
  DevBuf<int> num_active;                     // 1
  DevBuf<double> part_a, part_b;              // nchunk x t partial sums
  std::vector<int> host_iters;
};

// Optional event timing of kernel classes (measurement only).
enum TimedKind : int {
  kTimeSpmmB = 0,     // Y = B X (ELL)
  kTimeSpmmBt = 1,    // Y = B^T X (CSR)
  kTimeTrsmLower = 2, // sync-free rows of B Y = X
  kTimeTrsmUpper = 3, // sync-free rows of B^T Y = X
  kTimeDenseLower = 4, // dense products of B Y = X (leading block, per-problem inverses)
  kTimeDenseUpper = 5, // dense products of B^T Y = X (leading block, per-problem inverses)
  kTimeLevelLower = 6, // level-scheduled rows of B Y = X (wide blocks)
  kTimeLevelUpper = 7, // level-scheduled rows of B^T Y = X (wide blocks)
  kTimeLevelUpperSplit = 8, // the same for levels of long B^T rows
  kTimeLevelUpperFold = 9,  // head rows' tail entries of B^T Y = X, one launch
  kTimeDenseWide = 10,      // leading rows of the wide solves (dense inverse, matrix cores)
  kTimeKinds = 11
};

struct Timing {
  bool on = false;
  unsigned mask = 0;  // kinds recorded while on (bit k = kind k)
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int kind;
    size_t ev;
    double bytes;
  };
  std::vector<Rec> recs;
};

struct Model {
  int device = 0;
  int num_cus = 1;
  // Work streams of a sync-free solve at most (0 = no cap).  Solves of
  // models that run concurrently on one GPU together need every stream of
  // every solve to keep a resident wave: their caps must add up to at most
  // the CU count (the serving loop sets CUs / slots).
  int max_streams = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int m = 0;
  int cov = 0;
  double sigma2 = 1.0, rho = 1.0;
  bool deriv = false;

  DevBuf<double> coords_buf;  // n x 2
  const double* coords = nullptr;
  DevBuf<int> nbr;            // n x m
  DevBuf<double> bval;        // n x m, B entries (-A)
  DevBuf<double> dval;        // n
  DevBuf<double> dinv;        // n
  DevBuf<double> dbval_rho;   // n x m (dB/drho); dB/dsigma2 = 0
  DevBuf<double> dd_sigma2, dd_rho;  // n
  // B^T in CSR
  int64_t nnz = 0;
  DevBuf<int> bt_ptr, bt_col, bt_src;
  DevBuf<double> bt_val;
  DevBuf<float> bval_f, bt_val_f;  // FP32 copies for the mixed-precision form
  int64_t factor_version = 0, f32_version = -1;  // FP32 copies made at factor_version
  bool force_levels = false;  // level-scheduled solves for every block width (autotuner)

  // head rows 0..head_rows-1: the wide blocks' B^T solve takes them after the
  // tail (level schedules below); the rows below dense_rows are solved with
  // the dense inverse of B's leading block (dense.hip), in both directions and
  // at every width (dense_wide of them for wide blocks)
  int head_rows = 0;
  int dense_rows = 0;
  DevBuf<double> dense_gf, dense_gb;  // G = B_KK^{-1}: column-major, row-major
  DevBuf<double> dense_xp;            // K x t folded right-hand sides of B^T solves
  DevBuf<double> dense_part;          // partial products of the dense applications
  DevBuf<int> dense_lo;               // first B^T entry with child >= K, rows < K
  // wide blocks (t > 64): the leading dense_wide rows from G's leading block
  // (matrix cores), the level schedules of the other rows with those known
  int dense_wide = 0;
  DevBuf<int> dense_lo_w;             // as dense_lo for dense_wide
  DevBuf<int> dfull_order_f;          // rows dense_wide..n-1 in forward level order
  std::vector<int> dlvl_ptr_f;
  std::vector<int64_t> dlvl_nnz_f;
  DevBuf<int> dhlv_rows_b;            // head rows dense_wide..H-1, backward levels
  std::vector<int> dhlv_ptr_b;
  std::vector<int64_t> dhlv_nnz_b;
  // packed block-diagonal systems of small problems (batching): every
  // problem's B inverted whole, solves as per-problem dense products
  bool bd_ready = false, bd_use = false;
  int bd_C = 1, bd_kmax = 0, bd_inv_n = 0, bd_lo_n = 0, bd_up_n = 0;
  int64_t bd_part_rows = 0;
  DevBuf<int> bd_start;                       // P + 1 packed row starts
  DevBuf<int64_t> bd_gofs, bd_pofs;           // G and partial offsets per problem
  DevBuf<int> bd_inv_p, bd_inv_c0;            // inverse blocks
  DevBuf<int> bd_lo_p, bd_lo_chunk, bd_lo_seg;  // product blocks, G x
  DevBuf<int> bd_up_p, bd_up_chunk, bd_up_seg;  // product blocks, G^T x
  DevBuf<double> bd_gf, bd_gb, bd_part;
  const int* bd_row_prob = nullptr;           // packed row -> problem
  const int* bd_row_local = nullptr;          // packed row -> row in its problem
  // sync-free tails of narrow blocks: rows >= dense_rows in level order, per
  // direction, and the number of dependency levels each spans
  DevBuf<int> tail_order_f, tail_order_bn;
  int tail_levels_f = 0, tail_levels_b = 0;
  int nnz_bt_dense = 0;  // B^T entries of the rows below dense_rows
  // B's rows with their slots in the forward tail's consumption order
  DevBuf<int> tnbr, tsrc;
  DevBuf<double> tval;
  DevBuf<int> tail_order_b;  // rows >= head_rows, backward level order (wide blocks)
  DevBuf<int> full_order_f, full_order_b;       // all rows in level order
  // level l of the full orders = positions [lvl_ptr[l], lvl_ptr[l + 1]); nnz
  // of the rows of each level (host copies, for the level-scheduled solves)
  std::vector<int> lvl_ptr_f, lvl_ptr_b;
  std::vector<int64_t> lvl_nnz_f, lvl_nnz_b;
  DevBuf<int> head_split;                       // first tail entry of head B^T rows
  // Level-scheduled B^T solves run in three stages: the tail rows by level
  // (tail_order_b, tlvl_*), one fold of every head row's tail entries, then
  // the head rows by their head-internal levels (hlv_rows_b, hlv_*).
  std::vector<int> tlvl_ptr_b, hlv_ptr_b;
  std::vector<int64_t> tlvl_nnz_b, hlv_nnz_b;
  DevBuf<int> hlv_rows_b;
  int64_t fold_nnz = 0;                         // tail entries of the head rows
  DevBuf<double> lvl_fold;                      // head rows' folded right-hand sides
  // grouped products for wide blocks (group.hip); off when a group would
  // gather more columns than its build can sort
  bool grp_ok = false;
  int64_t grp_count = 0;
  GroupOp grp_b, grp_bt;

  // neighbour-search grid
  int grid_G = 0;
  void* grid_geom = nullptr;
  void* grid_start = nullptr;
  void* grid_pts = nullptr;
  void* grid_xy = nullptr;
  std::vector<void*> owned;  // released by vl_free
  Status ws_alloc(void** p, size_t bytes) {
    VL_TRY(device_alloc(p, bytes));
    owned.push_back(*p);
    return Status::ok();
  }

  // Lanczos coefficients (alpha, beta) of the last Lanczos prediction
  std::vector<double> last_lanczos_alpha, last_lanczos_beta;

  // gradient of the last likelihood call in the offset F (n), when asked
  DevBuf<double> grad_F;
  bool has_grad_F = false;
  // and in the likelihood's auxiliary parameter (Gaussian, Gamma)
  double grad_xi = 0.0;
  bool has_grad_xi = false;

  // likelihood state
  bool has_mode = false;
  int lik = 0;
  double aux = 0.0;
  DevBuf<double> y, F, mode, W, g, mode_old;

  // wall time (us) of the latest factor build, mode, likelihood and
  // prediction call, and the FP32 preconditioner deviation of the latest
  // mixed-precision block solve
  double t_build_us = 0, t_mode_us = 0, t_slq_us = 0, t_pred_us = 0;
  double last_f32_dev = 0;
  DevBuf<double> mx_chk;  // 3 n FP64 + 2 n FP32: the deviation check's vectors

  // diagnostics
  DevBuf<int> status_buf;
  int* status = nullptr;
  std::vector<int> newton_cg_iters;
  std::vector<int> newton_halvings;  // step halvings per Newton iteration
  std::vector<int> last_block_iters;
  std::vector<double> last_quad, last_r0z0;
  DevBuf<int> pred_nbr;
  DevBuf<double> pred_bval, pred_dval;
  int64_t last_np = 0;

  // reusable workspaces
  CgState cg;
  CgState cg1;  // single-column solves
  DevBuf<float> mx_rhs, mx_f2;    // n x t FP32 blocks of the mixed-precision solves
  DevBuf<double> mx_a;            // n x t FP64 scratch (batched probes)
  DevBuf<double> red_part;  // partial sums of reductions
  DevBuf<double> red_out;
  DevBuf<double> vec_a, vec_b, vec_c, vec_d, vec_e, dWv;  // n-length scratch vectors
  // LRAC preconditioner: pivoted Cholesky factor (n x lrac_K, zero columns
  // past lrac_k), pivots, I + L^T W L (factored in place; log det after it)
  bool lrac_ready = false;
  int lrac_k = 0, lrac_K = 0;
  DevBuf<double> lrac_L, lrac_pval, lrac_part, lrac_gpart, lrac_M, lrac_S, lrac_S2, lrac_Minv;
  // d L / d theta (2 x n x lrac_K, sigma2 then rho), the residual diagonals'
  // derivatives (2 x n) and the pivots' values of them per column
  bool lrac_dL_ready = false;
  DevBuf<double> lrac_dL, lrac_dd, lrac_snap;
  DevBuf<int> lrac_piv;
  DevBuf<double> rhs_blk;  // n x t right-hand sides of block solves
  DevBuf<int> counter;     // dynamic work counters of sync-free kernels
  // Scratch supplied for the call in progress by the allocation-free entry
  // point: while set, the solves of t <= 64 columns take their work counters
  // and dense-product buffers from it and reserve nothing.
  struct ExtScratch {
    int* counter = nullptr;   // one counter slot (kSlotInts ints)
    double* part = nullptr;   // partial products of the dense leading block
    size_t part_count = 0;
    double* xp = nullptr;     // folded right-hand sides of the B^T dense block
    size_t xp_count = 0;
  };
  const ExtScratch* ext = nullptr;
  double* host_pin = nullptr;  // pinned host scalars (64 doubles)
  hipEvent_t poll_evt = nullptr;  // completion of this model's last polling kernel
  Timing timing;
  ~Model();  // releases poll_evt (util.hip)
};

// Records the message of a failed status for vl_last_error (api.hip).
vl_status report(const Status& s);

// Brackets one kernel launch with events when timing is enabled.
class TimedLaunch {
 public:
  TimedLaunch(Model& M, int kind, double bytes);
  ~TimedLaunch();

 private:
  Model& M_;
  bool on_;
  size_t ev_;
};

// Kernels whose blocks wait on one another (the sync-free solves and the
// level computation) need every one of their work streams to have a
// resident block.  Two such kernels running at once on a device (models on
// different streams) could each hold the compute units the other's
// undispatched blocks need, so they are enqueued in one device-wide order:
// each waits for the completion of the previous one.  Kernels that never
// wait keep overlapping; they always finish, so the waiting kernel's blocks
// are dispatched in the end.  Construct around the launch.
class PollingOrder {
 public:
  explicit PollingOrder(Model& M);
  ~PollingOrder();

 private:
  Model& M_;
};

// ---- utilities (util.hip)
Status fill_int(int* p, int v, int64_t count, hipStream_t s);
Status fill_double(double* p, double v, int64_t count, hipStream_t s);
Status exclusive_scan_int(const int* in, int* out, int64_t count, hipStream_t s);
Status copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s);
Status read_status(Model& M);
// Validates a likelihood code and takes its parameter from aux_host[0]
// (Gaussian noise variance or Gamma shape; 0 for the others).
Status likelihood_aux(int lik, const double* aux_host, double* aux);
inline bool lik_has_aux(int lik) { return lik == VL_LIK_GAUSSIAN || lik == VL_LIK_GAMMA; }

// ---- neighbour search (knn.hip)
Status knn_build_grid(Model& M);
Status knn_query(Model& M, const double* q_xy, int64_t nq, int* nbr_out);

// ---- factor (factor.hip)
Status factor_rows(Model& M, const double* q_xy, int64_t nrows, const int* nbr, double* bval,
                   double* dval, bool deriv, double* dbval_rho, double* dd_sigma2,
                   double* dd_rho);

// ---- sparse kernels (sparse.hip)
Status build_transpose(Model& M);
Status refresh_transpose_values(Model& M);
Status build_tail_orders(Model& M);
// out_j = base_j - sum over the B^T entries [beg[j], end[j]) of B^T row j
// (values from Y), rows j < rows, wide blocks.
Status fold_rows(Model& M, int rows, const int* beg, const int* end, const double* base,
                 const double* Y, double* out, int t);
Status fold_rows(Model& M, int rows, const int* beg, const int* end, const double* base,
                 const float* Y, double* out, int t);  // FP32 Y and B^T values

// Y = rowscale o (X + B_off X)                              (spmm_b)
// Y = diag o diagvec + X + B_off^T X                         (spmm_bt)
Status spmm_b(Model& M, const double* X, double* Y, int t, const double* rowscale);
Status spmm_bt(Model& M, const double* X, double* Y, int t, const double* diag,
               const double* diagvec);
// triangular solves: B Y = rowscale o X (lower) / B^T Y = X (upper)
Status trsm_b(Model& M, const double* X, double* Y, int t, const double* rowscale,
              bool prefilled);
Status trsm_bt(Model& M, const double* X, double* Y, int t, bool prefilled);
int spmm_nblocks(int64_t n, int t);

// ---- grouped products (group.hip)
Status build_groups(Model& M);
Status refresh_group_values(Model& M);
bool group_spmm_ok(const Model& M, int t);
Status spmm_group_b(Model& M, const double* X, double* Y, int t, const double* rs);
Status spmm_group_bt(Model& M, const double* X, double* Y, int t, const double* d,
                     const double* V);

// ---- head schedules of the wide B^T solves (head.hip)
constexpr int kHeadRows = 12288;  // with the dense first 4096 rows (measured best at n = 1e5)
Status build_head_schedule(Model& M);

// ---- dense leading block (dense.hip)
constexpr int kDenseRows = 4096;
constexpr int kDenseWide = 2048;  // leading rows taken from G by the wide solves
Status dense_wide_lower(Model& M, const double* X, double* Y, int t, const double* rs);
Status dense_wide_upper(Model& M, const double* Xh, double* Y, int t);
Status dense_wide_lower_f32(Model& M, const float* X, float* Y, double* Yd, int t,
                            const double* rs);
Status dense_wide_upper_f32(Model& M, const double* Xh, float* Y, int t);
// block-diagonal form (batching): available when every problem has at most
// kDenseRows rows and the dense blocks fit in kBdBytesCap bytes
constexpr double kBdBytesCap = 8e9;
Status bd_build(Model& M, const std::vector<int64_t>& start, const std::vector<int64_t>& n,
                const int* row_prob, const int* row_local);
Status bd_lower(Model& M, const double* X, double* Y, int t, const double* rs);
Status bd_upper(Model& M, const double* X, double* Y, int t);
Status build_dense(Model& M);
Status dense_factor(Model& M);
Status dense_lower(Model& M, const double* X, double* Y, int t, const double* rs);
Status dense_upper(Model& M, const double* X, double* Y, int t);
Status dense_lower_f32(Model& M, const float* X, float* Y, int t, const double* rs);
Status dense_upper_f32(Model& M, const double* X, float* Y, int t);

// ---- solver kernels (solver.hip)
Status tridiag_quadrature(Model& M, CgState& S, double* out_dev);

}  // namespace vl
