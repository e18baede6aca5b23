// Triangular solves with the Vecchia factor that allocate no device memory,
// for callers that cannot allocate (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).  They run the kernels of vl_trsm
// for blocks of at most 64 columns; the scratch those kernels need beyond
// the inputs and outputs (the work-stream counters and abort flag of the
// sync-free rows, the segment partials of the dense leading block and the
// folded right-hand sides of its B^T product) comes from one fixed device
// array per GPU instead of the model's workspaces.
//
// Every call on a GPU shares that GPU's array, and the array keeps the last
// call's contents: each call resets its counters with a kernel before the
// solve and writes every partial it reads, so nothing depends on what an
// earlier call left.  Calls that overlap on one GPU (two streams, two host
// threads) race on the array.
#include <mutex>

#include "vl_internal.h"
#include "vl_ops.h"

namespace vl {

Model* model_of(vl_model* h);

constexpr size_t kNoAllocScratchBytes = size_t(40) << 20;  // 40 MiB per GPU
constexpr int kNoAllocMaxT = 64;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[kNoAllocMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (the array's name is a host-side stand-in).
static Status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return Status::invalid("device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    int cur = 0;
    VL_HIP(hipGetDevice(&cur));
    if (cur != dev) VL_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return Status::hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return Status::make(VL_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_dev[dev]);
  return Status::ok();
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of scratch a solve of t columns needs on model M.
static size_t noalloc_bytes(const Model& M, int t, size_t* part_off, size_t* xp_off,
                            size_t* part_count, size_t* xp_count) {
  const size_t K = static_cast<size_t>(M.dense_rows);
  const size_t nseg = (K + 255) / 256;
  *part_count = nseg * K * static_cast<size_t>(t);
  *xp_count = K * static_cast<size_t>(t);
  *part_off = align256(sizeof(int) * kSlotInts);
  *xp_off = *part_off + align256(sizeof(double) * (*part_count > 0 ? *part_count : 1));
  return *xp_off + align256(sizeof(double) * (*xp_count > 0 ? *xp_count : 1));
}

static Status trsm_noalloc(Model& M, int transpose, const double* X, double* Y, int t) {
  if (t < 1) return Status::invalid("t must be positive");
  if (t > kNoAllocMaxT) return Status::invalid("t above 64: the allocation-free solve covers at most 64 columns");
  if (M.bd_use || M.force_levels)
    return Status::make(VL_ERR_STATE, "the allocation-free solve needs the single-model schedules");
  size_t part_off, xp_off, part_count, xp_count;
  const size_t need = noalloc_bytes(M, t, &part_off, &xp_off, &part_count, &xp_count);
  if (need > kNoAllocScratchBytes)
    return Status::invalid("the solve needs more scratch than the fixed 40 MiB array holds");
  unsigned char* base = nullptr;
  VL_TRY(scratch_address(M.device, &base));
  Model::ExtScratch ext;
  ext.counter = reinterpret_cast<int*>(base);
  ext.part = reinterpret_cast<double*>(base + part_off);
  ext.part_count = part_count;
  ext.xp = reinterpret_cast<double*>(base + xp_off);
  ext.xp_count = xp_count;
  M.ext = &ext;
  Status s = transpose ? trsm_bt(M, X, Y, t, false) : trsm_b(M, X, Y, t, nullptr, false);
  M.ext = nullptr;
  VL_TRY(s);
  VL_TRY(sync_stream(M.stream));
  return read_status(M);
}

}  // namespace vl

extern "C" vl_status vl_trsm_noalloc(vl_model* h, int transpose, const double* X, double* Y,
                                     int t) {
  try {
    if (!h || !X || !Y) return vl::report(vl::Status::invalid("null argument"));
    return vl::report(vl::trsm_noalloc(*vl::model_of(h), transpose, X, Y, t));
  } catch (...) {
    return vl::report(vl::Status::make(VL_ERR_HIP, "unexpected exception"));
  }
}
