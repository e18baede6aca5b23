// Small device utilities: fills, a multi-block exclusive scan, launch checks.
#include <mutex>
#include <unordered_map>

#include "vl_internal.h"

namespace vl {

Status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return Status::hip(e, what);
  return Status::ok();
}

Status sync_stream(hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return Status::hip(e, "hipStreamSynchronize");
  return Status::ok();
}

// ---- device allocation ----------------------------------------------------
// Every device buffer of the library comes from here: the caller-installed
// allocator (vl_set_allocator) or, by default, the stream-ordered
// hipMallocAsync on the stream of the call in progress.  Each live pointer
// remembers who allocated it, so that a hook installed or removed while
// models exist never frees another allocator's memory.
namespace {
struct AllocOwner {
  vl_alloc_fn a = nullptr;  // nullptr: hipMallocAsync / hipFreeAsync
  vl_free_fn f = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
AllocOwner g_hook;
std::unordered_map<void*, AllocOwner> g_live;
thread_local hipStream_t g_call_stream = nullptr;
}  // namespace

CallStream::CallStream(hipStream_t s) : prev_(g_call_stream) { g_call_stream = s; }
CallStream::~CallStream() { g_call_stream = prev_; }

Status set_allocator(vl_alloc_fn a, vl_free_fn f, void* ctx) {
  if ((a == nullptr) != (f == nullptr))
    return Status::invalid("allocator and deallocator must be given together");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_hook.a = a;
  g_hook.f = f;
  g_hook.ctx = ctx;
  return Status::ok();
}

Status device_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  AllocOwner own;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    own = g_hook;
  }
  if (own.a) {
    *p = own.a(bytes, static_cast<void*>(g_call_stream), own.ctx);
    if (!*p) return Status::make(VL_ERR_OOM, "the installed allocator returned NULL");
  } else {
    hipError_t e = hipMallocAsync(p, bytes, g_call_stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return Status::make(VL_ERR_OOM, std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_live[*p] = own;
  return Status::ok();
}

void device_free(void* p) {
  if (!p) return;
  AllocOwner own;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;  // not ours
    own = it->second;
    g_live.erase(it);
  }
  if (own.f) {
    own.f(p, static_cast<void*>(g_call_stream), own.ctx);
  } else {
    (void)hipFreeAsync(p, g_call_stream);
  }
}

Status copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  VL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return Status::ok();
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, T v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned fill_grid(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return static_cast<unsigned>(g);
}

Status fill_int(int* p, int v, int64_t count, hipStream_t s) {
  if (count <= 0) return Status::ok();
  hipLaunchKernelGGL(fill_kernel<int>, dim3(fill_grid(count)), dim3(256), 0, s, p, v, count);
  return check_launch("fill_int");
}

Status fill_double(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return Status::ok();
  hipLaunchKernelGGL(fill_kernel<double>, dim3(fill_grid(count)), dim3(256), 0, s, p, v, count);
  return check_launch("fill_double");
}

// ---- exclusive scan over int: block scans, a scan of block sums, offsets
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(kScanBlock) void scan_blocks(const int* __restrict__ in,
                                                           int* __restrict__ out, int64_t count,
                                                           int* __restrict__ block_sums) {
  __shared__ int s[kScanBlock];
  int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  int v = (i < count) ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    int add = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < count) out[i] = s[threadIdx.x] - v;  // exclusive
  if (threadIdx.x == kScanBlock - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

// single block: exclusive scan of the block sums, each thread a contiguous run
__global__ __launch_bounds__(kScanBlock) void scan_sums(int* __restrict__ sums, int nb) {
  __shared__ int s[kScanBlock];
  const int per = (nb + kScanBlock - 1) / kScanBlock;
  const int b0 = threadIdx.x * per;
  int local = 0;
  for (int b = b0; b < b0 + per && b < nb; ++b) local += sums[b];
  s[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    int add = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int run = s[threadIdx.x] - local;
  for (int b = b0; b < b0 + per && b < nb; ++b) {
    int v = sums[b];
    sums[b] = run;
    run += v;
  }
}

__global__ void scan_add(int* __restrict__ out, int64_t count, const int* __restrict__ sums) {
  int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  if (i < count) out[i] += sums[blockIdx.x];
}

Status exclusive_scan_int(const int* in, int* out, int64_t count, hipStream_t s) {
  if (count <= 0) return Status::ok();
  const int64_t nb = (count + kScanBlock - 1) / kScanBlock;
  DevBuf<int> sums;
  VL_TRY(sums.alloc(nb));
  hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, count,
                     sums.p);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanBlock), 0, s, sums.p, (int)nb);
  hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, count, sums.p);
  VL_TRY(check_launch("scan"));
  return sync_stream(s);  // `sums` is released on return
}

TimedLaunch::TimedLaunch(Model& M, int kind, double bytes)
    : M_(M), on_(M.timing.on && ((M.timing.mask >> kind) & 1u)), ev_(0) {
  if (!on_) return;
  Timing& T = M.timing;
  while (T.pool.size() < T.used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      on_ = false;
      return;
    }
    T.pool.push_back(e);
  }
  ev_ = T.used;
  T.used += 2;
  T.recs.push_back({kind, ev_, bytes});
  (void)hipEventRecord(T.pool[ev_], M.stream);
}

TimedLaunch::~TimedLaunch() {
  if (on_) (void)hipEventRecord(M_.timing.pool[ev_ + 1], M_.stream);
}

static std::mutex g_poll_mu;
static hipEvent_t g_poll_last = nullptr;
static int g_poll_dev = -1;

PollingOrder::PollingOrder(Model& M) : M_(M) {
  g_poll_mu.lock();
  if (!M.poll_evt && hipEventCreateWithFlags(&M.poll_evt, hipEventDisableTiming) != hipSuccess) {
    M.poll_evt = nullptr;
    (void)hipGetLastError();
  }
  if (g_poll_last && g_poll_last != M.poll_evt && g_poll_dev == M.device)
    (void)hipStreamWaitEvent(M.stream, g_poll_last, 0);
}

PollingOrder::~PollingOrder() {
  if (M_.poll_evt && hipEventRecord(M_.poll_evt, M_.stream) == hipSuccess) {
    g_poll_last = M_.poll_evt;
    g_poll_dev = M_.device;
  }
  g_poll_mu.unlock();
}

// The event may still be the last one in the order: forget it first.  The
// owner has synchronised its stream, so the event has completed.
Model::~Model() {
  if (!poll_evt) return;
  {
    std::lock_guard<std::mutex> lk(g_poll_mu);
    if (g_poll_last == poll_evt) g_poll_last = nullptr;
  }
  (void)hipEventDestroy(poll_evt);
}

Status read_status(Model& M) {
  int st = 0;
  VL_HIP(hipMemcpyAsync(&st, M.status, sizeof(int), hipMemcpyDeviceToHost, M.stream));
  VL_TRY(sync_stream(M.stream));
  if (st == 0) return Status::ok();
  VL_HIP(hipMemsetAsync(M.status, 0, sizeof(int), M.stream));
  if (st & kErrNotSpd)
    return Status::make(VL_ERR_NOT_SPD, "a neighbour covariance is not positive definite");
  if (st & kErrTimeout)
    return Status::make(VL_ERR_TIMEOUT, "a sync-free solve exceeded its wait bound");
  return Status::make(VL_ERR_NONFINITE, "non-finite value in a device computation");
}

}  // namespace vl
