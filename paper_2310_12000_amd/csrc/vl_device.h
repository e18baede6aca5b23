// Device-side building blocks shared by the gfx950 kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vl {

constexpr int kWave = 64;

// A value that arithmetic never produces: a negative signalling NaN with a
// fixed payload.  Sync-free triangular solves pre-fill their output with it;
// a consumer treats a neighbour's value as ready once it differs.
constexpr unsigned long long kSentinelBits = 0xFFF4DEADBEEFCAFEull;

__device__ __forceinline__ double sentinel() {
  return __longlong_as_double(static_cast<long long>(kSentinelBits));
}
__device__ __forceinline__ bool is_sentinel(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v)) == kSentinelBits;
}
__device__ __forceinline__ float sentinel_f() { return __int_as_float(0xFFA5BEEF); }
__device__ __forceinline__ bool is_sentinel(float v) {
  return static_cast<unsigned>(__float_as_int(v)) == 0xFFA5BEEFu;
}

// The sentinel of a storage type (double; float in the mixed-precision form).
template <typename T>
__device__ __forceinline__ T sentinel_of();
template <>
__device__ __forceinline__ double sentinel_of<double>() {
  return sentinel();
}
template <>
__device__ __forceinline__ float sentinel_of<float>() {
  return sentinel_f();
}

// In-order consumption of one window of a triangular-solve row.  Entries
// k0 <= k < W are taken while their values are ready (slot < 0 = no entry;
// its value and coefficient are 0), applying acc -= v[k] * y[k] in order.
// Returns the first position still waiting (W once the window is done).
// Branch-free: the ready prefix and the updates are computed with selects.
// The values y may be stored in FP64 or FP32; the update is FP64.
template <int W, typename TY>
__device__ __forceinline__ int consume_ready(const int* cb, const double* vb, const TY* yv,
                                             int k0, double& acc) {
  int fm = W;
#pragma unroll
  for (int k = W - 1; k >= 0; --k) fm = (k >= k0 && cb[k] >= 0 && is_sentinel(yv[k])) ? k : fm;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const double nx = acc - vb[k] * static_cast<double>(yv[k]);
    acc = (k >= k0 && k < fm) ? nx : acc;
  }
  return fm;
}

// VEC consecutive elements as one access (the caller guarantees that p is
// aligned to 16 bytes for the vector forms): doubles VEC = 1, 2, 4 (4 as two
// 16-byte accesses), floats VEC = 1, 2, 4.
template <int VEC>
__device__ __forceinline__ void vld(const double* p, double* v) {
  if constexpr (VEC == 1) {
    v[0] = p[0];
  } else {
#pragma unroll
    for (int h = 0; h < VEC; h += 2) {
      const double2 q = *reinterpret_cast<const double2*>(p + h);
      v[h] = q.x;
      v[h + 1] = q.y;
    }
  }
}
template <int VEC>
__device__ __forceinline__ void vst(double* p, const double* v) {
  if constexpr (VEC == 1) {
    p[0] = v[0];
  } else {
#pragma unroll
    for (int h = 0; h < VEC; h += 2) *reinterpret_cast<double2*>(p + h) = make_double2(v[h], v[h + 1]);
  }
}
template <int VEC>
__device__ __forceinline__ void vld(const float* p, float* v) {
  if constexpr (VEC == 1) {
    v[0] = p[0];
  } else if constexpr (VEC == 2) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    v[0] = q.x;
    v[1] = q.y;
  } else {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  }
}
template <int VEC>
__device__ __forceinline__ void vst(float* p, const float* v) {
  if constexpr (VEC == 1) {
    p[0] = v[0];
  } else if constexpr (VEC == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  } else {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Partial sums over the entries [b, e) of one row for 64 * VEC columns: wave
// w of the block takes the entries b + w, b + w + 4, ...; the 4 partial sums
// are added in wave order by wave 0, which returns true and leaves them in
// `tot`.
template <int VEC, typename TV, typename TY>
__device__ __forceinline__ bool split_row_sum(int t, int c, int b, int e,
                                              const int* __restrict__ idx,
                                              const TV* __restrict__ vals,
                                              const TY* __restrict__ Y, double* tot) {
  __shared__ double s_part[4][64 * VEC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double part[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) part[v] = 0.0;
  if (c < t) {
    for (int q = b + w; q < e; q += 4 * 8) {
      int cb[8];
      TV vb[8];
      TY y[8][VEC];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        cb[k] = (q + 4 * k < e) ? idx[q + 4 * k] : -1;
        vb[k] = (q + 4 * k < e) ? vals[q + 4 * k] : TV(0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (cb[k] >= 0) {
          vld<VEC>(Y + (int64_t)cb[k] * t + c, y[k]);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v) y[k][v] = TY(0);
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v)
          part[v] += static_cast<double>(vb[k]) * static_cast<double>(y[k][v]);
    }
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v) s_part[w][lane * VEC + v] = part[v];
  __syncthreads();
  if (w != 0 || c >= t) return false;
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const int o = lane * VEC + v;
    tot[v] = ((s_part[0][o] + s_part[1][o]) + s_part[2][o]) + s_part[3][o];
  }
  return true;
}

// Device-coherent polling load / publishing store of one value.  Relaxed
// ordering is enough: every published value carries its own readiness.
template <typename T>
__device__ __forceinline__ T poll_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void publish(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Broadcast a double from a wave-uniform lane.
__device__ __forceinline__ double readlane(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Squared distance of two 2-D points as dx*dx + dy*dy, rounded after each
// operation (no fused multiply-add), so that neighbour ranking matches a
// reference evaluated the same way.
__device__ __forceinline__ double sqdist(double ax, double ay, double bx, double by) {
  double dx = __dsub_rn(ax, bx);
  double dy = __dsub_rn(ay, by);
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

constexpr double kSqrt3 = 1.7320508075688772;

// Covariance as a function of squared distance: exponential
// sigma2 exp(-d/rho) or Matern-3/2 sigma2 (1 + sqrt3 d/rho) exp(-sqrt3 d/rho).
__device__ __forceinline__ double cov_eval(int kind, double d2, double sigma2, double rho) {
  double d = sqrt(d2);
  if (kind == 0) return sigma2 * exp(-d / rho);
  double a = kSqrt3 * d / rho;
  return sigma2 * (1.0 + a) * exp(-a);
}

// d c / d rho as a function of squared distance.
__device__ __forceinline__ double cov_drho(int kind, double d2, double sigma2, double rho) {
  double d = sqrt(d2);
  if (kind == 0) return sigma2 * exp(-d / rho) * d / (rho * rho);
  double a = kSqrt3 * d / rho;
  return sigma2 * a * a * exp(-a) / rho;
}

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t probe_key(uint64_t seed, uint32_t tag, uint64_t col,
                                              uint64_t row) {
  return seed ^ (static_cast<uint64_t>(tag) << 56) ^ (col << 32) ^ row;
}
// +1 / -1 from the top bit.
__device__ __forceinline__ double rademacher(uint64_t seed, uint32_t tag, uint64_t col,
                                             uint64_t row) {
  return (mix64(probe_key(seed, tag, col, row)) >> 63) ? -1.0 : 1.0;
}
// Box-Muller on the hashes of tags `tag` and `tag | 0x80`.
__device__ __forceinline__ double gaussian(uint64_t seed, uint32_t tag, uint64_t col,
                                           uint64_t row) {
  const double scale = 1.1102230246251565e-16;  // 2^-53
  uint64_t h1 = mix64(probe_key(seed, tag, col, row));
  uint64_t h2 = mix64(probe_key(seed, tag | 0x80u, col, row));
  double u1 = static_cast<double>((h1 >> 11) + 1ull) * scale;
  double u2 = static_cast<double>(h2 >> 11) * scale;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Error bits written by kernels into the model's device status word.
enum : int {
  kErrNotSpd = 1,
  kErrTimeout = 2,
  kErrNonfinite = 4,
};

__device__ __forceinline__ void raise_error(int* status, int bit) {
  atomicOr(status, bit);
}

// Column layout of an n x t row-major block processed by one wave:
// lanes_per_row = min(64, next power of two >= t); a wave covers
// 64 / lanes_per_row rows; for t > 64 a row is split into 64-column slices.
struct ColMap {
  int t;        // columns
  int lpr_log;  // log2(lanes per row)
  int slices;   // ceil(t / 64) when t > 64, else 1
  int rpw_log;  // log2(rows per wave) = 6 - lpr_log
};

// Probe tags: part of the counter layout, which a CPU reference implementation
// reproduces with the same numbers.
enum : uint32_t {
  kTagSlq = 1,
  kTagPredZ1 = 2,
  kTagPredZ2 = 3,
  kTagLracN = 4,
  kTagLracK = 5,
};

}  // namespace vl
