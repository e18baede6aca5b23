// Nearest-earlier-neighbour search for the Vecchia approximation (Sec. 2.1):
// N(i) = the min(i, m) nearest locations among 0..i-1, ordered by (squared
// distance, index).  Prediction points (Sec. 2.2.1, observed locations first)
// take the m nearest among all n training locations.
//
// Locations are binned into a uniform G x G grid (G a power of two, about two
// points per cell) whose cells are numbered in Morton order, so the cell
// arrays are spatially local.  A query scans Chebyshev rings of cells around
// its own cell and stops once the m-th best squared distance is strictly below
// the squared distance from the query to the edge of the scanned box (no
// unscanned point can then enter or tie into the set).  Queries whose
// eligible set is small (early rows) scan the eligible prefix directly.
#include "vl_internal.h"

namespace vl {

__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
  v &= 0x0000ffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__device__ __forceinline__ uint32_t morton2(uint32_t x, uint32_t y) {
  return spread_bits(x) | (spread_bits(y) << 1);
}

// Bounding box: per-block min/max, then a single block folds them.
__global__ void bbox_partial(const double* __restrict__ xy, int64_t n, double* __restrict__ part) {
  __shared__ double s[4][256];
  double lo_x = 1e300, lo_y = 1e300, hi_x = -1e300, hi_y = -1e300;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x = xy[2 * i], y = xy[2 * i + 1];
    lo_x = fmin(lo_x, x); lo_y = fmin(lo_y, y);
    hi_x = fmax(hi_x, x); hi_y = fmax(hi_y, y);
  }
  s[0][threadIdx.x] = lo_x; s[1][threadIdx.x] = lo_y;
  s[2][threadIdx.x] = hi_x; s[3][threadIdx.x] = hi_y;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + o]);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + o]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + o]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) part[blockIdx.x * 4 + k] = s[k][0];
  }
}

__global__ void bbox_final(const double* __restrict__ part, int nb, int G,
                           GridGeom* __restrict__ geom) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo_x = 1e300, lo_y = 1e300, hi_x = -1e300, hi_y = -1e300;
  for (int b = 0; b < nb; ++b) {
    lo_x = fmin(lo_x, part[4 * b]); lo_y = fmin(lo_y, part[4 * b + 1]);
    hi_x = fmax(hi_x, part[4 * b + 2]); hi_y = fmax(hi_y, part[4 * b + 3]);
  }
  double ext = fmax(hi_x - lo_x, hi_y - lo_y);
  if (!(ext > 0.0)) ext = 1.0;
  ext *= (1.0 + 1e-9);
  geom->x0 = lo_x;
  geom->y0 = lo_y;
  geom->h = ext / G;
  geom->G = G;
  geom->slack = 1e-12 * ext;
}

__device__ __forceinline__ int cell_coord(double v, double v0, double h, int G) {
  int c = static_cast<int>(floor((v - v0) / h));
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

__global__ void grid_count(const double* __restrict__ xy, int64_t n,
                           const GridGeom* __restrict__ geom, int* __restrict__ cell_of,
                           int* __restrict__ count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  GridGeom g = *geom;
  int cx = cell_coord(xy[2 * i], g.x0, g.h, g.G);
  int cy = cell_coord(xy[2 * i + 1], g.y0, g.h, g.G);
  int c = static_cast<int>(morton2(cx, cy));
  cell_of[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void grid_fill(const double* __restrict__ xy, int64_t n,
                          const int* __restrict__ cell_of, const int* __restrict__ start,
                          int* __restrict__ cursor, int* __restrict__ pts,
                          double* __restrict__ pts_xy) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell_of[i];
  int pos = start[c] + atomicAdd(&cursor[c], 1);
  pts[pos] = static_cast<int>(i);
  pts_xy[2 * pos] = xy[2 * i];
  pts_xy[2 * pos + 1] = xy[2 * i + 1];
}

// Top-m list kept sorted by (d2, index) in LDS, one list per thread.
struct TopM {
  double* d;
  int* j;
  int cnt;
  int cap;
  __device__ __forceinline__ void offer(double d2, int idx) {
    if (cnt == cap) {
      double dl = d[cnt - 1];
      if (d2 > dl || (d2 == dl && idx > j[cnt - 1])) return;
    }
    int p = (cnt < cap) ? cnt : cap - 1;
    while (p > 0) {
      double dp = d[p - 1];
      if (dp < d2 || (dp == d2 && j[p - 1] < idx)) break;
      d[p] = dp;
      j[p] = j[p - 1];
      --p;
    }
    d[p] = d2;
    j[p] = idx;
    if (cnt < cap) ++cnt;
  }
};

constexpr int kKnnBlock = 64;
constexpr int kKnnMaxM = 32;

// One thread per query.  Training rows (q_xy == nullptr): query i, eligible
// j < i.  Prediction rows: query coordinates q_xy[p], eligible all j < n.
__global__ __launch_bounds__(kKnnBlock) void knn_kernel(
    const double* __restrict__ xy, int64_t n, const double* __restrict__ q_xy, int64_t nq,
    int m, int brute_limit, const GridGeom* __restrict__ geom, const int* __restrict__ start,
    const int* __restrict__ pts, const double* __restrict__ pts_xy, int* __restrict__ nbr) {
  __shared__ double s_d[kKnnBlock * kKnnMaxM];
  __shared__ int s_j[kKnnBlock * kKnnMaxM];
  int64_t q = blockIdx.x * (int64_t)kKnnBlock + threadIdx.x;
  if (q >= nq) return;
  TopM top{&s_d[threadIdx.x * kKnnMaxM], &s_j[threadIdx.x * kKnnMaxM], 0, 0};
  const bool train = (q_xy == nullptr);
  const int64_t lim = train ? q : n;            // eligible: j < lim
  const int want = static_cast<int>(lim < m ? lim : m);
  top.cap = want;
  double qx = train ? xy[2 * q] : q_xy[2 * q];
  double qy = train ? xy[2 * q + 1] : q_xy[2 * q + 1];
  if (want > 0) {
    if (lim <= brute_limit) {
      for (int64_t j = 0; j < lim; ++j)
        top.offer(sqdist(qx, qy, xy[2 * j], xy[2 * j + 1]), static_cast<int>(j));
    } else {
      GridGeom g = *geom;
      int cx = cell_coord(qx, g.x0, g.h, g.G);
      int cy = cell_coord(qy, g.y0, g.h, g.G);
      for (int r = 0;; ++r) {
        int xlo = cx - r, xhi = cx + r, ylo = cy - r, yhi = cy + r;
        for (int y = ylo; y <= yhi; ++y) {
          if (y < 0 || y >= g.G) continue;
          const bool edge_row = (y == ylo || y == yhi);
          for (int x = xlo; x <= xhi; x += (edge_row ? 1 : (xhi - xlo))) {
            if (x >= 0 && x < g.G) {
              int c = static_cast<int>(morton2(x, y));
              for (int p = start[c]; p < start[c + 1]; ++p) {
                int j = pts[p];
                if (j < lim) top.offer(sqdist(qx, qy, pts_xy[2 * p], pts_xy[2 * p + 1]), j);
              }
            }
            if (xhi == xlo) break;
          }
        }
        // squared distance from the query to the boundary of the scanned box;
        // sides on the grid border have nothing beyond them
        double bnd = 1e300;
        if (xlo > 0) bnd = fmin(bnd, qx - (g.x0 + xlo * g.h));
        if (xhi < g.G - 1) bnd = fmin(bnd, (g.x0 + (xhi + 1) * g.h) - qx);
        if (ylo > 0) bnd = fmin(bnd, qy - (g.y0 + ylo * g.h));
        if (yhi < g.G - 1) bnd = fmin(bnd, (g.y0 + (yhi + 1) * g.h) - qy);
        if (bnd >= 1e300) break;  // the box covers the whole grid
        bnd -= g.slack;
        if (top.cnt == want && bnd > 0.0 && top.d[want - 1] < bnd * bnd) break;
      }
    }
  }
  int* out = nbr + q * m;
  for (int k = 0; k < m; ++k) out[k] = (k < top.cnt) ? top.j[k] : -1;
}

}  // namespace vl

// --------------------------------------------------------------------------
// host driver
// --------------------------------------------------------------------------
namespace vl {

Status knn_build_grid(Model& M) {
  const int64_t n = M.n;
  int G = 1;
  while (static_cast<double>(G) * G * 2.0 < static_cast<double>(n)) G *= 2;
  if (G > 32768) G = 32768;
  M.grid_G = G;
  const int64_t ncell = static_cast<int64_t>(G) * G;
  const int nb = 256;
  VL_TRY(M.ws_alloc(&M.grid_geom, sizeof(GridGeom)));
  VL_TRY(M.ws_alloc(&M.grid_start, sizeof(int) * (ncell + 1)));
  VL_TRY(M.ws_alloc(&M.grid_pts, sizeof(int) * n));
  VL_TRY(M.ws_alloc(&M.grid_xy, sizeof(double) * 2 * n));
  DevBuf<double> part;
  DevBuf<int> cell_of, cnt;
  VL_TRY(part.alloc(4 * nb));
  VL_TRY(cell_of.alloc(n));
  VL_TRY(cnt.alloc(ncell + 1));
  hipStream_t s = M.stream;
  hipLaunchKernelGGL(bbox_partial, dim3(nb), dim3(256), 0, s, M.coords, n, part.p);
  hipLaunchKernelGGL(bbox_final, dim3(1), dim3(64), 0, s, part.p, nb, G,
                     static_cast<GridGeom*>(M.grid_geom));
  VL_TRY(fill_int(cnt.p, 0, ncell + 1, s));
  const int tb = 256;
  const unsigned gb = static_cast<unsigned>((n + tb - 1) / tb);
  hipLaunchKernelGGL(grid_count, dim3(gb), dim3(tb), 0, s, M.coords, n,
                     static_cast<const GridGeom*>(M.grid_geom), cell_of.p, cnt.p);
  VL_TRY(exclusive_scan_int(cnt.p, static_cast<int*>(M.grid_start), ncell + 1, s));
  VL_TRY(fill_int(cnt.p, 0, ncell + 1, s));
  hipLaunchKernelGGL(grid_fill, dim3(gb), dim3(tb), 0, s, M.coords, n, cell_of.p,
                     static_cast<const int*>(M.grid_start), cnt.p,
                     static_cast<int*>(M.grid_pts), static_cast<double*>(M.grid_xy));
  VL_TRY(check_launch("grid build"));
  VL_TRY(sync_stream(s));  // temporaries are released on return
  return Status::ok();
}

Status knn_query(Model& M, const double* q_xy, int64_t nq, int* nbr_out) {
  if (M.m > kKnnMaxM) return Status::invalid("m exceeds 32");
  if (M.m == 0 || nq == 0) {
    if (nq > 0 && M.m > 0) VL_TRY(fill_int(nbr_out, -1, nq * M.m, M.stream));
    return Status::ok();
  }
  const int brute_limit = 1024;
  const unsigned gb = static_cast<unsigned>((nq + kKnnBlock - 1) / kKnnBlock);
  hipLaunchKernelGGL(knn_kernel, dim3(gb), dim3(kKnnBlock), 0, M.stream, M.coords, M.n, q_xy,
                     nq, M.m, brute_limit, static_cast<const GridGeom*>(M.grid_geom),
                     static_cast<const int*>(M.grid_start), static_cast<const int*>(M.grid_pts),
                     static_cast<const double*>(M.grid_xy), nbr_out);
  return check_launch("knn");
}

}  // namespace vl
