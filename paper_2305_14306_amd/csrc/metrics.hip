// Coverage and spacing of a sample on the GPU (arXiv 2305.14306, Sec. 3.1, Fig. 3): for
// every query point the squared distance to its nearest sample, exact in double, and
// the maximum over the queries. With the cloud as queries the maximum is the covering
// radius (squared); with the samples themselves as queries (each skipping itself) the
// values are the spacing distribution Fig. 3 plots. C ABI in include/hav.h (hav_nn_*).
//
// The samples are counting-sorted into a uniform grid of cubic cells (a dense cell
// array of at most kNnCells cells, the cell size chosen on the device from the
// samples' bounding box, so no host round trip). A query scans rings of cells around
// its own cell (Chebyshev distance 0, 1, 2, ...) and stops once its best distance is
// below the gap to the next ring, so the minimum is exact.
//
// The same grid, built over the cloud with cells at least the radius wide, serves the
// ball query that groups points around the sampled centres (the grouping that follows
// sampling in a set-abstraction block, Sec. 3.1): each centre scans its 27 cells and
// keeps the K lowest-index points strictly inside the radius.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/hav.h"
#include "hav_device.hpp"

namespace hav {
namespace {

constexpr int kNnThreads = 256;
constexpr int64_t kNnCells = 1 << 22;      // dense cell array cap
constexpr int kNnScanTile = 4096;          // cells per block of the offset scan
constexpr int kNnBoxBlocks = 1024;
constexpr uint32_t kNnSpinLimit = 1u << 22;

template <typename T>
__device__ __forceinline__ T nn_ld(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void nn_st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct NnHdr {
  double mn[3];
  double h, inv_h;
  int64_t dims[3];
  int64_t ncell;
  uint32_t ord[32];
  uint32_t sync_top[32];
  uint32_t sync_grp[16][32];
  unsigned long long max_d2;
  uint32_t bad;
};

struct NnWs {
  NnHdr* h;
  uint32_t* part;      // [kNnBoxBlocks][6] ordered-bits partial boxes
  uint32_t* cnt;       // [kNnCells] samples per cell, then running cursor
  uint32_t* off;       // [kNnCells + 1] first sample of each cell
  uint32_t* tcnt;      // [kNnCells / kNnScanTile] dispatch-ordered scan slots
  float* sorted;       // [M][3] samples in cell order
  int32_t* sorted_id;  // [M] their indices
};

__device__ __forceinline__ uint32_t nn_ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float nn_unordered(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ bool nn_arrive_last(NnHdr* h, int block, int nblocks) {
  __shared__ int s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = block & 15;
    const int gsize = (nblocks - g + 15) / 16;
    const int ngroups = nblocks < 16 ? nblocks : 16;
    int last = 0;
    if (atomicAdd(&h->sync_grp[g][0], 1u) == static_cast<uint32_t>(gsize - 1)) {
      atomicExch(&h->sync_grp[g][0], 0u);
      if (atomicAdd(&h->sync_top[0], 1u) == static_cast<uint32_t>(ngroups - 1)) {
        atomicExch(&h->sync_top[0], 0u);
        last = 1;
      }
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// Bounding box of the samples; the last block derives the grid: cubic cells of size
// h = 1.5 (volume / M)^(1/3) (about three samples per cell), at least min_h, grown
// until the cell count fits the dense array.
__global__ void __launch_bounds__(kNnThreads) k_nn_box(NnWs w, const float* __restrict__ s, int64_t M,
                                                      double min_h) {
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kNnThreads + threadIdx.x; i < M;
       i += static_cast<int64_t>(gridDim.x) * kNnThreads)
    for (int a = 0; a < 3; ++a) {
      const uint32_t o = nn_ordered(s[3 * i + a]);
      lo[a] = min(lo[a], o);
      hi[a] = max(hi[a], o);
    }
  __shared__ uint32_t red[6][kNnThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t v[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
  for (int k = 0; k < 6; ++k) {
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t y = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v[k]), o, 64));
      v[k] = k < 3 ? min(v[k], y) : max(v[k], y);
    }
    if (lane == 0) red[k][wv] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    uint32_t x = red[k][0];
    for (int q = 1; q < kNnThreads / 64; ++q) x = k < 3 ? min(x, red[k][q]) : max(x, red[k][q]);
    nn_st(&w.part[blockIdx.x * 6 + k], x);
  }
  if (!nn_arrive_last(w.h, blockIdx.x, gridDim.x)) return;
  if (threadIdx.x != 0) return;
  uint32_t b[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
  for (unsigned q = 0; q < gridDim.x; ++q)
    for (int k = 0; k < 6; ++k) {
      const uint32_t x = nn_ld(&w.part[q * 6 + k]);
      b[k] = k < 3 ? min(b[k], x) : max(b[k], x);
    }
  NnHdr* h = w.h;
  double ext[3], vol = 1.0;
  for (int a = 0; a < 3; ++a) {
    h->mn[a] = nn_unordered(b[a]);
    ext[a] = static_cast<double>(nn_unordered(b[3 + a])) - h->mn[a];
    vol *= ext[a] > 1e-9 ? ext[a] : 1e-9;
  }
  // at most 256 cells along the longest axis, so a ring search stays short even for
  // flat or linear sample sets
  const double emax = fmax(ext[0], fmax(ext[1], ext[2]));
  double cs = 1.5 * cbrt(vol / static_cast<double>(M));
  cs = fmax(cs, fmax(min_h, emax / 256.0));
  if (!(cs > 1e-30)) cs = 1e-30;
  double dd[3], ncd = 1.0;
  for (int it = 0; it < 64; ++it) {
    ncd = 1.0;
    for (int a = 0; a < 3; ++a) {
      dd[a] = floor(ext[a] / cs) + 1.0;
      ncd *= dd[a];
    }
    if (ncd <= static_cast<double>(kNnCells)) break;
    cs *= 1.01 * cbrt(ncd / static_cast<double>(kNnCells));
  }
  if (!(ncd <= static_cast<double>(kNnCells))) {  // (not reached) one cell
    cs = 2.0 * emax + 1.0;
    dd[0] = dd[1] = dd[2] = 1.0;
    ncd = 1.0;
  }
  h->h = cs;
  h->inv_h = 1.0 / cs;
  for (int a = 0; a < 3; ++a) h->dims[a] = static_cast<int64_t>(dd[a]);
  h->ncell = static_cast<int64_t>(ncd);
  h->max_d2 = 0ull;
  h->bad = 0u;
}

__device__ __forceinline__ int64_t nn_cell_axis(double x, const NnHdr& h, int a) {
  const double c = floor((x - h.mn[a]) * h.inv_h);
  return static_cast<int64_t>(fmin(fmax(c, -0x1p60), 0x1p60));
}

__device__ __forceinline__ int64_t nn_cell_of(const float* p, const NnHdr& h) {
  int64_t c[3];
  for (int a = 0; a < 3; ++a) {
    int64_t v = nn_cell_axis(p[a], h, a);
    v = v < 0 ? 0 : (v >= h.dims[a] ? h.dims[a] - 1 : v);
    c[a] = v;
  }
  return c[0] + h.dims[0] * (c[1] + h.dims[1] * c[2]);
}

__global__ void __launch_bounds__(kNnThreads) k_nn_count(NnWs w, const float* __restrict__ s, int64_t M) {
  const NnHdr& h = *w.h;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kNnThreads + threadIdx.x; i < M;
       i += static_cast<int64_t>(gridDim.x) * kNnThreads)
    atomicAdd(&w.cnt[nn_cell_of(s + 3 * i, h)], 1u);
}

// Exclusive scan of the cell counts into offsets, one pass: blocks take their tile in
// dispatch order and chain the tile totals (a block waits only for tiles of blocks
// that started before it; bounded). Counts are zeroed for the scatter's cursors.
__global__ void __launch_bounds__(kNnThreads) k_nn_scan(NnWs w, int64_t M) {
  NnHdr* h = w.h;
  const int64_t ncell = h->ncell;
  __shared__ uint32_t s_tmp[kNnThreads / 64];
  __shared__ int s_lb, s_bad;
  if (threadIdx.x == 0) {
    s_lb = static_cast<int>(atomicAdd(&h->ord[0], 1u));
    s_bad = 0;
  }
  __syncthreads();
  const int lb = s_lb;
  constexpr int kPer = kNnScanTile / kNnThreads;
  const int64_t base = static_cast<int64_t>(lb) * kNnScanTile + static_cast<int64_t>(threadIdx.x) * kPer;
  uint32_t v[kPer], sum = 0;
  for (int k = 0; k < kPer; ++k) {
    v[k] = base + k < ncell ? w.cnt[base + k] : 0u;
    sum += v[k];
  }
  uint32_t ex;
  const uint32_t tot = block_exclusive_scan<kNnThreads>(sum, &ex, s_tmp);
  if (threadIdx.x == 0) nn_st(&w.tcnt[lb], tot + 1u);
  uint32_t before = 0;
  for (int i = threadIdx.x; i < lb; i += kNnThreads) {
    uint32_t x, spins = 0;
    while ((x = nn_ld(&w.tcnt[i])) == 0u) {
      if (++spins > kNnSpinLimit) {
        s_bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (x) before += x - 1u;
  }
  before = block_sum_u32<kNnThreads>(before, s_tmp);
  uint32_t r = before + ex;
  for (int k = 0; k < kPer; ++k) {
    if (base + k < ncell) {
      w.off[base + k] = r;
      w.cnt[base + k] = 0u;
    }
    r += v[k];
  }
  if (s_bad && threadIdx.x == 0) atomicOr(&h->bad, 1u);
  if (!nn_arrive_last(h, lb, gridDim.x)) return;
  if (threadIdx.x == 0) {
    w.off[ncell] = static_cast<uint32_t>(M);
    atomicExch(&h->ord[0], 0u);
  }
  for (unsigned i = threadIdx.x; i < gridDim.x; i += kNnThreads) nn_st(&w.tcnt[i], 0u);
}

__global__ void __launch_bounds__(kNnThreads) k_nn_scatter(NnWs w, const float* __restrict__ s, int64_t M) {
  const NnHdr& h = *w.h;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kNnThreads + threadIdx.x; i < M;
       i += static_cast<int64_t>(gridDim.x) * kNnThreads) {
    const int64_t c = nn_cell_of(s + 3 * i, h);
    const uint32_t at = w.off[c] + atomicAdd(&w.cnt[c], 1u);
    if (at < static_cast<uint64_t>(M)) {
      for (int a = 0; a < 3; ++a) w.sorted[3 * static_cast<int64_t>(at) + a] = s[3 * i + a];
      w.sorted_id[at] = static_cast<int32_t>(i);
    }
  }
}

// Nearest sample of every query: squared distance in double ((dx*dx + dy*dy) + dz*dz,
// dx = sample - query, no fused multiply-add); `self`: query j skips sample j.
__global__ void __launch_bounds__(kNnThreads) k_nn_query(NnWs w, const float* __restrict__ q, int64_t Q,
                                                        int32_t self, double* __restrict__ out) {
  const NnHdr& h = *w.h;
  unsigned long long bmax = 0ull;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kNnThreads + threadIdx.x; j < Q;
       j += static_cast<int64_t>(gridDim.x) * kNnThreads) {
    const double px = q[3 * j], py = q[3 * j + 1], pz = q[3 * j + 2];
    const int64_t cx = nn_cell_axis(px, h, 0), cy = nn_cell_axis(py, h, 1), cz = nn_cell_axis(pz, h, 2);
    // rings before r0 hold no cell of the grid, rings after rmax neither
    const int64_t c3[3] = {cx, cy, cz};
    int64_t r0 = 0, rmax = 0;
    for (int a = 0; a < 3; ++a) {
      const int64_t top = h.dims[a] - 1;
      const int64_t out_by = c3[a] < 0 ? -c3[a] : (c3[a] > top ? c3[a] - top : 0);
      const int64_t far = c3[a] > top - c3[a] ? c3[a] : top - c3[a];
      r0 = out_by > r0 ? out_by : r0;
      rmax = far > rmax ? far : rmax;
    }
    double best = INFINITY;
    for (int64_t r = r0; r <= rmax; ++r) {
      const int64_t z0 = cz - r < 0 ? 0 : cz - r, z1 = cz + r > h.dims[2] - 1 ? h.dims[2] - 1 : cz + r;
      const int64_t y0 = cy - r < 0 ? 0 : cy - r, y1 = cy + r > h.dims[1] - 1 ? h.dims[1] - 1 : cy + r;
      const int64_t x0 = cx - r < 0 ? 0 : cx - r, x1 = cx + r > h.dims[0] - 1 ? h.dims[0] - 1 : cx + r;
      for (int64_t z = z0; z <= z1; ++z) {
        for (int64_t y = y0; y <= y1; ++y) {
          const bool shell = (z == cz - r || z == cz + r || y == cy - r || y == cy + r);
          // on the ring's shell every x; inside it only the two end cells
          const int64_t xs[2] = {cx - r, cx + r};
          const int nx = shell ? static_cast<int>(x1 - x0 + 1) : (r == 0 ? 1 : 2);
          for (int t = 0; t < nx; ++t) {
            const int64_t x = shell ? x0 + t : xs[t];
            if (x < 0 || x >= h.dims[0]) continue;
            const int64_t c = x + h.dims[0] * (y + h.dims[1] * z);
            const uint32_t e = w.off[c + 1];
            for (uint32_t k = w.off[c]; k < e; ++k) {
              if (self && w.sorted_id[k] == j) continue;
              const double ex = static_cast<double>(w.sorted[3 * static_cast<int64_t>(k)]) - px;
              const double ey = static_cast<double>(w.sorted[3 * static_cast<int64_t>(k) + 1]) - py;
              const double ez = static_cast<double>(w.sorted[3 * static_cast<int64_t>(k) + 2]) - pz;
              double d = ex * ex;
              d = d + ey * ey;
              d = d + ez * ez;
              best = d < best ? d : best;
            }
          }
        }
      }
      // every sample of a farther ring is at least r cells (less rounding) away
      const double gap = (static_cast<double>(r) - 1e-6) * h.h;
      if (gap > 0.0 && best <= gap * gap) break;
    }
    if (out) out[j] = best;
    const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(best));
    bmax = bits > bmax ? bits : bmax;
  }
  if (bmax) atomicMax(&w.h->max_d2, bmax);
}

constexpr int kBallMaxK = 64;

// Ball query: for centre j the lowest-index points i with d2 < r2 (d2 in float32 as
// ((dx*dx + dy*dy) + dz*dz), dx = x_i - c_j, no fused multiply-add), up to K of them in
// ascending index order; the rest of the row repeats the first, or is -1 when the ball
// is empty. count[j] = the number of points inside. Cells are at least the radius wide,
// so the 27 cells around the centre's cell hold every candidate. Each thread keeps its
// K smallest indices sorted in its own LDS row.
__global__ void __launch_bounds__(kNnThreads) k_ball(NnWs w, const float* __restrict__ ctr,
                                                    int64_t Q, float r2,
                                                    int32_t K, int32_t* __restrict__ out,
                                                    int32_t* __restrict__ count) {
  const NnHdr& h = *w.h;
  __shared__ int32_t kb[kNnThreads * kBallMaxK];
  int32_t* row = kb + threadIdx.x * kBallMaxK;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * kNnThreads + threadIdx.x; j < Q;
       j += static_cast<int64_t>(gridDim.x) * kNnThreads) {
    const float cxf = ctr[3 * j], cyf = ctr[3 * j + 1], czf = ctr[3 * j + 2];
    const int64_t cx = nn_cell_axis(cxf, h, 0), cy = nn_cell_axis(cyf, h, 1), cz = nn_cell_axis(czf, h, 2);
    int n = 0;
    int64_t total = 0;
    for (int64_t z = cz - 1; z <= cz + 1; ++z) {
      if (z < 0 || z >= h.dims[2]) continue;
      for (int64_t y = cy - 1; y <= cy + 1; ++y) {
        if (y < 0 || y >= h.dims[1]) continue;
        for (int64_t x = cx - 1; x <= cx + 1; ++x) {
          if (x < 0 || x >= h.dims[0]) continue;
          const int64_t c = x + h.dims[0] * (y + h.dims[1] * z);
          const uint32_t e = w.off[c + 1];
          for (uint32_t k = w.off[c]; k < e; ++k) {
            const float dx = w.sorted[3 * static_cast<int64_t>(k)] - cxf;
            const float dy = w.sorted[3 * static_cast<int64_t>(k) + 1] - cyf;
            const float dz = w.sorted[3 * static_cast<int64_t>(k) + 2] - czf;
            float d2 = dx * dx;
            d2 = d2 + dy * dy;
            d2 = d2 + dz * dz;
            if (!(d2 < r2)) continue;
            ++total;
            const int32_t id = w.sorted_id[k];
            if (n == K && id >= row[K - 1]) continue;
            // insert id into the sorted row (the largest drops out when full)
            int t = n < K ? n : K - 1;
            while (t > 0 && row[t - 1] > id) {
              row[t] = row[t - 1];
              --t;
            }
            row[t] = id;
            if (n < K) ++n;
          }
        }
      }
    }
    int32_t* o = out + j * static_cast<int64_t>(K);
    for (int t = 0; t < K; ++t) o[t] = t < n ? row[t] : (n > 0 ? row[0] : -1);
    if (count) count[j] = static_cast<int32_t>(total < 0x7FFFFFFF ? total : 0x7FFFFFFF);
  }
}

__global__ void k_nn_init(NnWs w, int64_t ncell_cap) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = i; k < ncell_cap; k += stride) w.cnt[k] = 0u;
  for (int64_t k = i; k < ncell_cap / kNnScanTile + 1; k += stride) w.tcnt[k] = 0u;
  uint32_t* hz = reinterpret_cast<uint32_t*>(w.h);
  for (int64_t k = i; k < static_cast<int64_t>(sizeof(NnHdr) / 4); k += stride) hz[k] = 0u;
}

// Empty the cell counts for the next call.
__global__ void k_nn_clear(NnWs w) {
  const int64_t nc = w.h->ncell;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < nc;
       k += static_cast<int64_t>(gridDim.x) * blockDim.x)
    w.cnt[k] = 0u;
}

__global__ void k_nn_result(NnWs w, double* max_d2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *max_d2 = w.h->bad ? -1.0 : __longlong_as_double(static_cast<long long>(w.h->max_d2));
  }
}

size_t nn_align(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct NnLayout {
  size_t h, part, cnt, off, tcnt, sorted, sorted_id, total;
};

NnLayout nn_layout(int64_t M) {
  NnLayout L;
  size_t o = 0;
  L.h = o;         o = nn_align(o + sizeof(NnHdr));
  L.part = o;      o = nn_align(o + static_cast<size_t>(kNnBoxBlocks) * 6 * 4);
  L.cnt = o;       o = nn_align(o + static_cast<size_t>(kNnCells) * 4);
  L.off = o;       o = nn_align(o + static_cast<size_t>(kNnCells + 1) * 4);
  L.tcnt = o;      o = nn_align(o + static_cast<size_t>(kNnCells / kNnScanTile + 1) * 4);
  L.sorted = o;    o = nn_align(o + static_cast<size_t>(M) * 12);
  L.sorted_id = o; o = nn_align(o + static_cast<size_t>(M) * 4);
  L.total = o;
  return L;
}

NnWs nn_ws(void* ws, const NnLayout& L) {
  char* b = static_cast<char*>(ws);
  return NnWs{reinterpret_cast<NnHdr*>(b + L.h),       reinterpret_cast<uint32_t*>(b + L.part),
              reinterpret_cast<uint32_t*>(b + L.cnt),  reinterpret_cast<uint32_t*>(b + L.off),
              reinterpret_cast<uint32_t*>(b + L.tcnt), reinterpret_cast<float*>(b + L.sorted),
              reinterpret_cast<int32_t*>(b + L.sorted_id)};
}

}  // namespace
}  // namespace hav

using namespace hav;

extern "C" {

size_t hav_nn_workspace_size(int64_t M) {
  if (M < 1 || M > HAV_NN_MAX_SAMPLES) return 0;
  return nn_layout(M).total;
}

hav_status_t hav_nn_workspace_init(void* ws, size_t ws_bytes, int64_t M, void* stream) {
  if (!ws || M < 1 || M > HAV_NN_MAX_SAMPLES) return HAV_ERR_INVALID_ARG;
  const NnLayout L = nn_layout(M);
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipLaunchKernelGGL(k_nn_init, dim3(1024), dim3(256), 0, static_cast<hipStream_t>(stream), nn_ws(ws, L),
                     static_cast<int64_t>(kNnCells));
  return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

hav_status_t hav_nn(const float* samples, int64_t M, const float* queries, int64_t Q, int32_t exclude_self,
                    double* d2_out, double* max_d2, void* ws, size_t ws_bytes, void* stream) {
  if (!samples || !queries || !max_d2 || !ws || M < 1 || M > HAV_NN_MAX_SAMPLES || Q < 1 ||
      Q > HAV_NN_MAX_SAMPLES || (exclude_self && (Q != M || M < 2)))
    return HAV_ERR_INVALID_ARG;
  const NnLayout L = nn_layout(M);
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const NnWs w = nn_ws(ws, L);
  const unsigned gb = static_cast<unsigned>(std::min<int64_t>(kNnBoxBlocks, (M + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_nn_box, dim3(gb), dim3(kNnThreads), 0, st, w, samples, M, 0.0);
  const unsigned gs = static_cast<unsigned>(std::min<int64_t>(4096, (M + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_nn_count, dim3(gs), dim3(kNnThreads), 0, st, w, samples, M);
  hipLaunchKernelGGL(k_nn_scan, dim3(static_cast<unsigned>(kNnCells / kNnScanTile)), dim3(kNnThreads), 0, st, w, M);
  hipLaunchKernelGGL(k_nn_scatter, dim3(gs), dim3(kNnThreads), 0, st, w, samples, M);
  const unsigned gq = static_cast<unsigned>(std::min<int64_t>(65536, (Q + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_nn_query, dim3(gq), dim3(kNnThreads), 0, st, w, queries, Q, exclude_self, d2_out);
  hipLaunchKernelGGL(k_nn_clear, dim3(1024), dim3(256), 0, st, w);
  hipLaunchKernelGGL(k_nn_result, dim3(1), dim3(64), 0, st, w, max_d2);
  return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

size_t hav_ball_workspace_size(int64_t N) { return hav_nn_workspace_size(N); }

hav_status_t hav_ball_workspace_init(void* ws, size_t ws_bytes, int64_t N, void* stream) {
  return hav_nn_workspace_init(ws, ws_bytes, N, stream);
}

hav_status_t hav_ball_query(const float* xyz, int64_t N, const float* centres, int64_t Q, float radius,
                            int32_t K, int32_t* idx, int32_t* count, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!xyz || !centres || !idx || !ws || N < 1 || N > HAV_NN_MAX_SAMPLES || Q < 1 ||
      Q > HAV_NN_MAX_SAMPLES || K < 1 || K > kBallMaxK || !(radius > 0.0f) || !std::isfinite(radius))
    return HAV_ERR_INVALID_ARG;
  const NnLayout L = nn_layout(N);
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const NnWs w = nn_ws(ws, L);
  const float r2 = radius * radius;
  // cells a little wider than the radius, so one ring of cells holds the whole ball
  const double min_h = static_cast<double>(radius) * 1.001;
  const unsigned gb = static_cast<unsigned>(std::min<int64_t>(kNnBoxBlocks, (N + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_nn_box, dim3(gb), dim3(kNnThreads), 0, st, w, xyz, N, min_h);
  const unsigned gs = static_cast<unsigned>(std::min<int64_t>(4096, (N + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_nn_count, dim3(gs), dim3(kNnThreads), 0, st, w, xyz, N);
  hipLaunchKernelGGL(k_nn_scan, dim3(static_cast<unsigned>(kNnCells / kNnScanTile)), dim3(kNnThreads), 0, st, w, N);
  hipLaunchKernelGGL(k_nn_scatter, dim3(gs), dim3(kNnThreads), 0, st, w, xyz, N);
  const unsigned gq = static_cast<unsigned>(std::min<int64_t>(65536, (Q + kNnThreads - 1) / kNnThreads));
  hipLaunchKernelGGL(k_ball, dim3(gq), dim3(kNnThreads), 0, st, w, centres, Q, r2, K, idx, count);
  hipLaunchKernelGGL(k_nn_clear, dim3(1024), dim3(256), 0, st, w);
  return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

}  // extern "C"
