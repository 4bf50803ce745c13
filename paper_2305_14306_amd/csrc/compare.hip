// The two samplers the latency study compares HAVSampler with (arXiv 2305.14306,
// Sec. 4.2, Fig. 7), for gfx950: farthest point sampling (Sec. 3.1, Eq. 1) and
// random point sampling. C ABI in include/hav.h (hav_fps*, hav_rps*).
//
// FPS is a chain of m dependent arg-max steps over all n points. The points stay in
// registers for the whole call (one launch): each block owns a slice, keeps the
// slice's distances to the selected set, and per step finds its farthest point. With
// one block the step ends at a block barrier. With several, every block posts its
// candidate in a per-step slot (value words, then a tag word written with release
// order) and every block reads all slots (acquire) and takes the same maximum, so a
// step costs one exchange instead of a kernel boundary. The blocks must all be
// resident at once: the host launches at most as many as the device holds (its
// occupancy times its compute units, one 1024-thread block per compute unit), and every
// wait is bounded, so a grid that other work keeps from starting whole raises the error
// flag instead of hanging. (An ordinary launch, not a cooperative one: a cooperative
// launch also made rocprofv3 fail when the process ended.)
//
// RPS keeps the m points of smallest SplitMix64 key and returns them in ascending
// order. The m-th smallest of n evenly spread keys lies near the fraction m / (n + 1)
// of the key range; one pass counts the keys below a window around that point and
// queues the keys inside it, and the last block ranks the queue (or, if the window
// missed, radix-selects over all keys, which are recomputed from the index). A second
// pass writes the kept indices in order (block counts chained in dispatch order).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/hav.h"
#include "hav_device.hpp"

namespace hav {
namespace {

template <typename T>
__device__ __forceinline__ T cmp_ld_agent(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void cmp_st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kCmpSpinLimit = 1u << 22;

// ----------------------------------------------------------------------------- FPS

constexpr int kFpsMaxBlocks = 256;
constexpr int kFpsMaxPer = 4;  // points per thread (registers; 8 would spill)

// A block's candidate of one step: squared distance (bits of a non-negative double),
// coordinates, and last the tag word (step + 1) << 32 | index.
struct alignas(32) FpsSlot {
  unsigned long long d, xy, z, tag;
};

struct FpsBest {
  double d;
  int32_t i;
};

// (d, -i) order: larger distance first, then the lower index (the first maximum of
// an ascending scan).
__device__ __forceinline__ bool fps_better(double d, int32_t i, double bd, int32_t bi) {
  return d > bd || (d == bd && i < bi);
}

__device__ __forceinline__ void fps_take(FpsBest& a, const FpsBest& b) {
  if (fps_better(b.d, b.i, a.d, a.i)) a = b;
}

__device__ __forceinline__ FpsBest fps_shfl_xor(const FpsBest& v, int o) {
  FpsBest r;
  const unsigned long long db = static_cast<unsigned long long>(__double_as_longlong(v.d));
  const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(db & 0xFFFFFFFFull), o, 64));
  const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(db >> 32), o, 64));
  r.d = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
  r.i = __shfl_xor(v.i, o, 64);
  return r;
}

// Block-wide best; every thread gets it. s_w holds one entry per wave.
template <int kT>
__device__ __forceinline__ FpsBest fps_block_best(FpsBest v, FpsBest* s_w) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fps_take(v, fps_shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s_w[wv] = v;
  __syncthreads();
  FpsBest b = s_w[0];
#pragma unroll
  for (int q = 1; q < kT / 64; ++q) fps_take(b, s_w[q]);
  return b;
}

// FPS over n points from `start`: out[j] is the j-th selected index. Squared
// distances in double, summed x, y, z in that order, no fused multiply-add. Block b
// owns points b*kT*PER + k*kT + t (thread t, k < PER), kept as doubles (exact).
template <int kT, int PER>
__global__ void __launch_bounds__(kT) k_fps(const float* __restrict__ xyz, int64_t n, int64_t m,
                                            int64_t start, int32_t* __restrict__ out,
                                            FpsSlot* slots, uint32_t* err) {
  const int B = gridDim.x, b = blockIdx.x, t = threadIdx.x;
  const int64_t first = static_cast<int64_t>(b) * kT * PER;
  double px[PER], py[PER], pz[PER], dist[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int64_t i = first + static_cast<int64_t>(k) * kT + t;
    px[k] = py[k] = pz[k] = 0.0;
    dist[k] = -1.0;  // no point: never a candidate
    if (i < n) {
      px[k] = xyz[3 * i];
      py[k] = xyz[3 * i + 1];
      pz[k] = xyz[3 * i + 2];
      dist[k] = INFINITY;
    }
  }
  __shared__ FpsBest s_w[kT / 64];
  __shared__ FpsBest s_all[kT / 64];
  __shared__ double s_c[3];
  __shared__ int s_bad;
  if (t == 0) s_bad = 0;
  if (B == 1 && t == 0) *err = 0u;  // (several blocks: cleared by k_fps_clear before)
  double cx = xyz[3 * start], cy = xyz[3 * start + 1], cz = xyz[3 * start + 2];
  int64_t cur = start;
  for (int64_t j = 0;; ++j) {
    if (b == 0 && t == 0) out[j] = static_cast<int32_t>(cur);
    if (j + 1 >= m) break;
    FpsBest v{-1.0, 0x7FFFFFFF};
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (dist[k] < 0.0) continue;
      const double dx = px[k] - cx, dy = py[k] - cy, dz = pz[k] - cz;
      double d = dx * dx;
      d = d + dy * dy;
      d = d + dz * dz;
      if (d < dist[k]) dist[k] = d;
      const int32_t i = static_cast<int32_t>(first + static_cast<int64_t>(k) * kT + t);
      if (fps_better(dist[k], i, v.d, v.i)) v = FpsBest{dist[k], i};
    }
    FpsBest best = fps_block_best<kT>(v, s_w);
    // the owner of the block's best publishes its coordinates
    {
      const int64_t rel = static_cast<int64_t>(best.i) - first;
      if (best.d >= 0.0 && rel >= 0 && rel < static_cast<int64_t>(kT) * PER && rel % kT == t) {
        const int kk = static_cast<int>(rel / kT);
#pragma unroll
        for (int k = 0; k < PER; ++k)
          if (k == kk) {
            s_c[0] = px[k];
            s_c[1] = py[k];
            s_c[2] = pz[k];
          }
      }
    }
    __syncthreads();
    double bx = s_c[0], by = s_c[1], bz = s_c[2];
    if (B > 1) {
      FpsSlot* row = slots + static_cast<size_t>(j & 1) * kFpsMaxBlocks;
      const unsigned long long tag = static_cast<unsigned long long>(j + 1) << 32;
      if (t == 0) {
        FpsSlot* s = row + b;
        cmp_st_agent(&s->d, static_cast<unsigned long long>(__double_as_longlong(best.d)));
        cmp_st_agent(&s->xy, (static_cast<unsigned long long>(__float_as_uint(static_cast<float>(by))) << 32) |
                                 __float_as_uint(static_cast<float>(bx)));
        cmp_st_agent(&s->z, static_cast<unsigned long long>(__float_as_uint(static_cast<float>(bz))));
        __hip_atomic_store(&s->tag, tag | static_cast<uint32_t>(best.i), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      FpsBest got{-1.0, 0x7FFFFFFF};
      unsigned long long gxy = 0ull, gz = 0ull;
      if (t < B) {
        FpsSlot* s = row + t;
        uint32_t spins = 0;
        unsigned long long tv;
        while (((tv = __hip_atomic_load(&s->tag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) >> 32) !=
               static_cast<unsigned long long>(j + 1)) {
          if (++spins > kCmpSpinLimit || cmp_ld_agent(err)) {
            atomicOr(err, 1u);
            s_bad = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if ((tv >> 32) == static_cast<unsigned long long>(j + 1)) {
          got.d = __longlong_as_double(static_cast<long long>(cmp_ld_agent(&s->d)));
          got.i = static_cast<int32_t>(tv & 0xFFFFFFFFull);
          gxy = cmp_ld_agent(&s->xy);
          gz = cmp_ld_agent(&s->z);
        }
      }
      best = fps_block_best<kT>(got, s_all);
      // the slot holding the winner gives its coordinates (slot t holds block t's best)
      if (t < B && got.i == best.i && got.d == best.d) {
        s_c[0] = __uint_as_float(static_cast<uint32_t>(gxy & 0xFFFFFFFFull));
        s_c[1] = __uint_as_float(static_cast<uint32_t>(gxy >> 32));
        s_c[2] = __uint_as_float(static_cast<uint32_t>(gz));
      }
      __syncthreads();
      if (s_bad) break;
      bx = s_c[0];
      by = s_c[1];
      bz = s_c[2];
    }
    cur = best.i;
    cx = bx;
    cy = by;
    cz = bz;
    __syncthreads();  // s_c is rewritten in the next step
  }
}

__global__ void k_fps_clear(FpsSlot* slots, uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * kFpsMaxBlocks) slots[i] = FpsSlot{0ull, 0ull, 0ull, 0ull};
  if (i == 0) *err = 0u;
}

size_t fps_ws_bytes() { return 2 * kFpsMaxBlocks * sizeof(FpsSlot) + 256; }

// Blocks of k_fps<kT, PER> the current device holds at once (0 if unknown).
template <int kT, int PER>
int fps_resident_blocks() {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_fps<kT, PER>), kT,
                                                    0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// hipErrorInvalidConfiguration when the device cannot hold `blocks` blocks at once.
template <int kT, int PER>
hipError_t launch_fps(int blocks, const float* xyz, int64_t n, int64_t m, int64_t start, int32_t* out,
                      FpsSlot* slots, uint32_t* err, hipStream_t st) {
  if (blocks > 1 && blocks > fps_resident_blocks<kT, PER>()) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_fps<kT, PER>), dim3(blocks), dim3(kT), 0, st, xyz, n, m, start, out, slots, err);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- RPS

constexpr int kRpsThreads = 256;
constexpr int kRpsPer = 8;
constexpr int kRpsTile = kRpsThreads * kRpsPer;
constexpr int kRpsGroups = 16;
constexpr int kRpsQueue = 1 << 16;   // window queue capacity (entries)
constexpr int kRpsLds = 2048;        // queue staged in LDS up to this size
constexpr int kRpsRank = 128;        // members ranked directly up to this many
constexpr double kRpsSigma = 6.0;

struct RpsHdr {
  uint32_t below[kRpsGroups][32];
  uint32_t inwin[kRpsGroups][32];
  uint32_t qn[32];
  uint32_t sync_grp[kRpsGroups][32];
  uint32_t sync_top[32];
  uint32_t ord[32];
  uint32_t bad[32];
  unsigned long long thr;
};

struct RpsWs {
  RpsHdr* h;
  unsigned long long* qp;  // [kRpsQueue] queued keys
  uint32_t* tcnt;          // [ntile] dispatch-ordered tile counts (+1)
};

// The key of point i: output i + 1 of a SplitMix64 generator seeded with `seed`.
__device__ __forceinline__ uint64_t rps_key(uint64_t seed, int64_t i) {
  return voxel_priority(seed + static_cast<uint64_t>(i) * 0x9E3779B97F4A7C15ull);
}

__device__ bool rps_arrive_last(RpsHdr* h, int block, int nblocks) {
  __shared__ int s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = block & (kRpsGroups - 1);
    const int gsize = (nblocks - g + kRpsGroups - 1) / kRpsGroups;
    const int ngroups = nblocks < kRpsGroups ? nblocks : kRpsGroups;
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

// Digit holding `rank` in a 256-bin histogram, and the rank inside it.
__device__ void rps_find_digit(const uint32_t* hist, uint32_t rank, int* digit, uint32_t* rest) {
  __shared__ uint32_t s_tmp[kRpsThreads / 64];
  __shared__ int s_d;
  __shared__ uint32_t s_r;
  const uint32_t v = threadIdx.x < 256 ? hist[threadIdx.x] : 0u;
  if (threadIdx.x == 0) {
    s_d = 255;
    s_r = 0;
  }
  uint32_t ex;
  block_exclusive_scan<kRpsThreads>(v, &ex, s_tmp);
  if (threadIdx.x < 256 && rank >= ex && rank < ex + v) {
    s_d = threadIdx.x;
    s_r = rank - ex;
  }
  __syncthreads();
  *digit = s_d;
  *rest = s_r;
  __syncthreads();
}

// Pass 1: count keys below the window, queue the keys inside it; the last block finds
// the m-th smallest key (the threshold).
__global__ void __launch_bounds__(kRpsThreads) k_rps_count(RpsWs w, int64_t n, int64_t m, uint64_t seed,
                                                           unsigned long long blo, unsigned long long bhi) {
  const int bx = blockIdx.x, gx = gridDim.x;
  RpsHdr* h = w.h;
  __shared__ uint32_t s_below, s_inwin;
  if (threadIdx.x == 0) {
    s_below = 0;
    s_inwin = 0;
  }
  __syncthreads();
  uint32_t below = 0;
  const int64_t base = static_cast<int64_t>(bx) * kRpsTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kRpsPer; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * kRpsThreads;
    if (i >= n) continue;
    const uint64_t p = rps_key(seed, i);
    if (p < blo) {
      ++below;
    } else if (p <= bhi) {
      atomicAdd(&s_inwin, 1u);
      const uint32_t q = atomicAdd(&h->qn[0], 1u);
      if (q < static_cast<uint32_t>(kRpsQueue)) cmp_st_agent(&w.qp[q], static_cast<unsigned long long>(p));
    }
  }
  if (below) atomicAdd(&s_below, below);
  __syncthreads();
  const int g = bx & (kRpsGroups - 1);
  if (threadIdx.x == 0) {
    if (s_below) atomicAdd(&h->below[g][0], s_below);
    if (s_inwin) atomicAdd(&h->inwin[g][0], s_inwin);
  }
  if (!rps_arrive_last(h, bx, gx)) return;
  // ---- last block
  __shared__ uint32_t s_sum[2];
  __shared__ uint32_t hst[256];
  __shared__ unsigned long long lp[kRpsLds];
  __shared__ unsigned long long ls[kRpsRank];
  __shared__ unsigned long long s_pfx, s_thr;
  __shared__ uint32_t s_rank, s_remain, s_nm;
  __shared__ int s_mode;
  if (threadIdx.x < 2) s_sum[threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x < 2 * kRpsGroups) {
    uint32_t* a = threadIdx.x < kRpsGroups ? &h->below[threadIdx.x][0] : &h->inwin[threadIdx.x - kRpsGroups][0];
    const uint32_t v = atomicExch(a, 0u);
    if (v) atomicAdd(&s_sum[threadIdx.x / kRpsGroups], v);
  }
  __shared__ uint32_t s_qn;
  if (threadIdx.x == 0) s_qn = atomicExch(&h->qn[0], 0u);
  __syncthreads();
  const uint32_t qn = s_qn;
  if (threadIdx.x == 0) {
    const uint32_t nb = s_sum[0], ni = s_sum[1];
    const uint64_t mm = static_cast<uint64_t>(m);
    // window: the threshold is inside iff fewer than m keys are below it and at least
    // m are below or inside it
    const bool ok = nb < mm && mm <= static_cast<uint64_t>(nb) + ni && qn <= static_cast<uint32_t>(kRpsQueue);
    s_mode = ok ? 1 : 2;
    s_rank = ok ? static_cast<uint32_t>(mm - 1 - nb) : static_cast<uint32_t>(mm - 1);
    s_remain = ok ? qn : static_cast<uint32_t>(n);
    s_pfx = 0;
    s_thr = ~0ull;
    s_nm = 0;
  }
  __syncthreads();
  const int mode = s_mode;
  const uint32_t total = mode == 1 ? qn : 0u;
  const bool staged = mode == 1 && total <= static_cast<uint32_t>(kRpsLds);
  if (staged)
    for (uint32_t j = threadIdx.x; j < total; j += kRpsThreads) lp[j] = cmp_ld_agent(&w.qp[j]);
  __syncthreads();
  // members: the queue (window) or every key (recomputed)
  const uint64_t count = mode == 1 ? total : static_cast<uint64_t>(n);
  auto key = [&](uint64_t j) -> uint64_t {
    if (mode == 2) return rps_key(seed, static_cast<int64_t>(j));
    return staged ? lp[j] : cmp_ld_agent(&w.qp[j]);
  };
  const uint64_t kbase = mode == 1 ? blo : 0ull;
  int hi = 64;
  if (mode == 1) {
    const uint64_t width = bhi - blo;
    hi = width ? 64 - __clzll(static_cast<long long>(width)) : 0;
  }
  while (s_remain > static_cast<uint32_t>(kRpsRank) && hi > 0) {
    const int wdt = hi >= 8 ? 8 : hi;
    const int sh = hi - wdt;
    for (int i = threadIdx.x; i < 256; i += kRpsThreads) hst[i] = 0;
    __syncthreads();
    const uint64_t pfx = s_pfx;
    for (uint64_t j = threadIdx.x; j < count; j += kRpsThreads) {
      const uint64_t r = key(j) - kbase;
      if (hi < 64 && (r >> hi) != (pfx >> hi)) continue;
      atomicAdd(&hst[(r >> sh) & ((1u << wdt) - 1u)], 1u);
    }
    __syncthreads();
    int dg;
    uint32_t rest;
    rps_find_digit(hst, s_rank, &dg, &rest);
    if (threadIdx.x == 0) {
      s_rank = rest;
      s_pfx = pfx | (static_cast<uint64_t>(dg) << sh);
      s_remain = hst[dg];
    }
    __syncthreads();
    hi = sh;
  }
  {
    const uint64_t pfx = s_pfx;
    for (uint64_t j = threadIdx.x; j < count; j += kRpsThreads) {
      const uint64_t p = key(j);
      const uint64_t r = p - kbase;
      if (hi >= 64 || (r >> hi) == (pfx >> hi)) {
        const uint32_t k = atomicAdd(&s_nm, 1u);
        if (k < static_cast<uint32_t>(kRpsRank)) ls[k] = p;
      }
    }
  }
  __syncthreads();
  const uint32_t nm = s_nm < static_cast<uint32_t>(kRpsRank) ? s_nm : static_cast<uint32_t>(kRpsRank);
  for (uint32_t j = threadIdx.x; j < nm; j += kRpsThreads) {
    const uint64_t pj = ls[j];
    uint32_t r = 0;
    for (uint32_t i = 0; i < nm; ++i) r += ls[i] < pj ? 1u : 0u;
    if (r == s_rank) s_thr = pj;
  }
  __syncthreads();
  if (threadIdx.x == 0) h->thr = s_thr;
}

// Pass 2: the kept indices (key <= threshold) in ascending order.
__global__ void __launch_bounds__(kRpsThreads) k_rps_out(RpsWs w, int64_t n, int64_t m, uint64_t seed,
                                                         int32_t* __restrict__ out) {
  const int gx = gridDim.x;
  RpsHdr* h = w.h;
  __shared__ uint32_t s_tmp[kRpsThreads / 64];
  __shared__ int s_lb, s_bad;
  if (threadIdx.x == 0) {
    s_lb = static_cast<int>(atomicAdd(&h->ord[0], 1u));
    s_bad = 0;
  }
  __syncthreads();
  const int lb = s_lb;
  const uint64_t thr = h->thr;
  const int64_t base = static_cast<int64_t>(lb) * kRpsTile + static_cast<int64_t>(threadIdx.x) * kRpsPer;
  uint32_t keep = 0, cnt = 0;
#pragma unroll
  for (int k = 0; k < kRpsPer; ++k) {
    const int64_t i = base + k;
    if (i < n && rps_key(seed, i) <= thr) {
      keep |= 1u << k;
      ++cnt;
    }
  }
  uint32_t ex;
  const uint32_t tot = block_exclusive_scan<kRpsThreads>(cnt, &ex, s_tmp);
  if (threadIdx.x == 0) cmp_st_agent(&w.tcnt[lb], tot + 1u);
  uint32_t sum = 0;
  for (int i = threadIdx.x; i < lb; i += kRpsThreads) {
    uint32_t v, spins = 0;
    while ((v = cmp_ld_agent(&w.tcnt[i])) == 0u) {
      if (++spins > kCmpSpinLimit) {
        s_bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (v) sum += v - 1u;
  }
  const uint32_t before = block_sum_u32<kRpsThreads>(sum, s_tmp);
  if (s_bad) {
    if (threadIdx.x == 0) atomicOr(&h->bad[0], 1u);
  } else {
    uint32_t r = before + ex;
#pragma unroll
    for (int k = 0; k < kRpsPer; ++k) {
      if ((keep >> k) & 1u) {
        if (r < static_cast<uint64_t>(m)) out[r] = static_cast<int32_t>(base + k);
        ++r;
      }
    }
  }
  if (!rps_arrive_last(h, blockIdx.x, gx)) return;
  for (int i = threadIdx.x; i < gx; i += kRpsThreads) cmp_st_agent(&w.tcnt[i], 0u);
  if (threadIdx.x == 0) atomicExch(&h->ord[0], 0u);
}

__global__ void k_rps_identity(int64_t n, int32_t* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<int32_t>(i);
}

__global__ void k_rps_init(RpsWs w, int64_t ntile) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t* hz = reinterpret_cast<uint32_t*>(w.h);
  if (i < static_cast<int64_t>(sizeof(RpsHdr) / 4)) hz[i] = 0u;
  if (i < ntile) w.tcnt[i] = 0u;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct RpsLayout {
  size_t h, qp, tcnt, total;
};

RpsLayout rps_layout(int64_t n) {
  RpsLayout L;
  size_t o = 0;
  L.h = o;    o = align256(o + sizeof(RpsHdr));
  L.qp = o;   o = align256(o + static_cast<size_t>(kRpsQueue) * 8);
  L.tcnt = o; o = align256(o + static_cast<size_t>((n + kRpsTile - 1) / kRpsTile) * 4);
  L.total = o;
  return L;
}

}  // namespace
}  // namespace hav

using namespace hav;

extern "C" {

size_t hav_fps_workspace_size(int64_t N) {
  if (N < 1 || N > HAV_FPS_MAX_POINTS) return 0;
  return fps_ws_bytes();
}

hav_status_t hav_fps(const float* xyz, int64_t N, int64_t M, int64_t start, int32_t* idx, void* ws,
                     size_t ws_bytes, int32_t blocks, void* stream) {
  if (!xyz || !idx || !ws || N < 1 || N > HAV_FPS_MAX_POINTS || M < 1 || M > N || start < 0 ||
      start >= N || blocks < 0 || blocks > kFpsMaxBlocks)
    return HAV_ERR_INVALID_ARG;
  if (ws_bytes < fps_ws_bytes()) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  FpsSlot* slots = static_cast<FpsSlot*>(ws);
  uint32_t* err = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + 2 * kFpsMaxBlocks * sizeof(FpsSlot));
  // blocks of 1024 threads with up to kFpsMaxPer points each (registers); one block
  // while the cloud fits it, else as many as needed at the full load
  constexpr int64_t kPerBlock = 1024 * kFpsMaxPer;
  int B = blocks;
  if (B == 0) B = static_cast<int>((N + kPerBlock - 1) / kPerBlock);
  const int64_t per = (N + static_cast<int64_t>(B) * 1024 - 1) / (static_cast<int64_t>(B) * 1024);
  if (per > kFpsMaxPer) return HAV_ERR_INVALID_ARG;  // too few blocks for this cloud
  hipError_t e = hipSuccess;
  if (B > 1) {
    hipLaunchKernelGGL(k_fps_clear, dim3((2 * kFpsMaxBlocks + 255) / 256), dim3(256), 0, st, slots, err);
    if ((e = hipGetLastError()) != hipSuccess) return HAV_ERR_HIP;
  }
  if (per <= 1) e = launch_fps<1024, 1>(B, xyz, N, M, start, idx, slots, err, st);
  else if (per <= 2) e = launch_fps<1024, 2>(B, xyz, N, M, start, idx, slots, err, st);
  else e = launch_fps<1024, 4>(B, xyz, N, M, start, idx, slots, err, st);
  return e == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

hav_status_t hav_fps_error(const void* ws, uint32_t* flag_host) {
  if (!ws || !flag_host) return HAV_ERR_INVALID_ARG;
  const uint32_t* err =
      reinterpret_cast<const uint32_t*>(static_cast<const char*>(ws) + 2 * kFpsMaxBlocks * sizeof(FpsSlot));
  return hipMemcpy(flag_host, err, 4, hipMemcpyDeviceToHost) == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

size_t hav_rps_workspace_size(int64_t N) {
  if (N < 1 || N > HAV_RPS_MAX_POINTS) return 0;
  return rps_layout(N).total;
}

hav_status_t hav_rps_workspace_init(void* ws, size_t ws_bytes, int64_t N, void* stream) {
  if (!ws || N < 1 || N > HAV_RPS_MAX_POINTS) return HAV_ERR_INVALID_ARG;
  const RpsLayout L = rps_layout(N);
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  char* base = static_cast<char*>(ws);
  const RpsWs w{reinterpret_cast<RpsHdr*>(base + L.h), reinterpret_cast<unsigned long long*>(base + L.qp),
                reinterpret_cast<uint32_t*>(base + L.tcnt)};
  const int64_t ntile = (N + kRpsTile - 1) / kRpsTile;
  const int64_t cover = std::max<int64_t>(ntile, static_cast<int64_t>(sizeof(RpsHdr) / 4));
  hipLaunchKernelGGL(k_rps_init, dim3(static_cast<unsigned>((cover + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w, ntile);
  return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

hav_status_t hav_rps(int64_t N, int64_t M, uint64_t seed, float window, int32_t* idx, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!idx || !ws || N < 1 || N > HAV_RPS_MAX_POINTS || M < 1 || M > N || !std::isfinite(window) ||
      window > 64.0f)
    return HAV_ERR_INVALID_ARG;
  const RpsLayout L = rps_layout(N);
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (M == N) {
    hipLaunchKernelGGL(k_rps_identity, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, st, N, idx);
    return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
  }
  char* base = static_cast<char*>(ws);
  const RpsWs w{reinterpret_cast<RpsHdr*>(base + L.h), reinterpret_cast<unsigned long long*>(base + L.qp),
                reinterpret_cast<uint32_t*>(base + L.tcnt)};
  // window around the expected position of the M-th smallest key
  const double x = static_cast<double>(M) / (static_cast<double>(N) + 1.0);
  const double sd = std::sqrt(x * (1.0 - x) / (static_cast<double>(N) + 2.0));
  const double k = window == 0.0f ? kRpsSigma : static_cast<double>(window);
  const double lo = (x - k * sd) * 0x1p64, hi = (x + k * sd) * 0x1p64;
  unsigned long long blo = lo <= 0.0 ? 0ull : (lo >= 0x1p64 ? ~0ull : static_cast<unsigned long long>(lo));
  unsigned long long bhi = hi >= 0x1p64 ? ~0ull : (hi <= 0.0 ? 0ull : static_cast<unsigned long long>(hi));
  if (k < 0.0) {  // no window: an empty one (every key is above it), so the last block
    blo = 0ull;   // radix-selects over all keys
    bhi = 0ull;
  }
  const unsigned grid = static_cast<unsigned>((N + kRpsTile - 1) / kRpsTile);
  hipLaunchKernelGGL(k_rps_count, dim3(grid), dim3(kRpsThreads), 0, st, w, N, M, seed, blo, bhi);
  if (hipGetLastError() != hipSuccess) return HAV_ERR_HIP;
  hipLaunchKernelGGL(k_rps_out, dim3(grid), dim3(kRpsThreads), 0, st, w, N, M, seed, idx);
  return hipGetLastError() == hipSuccess ? HAV_OK : HAV_ERR_HIP;
}

}  // extern "C"
