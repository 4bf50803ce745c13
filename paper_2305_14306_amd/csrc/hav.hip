// HAVSampler for MI355X (gfx950): kernels and the C ABI of include/hav.h.
//
// One stage samples exactly M of N points (arXiv 2305.14306, Sec. 3):
//   frame   per-axis min/max, grid origin = min corner, search bracket hi0
//   layers  (Sec. 3.4, Eq. 3) for each layer l with budget m_l, on unsampled points:
//     search  adaptive voxel search (Sec. 3.3): bisection on the voxel scale s; each
//             step runs the voxel counter Cnt (Sec. 3.2 voxel hashing) and a one-thread
//             controller on the device, so the host never waits for a count
//     select  centre-closest point per occupied voxel (Sec. 3.2) via a 64-bit
//             atomicMin of (bits(d^2) << 32 | index): ties go to the lowest index
//     exact m trim by SplitMix64 priority of the voxel (radix select of the m-th
//             smallest) or pad with the lowest-index unsampled points
//     mask    tag[i] = layer number of the pick
//   output  ascending indices by a two-level scan over tag
//
// All state lives in the caller's workspace; nothing is allocated here.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/hav.h"
#include "hav_device.hpp"

namespace hav {
namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;  // elements per thread in the scan kernels
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

struct Frame {
  uint32_t mn_ord[3];
  uint32_t mx_ord[3];
  int32_t nonfinite;
  int32_t status;
  float mn[3];
  float mx[3];
  float hi0;
};

struct Ctrl {
  float lo, hi, s;
  float v[3], inv[3];  // voxel size and reciprocal of the size being evaluated / chosen
  int32_t evals, done, accepted, layer;
  uint32_t count;      // new keys found by the current evaluation
  uint32_t c_lo, c_hi;
  uint32_t ncand;      // occupied voxels at the chosen size
  uint32_t m, upper;
  uint64_t prefix;     // radix select: priority bits fixed so far
  uint32_t rank;       // rank sought inside the current prefix bucket
  uint32_t trim;       // 1 if ncand > m
  uint32_t ncap;       // candidate list capacity (points in the stage)
  uint32_t hist[kRadixBins];
};

struct KParams {
  float aspect[3];
  float fixed_v[3];
  int32_t fixed;
};

__device__ __forceinline__ bool failed(const Frame* f) { return f->status != HAV_OK; }

// ----------------------------------------------------------------------------- frame

__global__ void k_begin(Frame* f, hav_info_t* info) {
  const int t = threadIdx.x;
  if (t < 3) {
    f->mn_ord[t] = 0xFFFFFFFFu;
    f->mx_ord[t] = 0u;
  }
  if (t == 0) {
    f->nonfinite = 0;
    f->status = HAV_OK;
  }
  int32_t* w = reinterpret_cast<int32_t*>(info);
  for (int i = t; i < static_cast<int>(sizeof(hav_info_t) / 4); i += blockDim.x) w[i] = 0;
}

__global__ void __launch_bounds__(kThreads) k_bbox(const float* __restrict__ xyz, int64_t n,
                                                   Frame* f) {
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
  uint32_t hi[3] = {0u, 0u, 0u};
  int bad = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float c = xyz[3 * i + a];
      bad |= !isfinite(c);
      const uint32_t o = float_to_ordered(c);
      lo[a] = min(lo[a], o);
      hi[a] = max(hi[a], o);
    }
  }
  __shared__ uint32_t s_lo[3][kThreads / 64], s_hi[3][kThreads / 64];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t l = wave_min_u32(lo[a]);
    const uint32_t h = wave_max_u32(hi[a]);
    if (lane == 0) {
      s_lo[a][wv] = l;
      s_hi[a][wv] = h;
    }
  }
  if (bad) s_bad = 1;
  __syncthreads();
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    uint32_t l = s_lo[a][0], h = s_hi[a][0];
    for (int w = 1; w < kThreads / 64; ++w) {
      l = min(l, s_lo[a][w]);
      h = max(h, s_hi[a][w]);
    }
    atomicMin(&f->mn_ord[a], l);
    atomicMax(&f->mx_ord[a], h);
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(&f->nonfinite, 1);
}

// Single thread: decode the box, compute hi0 and check the frame.
__global__ void k_frame(Frame* f, hav_info_t* info, KParams kp, int identity) {
  if (threadIdx.x != 0) return;
  if (f->nonfinite) {
    f->status = HAV_ERR_NONFINITE;
    info->status = HAV_ERR_NONFINITE;
    return;
  }
  float E = 0.0f;
  for (int a = 0; a < 3; ++a) {
    f->mn[a] = ordered_to_float(f->mn_ord[a]);
    f->mx[a] = ordered_to_float(f->mx_ord[a]);
    info->mn[a] = f->mn[a];
    info->mx[a] = f->mx[a];
    const float ext = f->mx[a] - f->mn[a];
    const float e = ext / kp.aspect[a];
    if (!(e <= E)) E = e;
  }
  if (identity) return;  // M == N: every point is kept, no frame checks apply
  if (!(E <= 0x1p100f)) {
    f->status = HAV_ERR_UNSUPPORTED;
    info->status = HAV_ERR_UNSUPPORTED;
    return;
  }
  // smallest power of two >= max(E, 2^-64); E is then a normal number
  const float Ec = E < 0x1p-64f ? 0x1p-64f : E;
  const uint32_t bits = __float_as_uint(Ec);
  const float hi0 = (bits & 0x7FFFFFu) ? __uint_as_float((bits & 0x7F800000u) + 0x00800000u) : Ec;
  f->hi0 = hi0;
  info->hi0 = hi0;
  if (kp.fixed) {
    for (int a = 0; a < 3; ++a) {
      const float inv = 1.0f / kp.fixed_v[a];
      const float q = (f->mx[a] - f->mn[a]) * inv;
      if (!(q < kKeyLimit)) {
        f->status = HAV_ERR_UNSUPPORTED;
        info->status = HAV_ERR_UNSUPPORTED;
        return;
      }
    }
  }
}

// ----------------------------------------------------------------------------- search

__device__ void set_scale(Ctrl* c, float s, const KParams& kp) {
  for (int a = 0; a < 3; ++a) {
    c->v[a] = s * kp.aspect[a];
    c->inv[a] = 1.0f / c->v[a];
  }
}

__global__ void k_layer_begin(const Frame* f, Ctrl* c, hav_info_t* info, KParams kp, int layer,
                              uint32_t m, uint32_t upper, uint32_t ncap) {
  if (threadIdx.x != 0 || failed(f)) return;
  c->lo = 0.0f;
  c->hi = f->hi0;
  c->evals = 0;
  c->accepted = 0;
  c->count = 0;
  c->c_lo = c->c_hi = 0;
  c->ncand = 0;
  c->ncap = ncap;
  c->m = m;
  c->upper = upper;
  c->layer = layer;
  info->m[layer] = static_cast<int32_t>(m);
  info->layers = layer + 1;
  if (kp.fixed) {
    c->done = 1;
    c->s = 0.0f;
    for (int a = 0; a < 3; ++a) {
      c->v[a] = kp.fixed_v[a];
      c->inv[a] = 1.0f / kp.fixed_v[a];
    }
  } else {
    c->done = 0;
    c->s = (c->lo + c->hi) * 0.5f;
    set_scale(c, c->s, kp);
  }
}

__global__ void __launch_bounds__(kThreads) k_fill_u64(unsigned long long* p, int64_t n,
                                                       unsigned long long value, const Frame* f,
                                                       const Ctrl* c) {
  if (failed(f) || (c && c->done)) return;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = value;
}

// Voxel counter Cnt (Sec. 3.3): distinct voxel keys among the unsampled points.
__global__ void __launch_bounds__(kThreads) k_count(const float* __restrict__ xyz, int64_t n,
                                                    const uint8_t* __restrict__ tag,
                                                    const Frame* f, Ctrl* c,
                                                    unsigned long long* keys, uint32_t mask,
                                                    int shift) {
  if (failed(f) || c->done) return;
  const float o0 = f->mn[0], o1 = f->mn[1], o2 = f->mn[2];
  const float i0 = c->inv[0], i1 = c->inv[1], i2 = c->inv[2];
  uint32_t mine = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    if (tag[i]) continue;
    float r;
    const uint32_t gx = axis_coord(xyz[3 * i + 0], o0, i0, &r);
    const uint32_t gy = axis_coord(xyz[3 * i + 1], o1, i1, &r);
    const uint32_t gz = axis_coord(xyz[3 * i + 2], o2, i2, &r);
    uint32_t slot;
    mine += table_insert(keys, mask, shift, pack_key(gx, gy, gz), &slot) ? 1u : 0u;
  }
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (mine) atomicAdd(&s_sum, mine);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(&c->count, s_sum);
}

// One bisection step of the adaptive voxel search (Sec. 3.3).
__global__ void k_ctrl(const Frame* f, Ctrl* c, hav_info_t* info, KParams kp, int t_max) {
  if (threadIdx.x != 0 || failed(f) || c->done) return;
  const uint32_t cnt = c->count;
  c->count = 0;
  c->evals += 1;
  const float s = c->s;
  const int L = c->layer;
  if (cnt >= c->m && cnt <= c->upper) {
    c->accepted = 1;
    c->done = 1;  // v, inv already hold this size
  } else {
    if (cnt < c->m) {
      c->hi = s;
      c->c_hi = cnt;
    } else {
      c->lo = s;
      c->c_lo = cnt;
    }
    if (c->evals >= t_max) {
      // no size in the window: the finest size with too many voxels if any (trim),
      // else the smallest size evaluated (pad)
      c->s = (c->lo > 0.0f) ? c->lo : c->hi;
      set_scale(c, c->s, kp);
      c->done = 1;
    } else {
      c->s = (c->lo + c->hi) * 0.5f;
      set_scale(c, c->s, kp);
    }
  }
  info->evals[L] = c->evals;
  info->accepted[L] = c->accepted;
  info->s[L] = c->done ? c->s : 0.0f;
}

// ----------------------------------------------------------------------------- select

// Centre-closest representative of every occupied voxel at the chosen size.
__global__ void __launch_bounds__(kThreads) k_select(const float* __restrict__ xyz, int64_t n,
                                                     const uint8_t* __restrict__ tag,
                                                     const Frame* f, Ctrl* c,
                                                     unsigned long long* keys,
                                                     unsigned long long* vals, uint32_t mask,
                                                     int shift) {
  if (failed(f)) return;
  const float v[3] = {c->v[0], c->v[1], c->v[2]};
  const float inv[3] = {c->inv[0], c->inv[1], c->inv[2]};
  const float o[3] = {f->mn[0], f->mn[1], f->mn[2]};
  uint32_t mine = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    if (tag[i]) continue;
    float r[3];
    uint32_t g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] = axis_coord(xyz[3 * i + a], o[a], inv[a], &r[a]);
    uint32_t slot;
    mine += table_insert(keys, mask, shift, pack_key(g[0], g[1], g[2]), &slot) ? 1u : 0u;
    const float d2 = centre_dist2(r, g, v);
    const unsigned long long packed =
        (static_cast<unsigned long long>(__float_as_uint(d2)) << 32) | static_cast<uint32_t>(i);
    atomicMin(&vals[slot], packed);
  }
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  if (mine) atomicAdd(&s_sum, mine);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(&c->ncand, s_sum);
}

// Turn the occupied slots into a candidate list (priority, point index).
__global__ void __launch_bounds__(kThreads) k_collect(const unsigned long long* keys,
                                                      const unsigned long long* vals,
                                                      uint32_t cap, const Frame* f, Ctrl* c,
                                                      uint64_t* cand_prio, int32_t* cand_idx,
                                                      uint32_t* cursor, int64_t n) {
  if (failed(f)) return;
  for (int64_t s = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; s < cap;
       s += static_cast<int64_t>(gridDim.x) * kThreads) {
    const unsigned long long k = keys[s];
    const bool occ = (k != kEmptyKey);
    const uint64_t bal = __ballot(occ);
    if (!bal) continue;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll(static_cast<unsigned long long>(bal)) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cursor, static_cast<uint32_t>(__popcll(bal)));
    base = __shfl(base, leader, 64);
    if (occ) {
      const uint32_t off = base + __popcll(bal & ((1ull << lane) - 1ull));
      if (off < n) {  // at most n distinct keys; the bound only guards the store
        cand_prio[off] = voxel_priority(k);
        cand_idx[off] = static_cast<int32_t>(vals[s] & 0xFFFFFFFFu);
      }
    }
  }
}

__global__ void k_trim_begin(const Frame* f, Ctrl* c, hav_info_t* info) {
  if (failed(f)) return;
  const int t = threadIdx.x;
  for (int i = t; i < kRadixBins; i += blockDim.x) c->hist[i] = 0;
  if (t == 0) {
    const uint32_t nc = c->ncand;
    const int L = c->layer;
    c->trim = nc > c->m ? 1u : 0u;
    c->prefix = 0;
    c->rank = c->m - 1;  // 0-based rank of the m-th smallest priority
    info->count[L] = static_cast<int32_t>(nc);
    info->trimmed[L] = nc > c->m ? static_cast<int32_t>(nc - c->m) : 0;
    info->padded[L] = nc < c->m ? static_cast<int32_t>(c->m - nc) : 0;
    if (!c->accepted) info->s[L] = c->s;
  }
}

// Radix select over the 64-bit priorities, kRadixBits per pass from the top.
__global__ void __launch_bounds__(kThreads) k_radix_hist(const uint64_t* __restrict__ prio,
                                                         const Frame* f, Ctrl* c, int pass) {
  if (failed(f) || !c->trim) return;
  __shared__ uint32_t h[kRadixBins];
  for (int i = threadIdx.x; i < kRadixBins; i += kThreads) h[i] = 0;
  __syncthreads();
  const uint32_t nc = min(c->ncand, c->ncap);
  const int shift = 64 - kRadixBits * (pass + 1);
  const int hi_shift = shift + kRadixBits;  // bits above this digit must equal prefix
  const uint64_t pref = c->prefix;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < nc;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const uint64_t p = prio[i];
    if (hi_shift < 64 && (p >> hi_shift) != (pref >> hi_shift)) continue;
    atomicAdd(&h[(p >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kRadixBins; i += kThreads)
    if (h[i]) atomicAdd(&c->hist[i], h[i]);
}

__global__ void k_radix_pick(const Frame* f, Ctrl* c, int pass) {
  if (failed(f) || !c->trim) return;
  if (threadIdx.x == 0) {
    const int shift = 64 - kRadixBits * (pass + 1);
    uint32_t rank = c->rank;
    uint32_t acc = 0;
    int b = 0;
    for (; b < kRadixBins; ++b) {
      const uint32_t h = c->hist[b];
      if (rank < acc + h) break;
      acc += h;
    }
    c->rank = rank - acc;
    c->prefix |= static_cast<uint64_t>(b) << shift;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kRadixBins; i += blockDim.x) c->hist[i] = 0;
}

// Mark the kept representatives: all of them, or those with priority <= the m-th
// smallest (c->prefix after the last pass).
__global__ void __launch_bounds__(kThreads) k_mark(const uint64_t* __restrict__ prio,
                                                   const int32_t* __restrict__ idx,
                                                   const Frame* f, const Ctrl* c, uint8_t* tag,
                                                   int64_t n) {
  if (failed(f)) return;
  const uint32_t nc = min(static_cast<int64_t>(c->ncand), n);
  const bool trim = c->trim;
  const uint64_t thr = c->prefix;
  const uint8_t t = static_cast<uint8_t>(c->layer + 1);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < nc;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int32_t j = idx[i];
    if ((!trim || prio[i] <= thr) && j >= 0 && j < n) tag[j] = t;
  }
}

// ----------------------------------------------------------------------------- scans

// Block-exclusive scan of one value per thread; returns the block total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* excl) {
  __shared__ uint32_t s_w[kThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wv] = x;
  __syncthreads();
  uint32_t wbase = 0, total = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wv) wbase += s_w[w];
    total += s_w[w];
  }
  *excl = wbase + x - v;
  __syncthreads();
  return total;
}

// mode 0: count tag == 0 (pad candidates); mode 1: count tag != 0 (output)
__device__ __forceinline__ bool scan_pred(uint8_t t, int mode) { return mode ? (t != 0) : (t == 0); }

__global__ void __launch_bounds__(kThreads) k_tile_count(const uint8_t* __restrict__ tag, int64_t n,
                                                         uint32_t* tile_sums, int mode,
                                                         const Frame* f, const Ctrl* c) {
  if (failed(f)) return;
  if (mode == 0 && c->ncand >= c->m) return;  // no pad needed
  const int64_t base = blockIdx.x * static_cast<int64_t>(kScanTile) + threadIdx.x * kScanItems;
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n && scan_pred(tag[base + k], mode)) ++cnt;
  uint32_t excl;
  const uint32_t tot = block_exclusive_scan(cnt, &excl);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place (one block, sequential over chunks).
__global__ void __launch_bounds__(kThreads) k_scan_tiles(uint32_t* tile_sums, int64_t ntiles,
                                                         int mode, const Frame* f, const Ctrl* c) {
  if (failed(f)) return;
  if (mode == 0 && c->ncand >= c->m) return;
  uint32_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += kThreads) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < ntiles ? tile_sums[i] : 0u;
    uint32_t excl;
    const uint32_t tot = block_exclusive_scan(v, &excl);
    if (i < ntiles) tile_sums[i] = carry + excl;
    carry += tot;
  }
}

// Pad: mark the lowest-index unsampled points until the layer has m picks.
__global__ void __launch_bounds__(kThreads) k_pad_mark(uint8_t* tag, int64_t n,
                                                       const uint32_t* tile_sums, const Frame* f,
                                                       const Ctrl* c) {
  if (failed(f) || c->ncand >= c->m) return;
  const uint32_t need = c->m - c->ncand;
  const uint8_t lt = static_cast<uint8_t>(c->layer + 1);
  const int64_t base = blockIdx.x * static_cast<int64_t>(kScanTile) + threadIdx.x * kScanItems;
  uint8_t t[kScanItems];
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    t[k] = base + k < n ? tag[base + k] : 1;
    cnt += (t[k] == 0);
  }
  uint32_t excl;
  block_exclusive_scan(cnt, &excl);
  uint32_t r = tile_sums[blockIdx.x] + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (t[k] == 0) {
      if (r < need) tag[base + k] = lt;
      ++r;
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_out_write(const uint8_t* __restrict__ tag, int64_t n,
                                                        const uint32_t* tile_sums, int32_t* idx,
                                                        int64_t M, const Frame* f) {
  if (failed(f)) return;
  const int64_t base = blockIdx.x * static_cast<int64_t>(kScanTile) + threadIdx.x * kScanItems;
  uint8_t t[kScanItems];
  uint32_t cnt = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    t[k] = base + k < n ? tag[base + k] : 0;
    cnt += (t[k] != 0);
  }
  uint32_t excl;
  block_exclusive_scan(cnt, &excl);
  uint32_t r = tile_sums[blockIdx.x] + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (t[k]) {
      if (r < M) idx[r] = static_cast<int32_t>(base + k);
      ++r;
    }
}

__global__ void __launch_bounds__(kThreads) k_iota(int32_t* idx, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    idx[i] = static_cast<int32_t>(i);
}

__global__ void __launch_bounds__(kThreads) k_zero_u8(uint8_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = 0;
}

__global__ void k_copy_info(const hav_info_t* src, hav_info_t* dst) {
  const int32_t* s = reinterpret_cast<const int32_t*>(src);
  int32_t* d = reinterpret_cast<int32_t*>(dst);
  for (int i = threadIdx.x; i < static_cast<int>(sizeof(hav_info_t) / 4); i += blockDim.x) d[i] = s[i];
}

// ----------------------------------------------------------------------------- chain

__global__ void __launch_bounds__(kThreads) k_gather(const float* __restrict__ xyz, int64_t n,
                                                     const int32_t* __restrict__ idx, int64_t m,
                                                     float* out) {
  for (int64_t q = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; q < 3 * m;
       q += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t p = q / 3;
    const int a = static_cast<int>(q - 3 * p);
    const int64_t j = idx[p];
    out[q] = (j >= 0 && j < n) ? xyz[3 * j + a] : 0.0f;
  }
}

__global__ void __launch_bounds__(kThreads) k_compose(const int32_t* __restrict__ local, int64_t m,
                                                      const int32_t* __restrict__ prev,
                                                      int64_t n_prev, int32_t* out) {
  for (int64_t q = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; q < m;
       q += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int64_t j = local[q];
    out[q] = (j >= 0 && j < n_prev) ? prev[j] : -1;
  }
}

// ============================================================================ host side

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t frame = 0, ctrl = 0, info = 0, cursor = 0, tag = 0, keys = 0, vals = 0, prio = 0,
         cidx = 0, tiles = 0, total = 0;
  uint32_t cap = 0;
  int shift = 0;
  int64_t ntiles = 0;
};

Layout make_layout(int64_t n) {
  Layout L;
  uint64_t cap = 1024;
  while (cap < 2 * static_cast<uint64_t>(n)) cap <<= 1;
  L.cap = static_cast<uint32_t>(cap);
  int lg = 0;
  while ((1ull << lg) < cap) ++lg;
  L.shift = 64 - lg;
  L.ntiles = (n + kScanTile - 1) / kScanTile;
  size_t o = 0;
  L.frame = o;  o = align_up(o + sizeof(Frame));
  L.ctrl = o;   o = align_up(o + sizeof(Ctrl));
  L.info = o;   o = align_up(o + sizeof(hav_info_t));
  L.cursor = o; o = align_up(o + sizeof(uint32_t));
  L.tag = o;    o = align_up(o + static_cast<size_t>(n));
  L.keys = o;   o = align_up(o + cap * 8);
  L.vals = o;   o = align_up(o + cap * 8);
  L.prio = o;   o = align_up(o + static_cast<size_t>(n) * 8);
  L.cidx = o;   o = align_up(o + static_cast<size_t>(n) * 4);
  L.tiles = o;  o = align_up(o + static_cast<size_t>(L.ntiles) * 4);
  L.total = o;
  return L;
}

bool params_ok(const hav_params_t* p) {
  if (!p || p->abi_version != HAV_ABI_VERSION) return false;
  if (p->layers < 1 || p->layers > HAV_MAX_LAYERS) return false;
  if (p->layer_ratio < 2 || p->layer_ratio > 16) return false;
  if (p->t_max < 1 || p->t_max > 20) return false;
  if (!std::isfinite(p->sigma) || p->sigma < 0.0 || p->sigma > 16.0) return false;
  if (p->flags & ~HAV_FIXED_VOXEL) return false;
  for (int a = 0; a < 3; ++a) {
    const float as = p->aspect[a];
    if (!std::isfinite(as) || as < 0x1p-16f || as > 0x1p16f) return false;
    if (p->flags & HAV_FIXED_VOXEL) {
      const float fv = p->fixed_voxel[a];
      if (!std::isfinite(fv) || fv < 0x1p-100f || fv > 0x1p100f) return false;
    }
  }
  return true;
}

// m_l = M r^(l-1) (r-1) / (r^k - 1), floored for l < k; the last layer takes the rest.
void layer_sizes(int64_t M, int k, int r, int64_t* m) {
  uint64_t rk = 1;
  for (int l = 0; l < k; ++l) rk *= static_cast<uint64_t>(r);
  uint64_t rl = 1;
  int64_t used = 0;
  for (int l = 0; l < k - 1; ++l) {
    m[l] = static_cast<int64_t>(static_cast<uint64_t>(M) * rl * static_cast<uint64_t>(r - 1) / (rk - 1));
    used += m[l];
    rl *= static_cast<uint64_t>(r);
  }
  m[k - 1] = M - used;
}

int grid_for(int64_t work, int per_block = kThreads) {
  const int64_t g = (work + per_block - 1) / per_block;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 4096)));
}

#define HAV_LAUNCH(...)                              \
  do {                                               \
    hipLaunchKernelGGL(__VA_ARGS__);                 \
    if (hipGetLastError() != hipSuccess) return HAV_ERR_HIP; \
  } while (0)

hav_status_t run_stage(const float* xyz, int64_t N, int64_t M, const hav_params_t* p, int32_t* idx,
                       char* ws, hav_info_t* info_dev, hipStream_t st) {
  const Layout L = make_layout(N);
  Frame* f = reinterpret_cast<Frame*>(ws + L.frame);
  Ctrl* c = reinterpret_cast<Ctrl*>(ws + L.ctrl);
  hav_info_t* info = reinterpret_cast<hav_info_t*>(ws + L.info);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(ws + L.cursor);
  uint8_t* tag = reinterpret_cast<uint8_t*>(ws + L.tag);
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(ws + L.keys);
  unsigned long long* vals = reinterpret_cast<unsigned long long*>(ws + L.vals);
  uint64_t* prio = reinterpret_cast<uint64_t*>(ws + L.prio);
  int32_t* cidx = reinterpret_cast<int32_t*>(ws + L.cidx);
  uint32_t* tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);

  KParams kp{};
  for (int a = 0; a < 3; ++a) {
    kp.aspect[a] = p->aspect[a];
    kp.fixed_v[a] = p->fixed_voxel[a];
  }
  kp.fixed = (p->flags & HAV_FIXED_VOXEL) ? 1 : 0;
  const bool identity = (M == N);

  HAV_LAUNCH(k_begin, dim3(1), dim3(64), 0, st, f, info);
  HAV_LAUNCH(k_bbox, dim3(grid_for(N)), dim3(kThreads), 0, st, xyz, N, f);
  HAV_LAUNCH(k_frame, dim3(1), dim3(1), 0, st, f, info, kp, identity ? 1 : 0);
  if (identity) {
    HAV_LAUNCH(k_iota, dim3(grid_for(N)), dim3(kThreads), 0, st, idx, N);
  } else {
    HAV_LAUNCH(k_zero_u8, dim3(grid_for(N)), dim3(kThreads), 0, st, tag, N);
    int64_t m[HAV_MAX_LAYERS];
    layer_sizes(M, p->layers, p->layer_ratio, m);
    int out_layer = 0;
    for (int l = 0; l < p->layers; ++l) {
      if (m[l] == 0) continue;
      const int lay = out_layer++;
      const double up = std::floor(static_cast<double>(m[l]) * (1.0 + p->sigma));
      const uint32_t upper = up >= 2147483647.0 ? 0x7FFFFFFFu : static_cast<uint32_t>(up);
      HAV_LAUNCH(k_layer_begin, dim3(1), dim3(1), 0, st, f, c, info, kp, lay,
                 static_cast<uint32_t>(m[l]), upper, static_cast<uint32_t>(N));
      if (!kp.fixed) {
        for (int t = 0; t < p->t_max; ++t) {
          HAV_LAUNCH(k_fill_u64, dim3(grid_for(L.cap)), dim3(kThreads), 0, st, keys,
                     static_cast<int64_t>(L.cap), kEmptyKey, f, c);
          HAV_LAUNCH(k_count, dim3(grid_for(N)), dim3(kThreads), 0, st, xyz, N, tag, f, c, keys,
                     L.cap - 1, L.shift);
          HAV_LAUNCH(k_ctrl, dim3(1), dim3(1), 0, st, f, c, info, kp, p->t_max);
        }
      }
      HAV_LAUNCH(k_fill_u64, dim3(grid_for(L.cap)), dim3(kThreads), 0, st, keys,
                 static_cast<int64_t>(L.cap), kEmptyKey, f, nullptr);
      HAV_LAUNCH(k_fill_u64, dim3(grid_for(L.cap)), dim3(kThreads), 0, st, vals,
                 static_cast<int64_t>(L.cap), ~0ull, f, nullptr);
      HAV_LAUNCH(k_fill_u64, dim3(1), dim3(64), 0, st,
                 reinterpret_cast<unsigned long long*>(cursor), 1, 0ull, f, nullptr);
      HAV_LAUNCH(k_select, dim3(grid_for(N)), dim3(kThreads), 0, st, xyz, N, tag, f, c, keys, vals,
                 L.cap - 1, L.shift);
      HAV_LAUNCH(k_collect, dim3(grid_for(L.cap)), dim3(kThreads), 0, st, keys, vals, L.cap, f, c,
                 prio, cidx, cursor, N);
      HAV_LAUNCH(k_trim_begin, dim3(1), dim3(kThreads), 0, st, f, c, info);
      for (int pass = 0; pass < 64 / kRadixBits; ++pass) {
        HAV_LAUNCH(k_radix_hist, dim3(grid_for(N)), dim3(kThreads), 0, st, prio, f, c, pass);
        HAV_LAUNCH(k_radix_pick, dim3(1), dim3(kThreads), 0, st, f, c, pass);
      }
      HAV_LAUNCH(k_mark, dim3(grid_for(N)), dim3(kThreads), 0, st, prio, cidx, f, c, tag, N);
      HAV_LAUNCH(k_tile_count, dim3(static_cast<unsigned>(L.ntiles)), dim3(kThreads), 0, st, tag, N,
                 tiles, 0, f, c);
      HAV_LAUNCH(k_scan_tiles, dim3(1), dim3(kThreads), 0, st, tiles, L.ntiles, 0, f, c);
      HAV_LAUNCH(k_pad_mark, dim3(static_cast<unsigned>(L.ntiles)), dim3(kThreads), 0, st, tag, N,
                 tiles, f, c);
    }
    HAV_LAUNCH(k_tile_count, dim3(static_cast<unsigned>(L.ntiles)), dim3(kThreads), 0, st, tag, N,
               tiles, 1, f, c);
    HAV_LAUNCH(k_scan_tiles, dim3(1), dim3(kThreads), 0, st, tiles, L.ntiles, 1, f, c);
    HAV_LAUNCH(k_out_write, dim3(static_cast<unsigned>(L.ntiles)), dim3(kThreads), 0, st, tag, N,
               tiles, idx, M, f);
  }
  if (info_dev) HAV_LAUNCH(k_copy_info, dim3(1), dim3(64), 0, st, info, info_dev);
  return HAV_OK;
}

bool chain_sizes_ok(int64_t N, const int64_t* M, int32_t n) {
  if (!M || n < 1 || n > 64) return false;
  int64_t prev = N;
  for (int32_t j = 0; j < n; ++j) {
    if (M[j] < 1 || M[j] > prev) return false;
    prev = M[j];
  }
  return true;
}

struct ChainLayout {
  size_t stage_ws = 0, buf0 = 0, buf1 = 0, local = 0, total = 0;
};

ChainLayout make_chain_layout(int64_t N, const int64_t* M, int32_t n) {
  ChainLayout C;
  C.stage_ws = 0;
  size_t o = align_up(make_layout(N).total);  // stage 0 is the largest stage
  C.buf0 = o; o = align_up(o + static_cast<size_t>(M[0]) * 12);
  C.buf1 = o; o = align_up(o + static_cast<size_t>(M[0]) * 12);
  C.local = o; o = align_up(o + static_cast<size_t>(M[0]) * 4);
  C.total = o;
  (void)n;
  return C;
}

}  // namespace
}  // namespace hav

using namespace hav;

extern "C" {

hav_params_t hav_params_default(void) {
  hav_params_t p;
  std::memset(&p, 0, sizeof(p));
  p.abi_version = HAV_ABI_VERSION;
  p.layers = 2;
  p.layer_ratio = 4;
  p.t_max = 20;
  p.sigma = 0.05;
  for (int a = 0; a < 3; ++a) {
    p.aspect[a] = 1.0f;
    p.fixed_voxel[a] = 1.0f;
  }
  p.flags = 0;
  return p;
}

const char* hav_status_string(hav_status_t s) {
  switch (s) {
    case HAV_OK: return "ok";
    case HAV_ERR_INVALID_ARG: return "invalid argument";
    case HAV_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case HAV_ERR_OUT_OF_MEMORY: return "out of memory";
    case HAV_ERR_UNSUPPORTED: return "unsupported input frame";
    case HAV_ERR_NONFINITE: return "non-finite coordinate";
    case HAV_ERR_HIP: return "HIP error";
  }
  return "unknown status";
}

size_t hav_workspace_size(int64_t N, int64_t M, const hav_params_t* params) {
  if (N < 1 || M < 1 || M > N || N >= (int64_t(1) << 31) || !params_ok(params)) return 0;
  return make_layout(N).total;
}

hav_status_t hav_sample(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                        int32_t* idx, void* ws, size_t ws_bytes, hav_info_t* info_dev,
                        void* stream) {
  if (!xyz || !idx || !ws || N < 1 || M < 1 || M > N || N >= (int64_t(1) << 31) ||
      !params_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  if (ws_bytes < make_layout(N).total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  return run_stage(xyz, N, M, params, idx, static_cast<char*>(ws), info_dev,
                   static_cast<hipStream_t>(stream));
}

size_t hav_chain_workspace_size(int64_t N, const int64_t* M_host, int32_t n_stages,
                                const hav_params_t* params) {
  if (N < 1 || N >= (int64_t(1) << 31) || !params_ok(params) ||
      !chain_sizes_ok(N, M_host, n_stages))
    return 0;
  return make_chain_layout(N, M_host, n_stages).total;
}

hav_status_t hav_sample_chain(const float* xyz, int64_t N, const int64_t* M_host,
                              int32_t n_stages, const hav_params_t* params, int32_t* idx_concat,
                              void* ws, size_t ws_bytes, hav_info_t* info_dev, void* stream) {
  if (!xyz || !idx_concat || !ws || N < 1 || N >= (int64_t(1) << 31) || !params_ok(params) ||
      !chain_sizes_ok(N, M_host, n_stages))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const ChainLayout C = make_chain_layout(N, M_host, n_stages);
  if (ws_bytes < C.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  float* bufs[2] = {reinterpret_cast<float*>(base + C.buf0), reinterpret_cast<float*>(base + C.buf1)};
  int32_t* local = reinterpret_cast<int32_t*>(base + C.local);
  const float* cur = xyz;
  int64_t n = N;
  int64_t off = 0, prev_off = 0;
  for (int32_t j = 0; j < n_stages; ++j) {
    const int64_t m = M_host[j];
    int32_t* out = idx_concat + off;
    int32_t* dst = (j == 0) ? out : local;
    const hav_status_t s = run_stage(cur, n, m, params, dst, base, info_dev ? info_dev + j : nullptr, st);
    if (s != HAV_OK) return s;
    if (j > 0)
      HAV_LAUNCH(k_compose, dim3(grid_for(m)), dim3(kThreads), 0, st, local, m,
                 idx_concat + prev_off, n, out);
    if (j + 1 < n_stages) {
      float* nxt = bufs[j & 1];
      HAV_LAUNCH(k_gather, dim3(grid_for(3 * m)), dim3(kThreads), 0, st, cur, n, dst, m, nxt);
      cur = nxt;
    }
    prev_off = off;
    off += m;
    n = m;
  }
  return HAV_OK;
}

}  // extern "C"
