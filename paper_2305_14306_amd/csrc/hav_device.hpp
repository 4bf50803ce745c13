// Device-side building blocks of the HAVSampler kernels (gfx950).
//
// Every floating-point step here is one correctly rounded binary32 operation; the
// library is compiled with -ffp-contract=off so that no multiply-add is fused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hav {

constexpr uint64_t kEmptyKey = ~0ull;      // packed keys use < 64 bits, never all ones
constexpr int kKeyBits = 21;               // bits per voxel coordinate in a packed key
constexpr float kKeyLimit = 2097152.0f;    // 2^21
constexpr int kBrickShift = 2;             // bricks of 4 x 4 x 4 voxels
constexpr int kBrickCoordBits = 19;        // 21 - 2

// Monotone map from a float to uint32 (IEEE total order: -0 < +0), so that the
// bounding box can be reduced with integer min/max.
__device__ __forceinline__ uint32_t float_to_ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_to_float(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

// Voxel coordinate along one axis (Sec. 3.2, Eq. 2) of a point already shifted into
// the stage frame (r = p - origin): g = floor(fl(r * inv)), inv = fl(1 / v).
__device__ __forceinline__ uint32_t axis_coord(float r, float inv) {
  const float q = r * inv;
  // q is never negative (r >= +0, inv > 0) and below 2^21, so converting with
  // truncation toward zero is exactly its floor
  return static_cast<uint32_t>(q);
}

__device__ __forceinline__ uint64_t pack_key(uint32_t gx, uint32_t gy, uint32_t gz) {
  return static_cast<uint64_t>(gx) | (static_cast<uint64_t>(gy) << kKeyBits) |
         (static_cast<uint64_t>(gz) << (2 * kKeyBits));
}

// Brick holding a voxel (4 x 4 x 4 voxels) and the voxel's bit inside the brick's
// 64-bit occupancy mask.
__device__ __forceinline__ uint64_t brick_key(uint32_t gx, uint32_t gy, uint32_t gz) {
  return static_cast<uint64_t>(gx >> kBrickShift) |
         (static_cast<uint64_t>(gy >> kBrickShift) << kBrickCoordBits) |
         (static_cast<uint64_t>(gz >> kBrickShift) << (2 * kBrickCoordBits));
}
__device__ __forceinline__ uint64_t brick_bit(uint32_t gx, uint32_t gy, uint32_t gz) {
  return 1ull << ((gx & 3u) | ((gy & 3u) << 2) | ((gz & 3u) << 4));
}

// Squared distance of a point to its voxel centre v * (g + 0.5) (Sec. 3.2, d_i),
// in the fixed order ((dx*dx + dy*dy) + dz*dz). Never negative, so its bit pattern
// orders like its value.
__device__ __forceinline__ float centre_dist2(float rx, float ry, float rz, uint32_t gx,
                                              uint32_t gy, uint32_t gz, float vx, float vy,
                                              float vz) {
  const float cx = vx * (static_cast<float>(gx) + 0.5f);
  const float cy = vy * (static_cast<float>(gy) + 0.5f);
  const float cz = vz * (static_cast<float>(gz) + 0.5f);
  const float dx = rx - cx;
  const float dy = ry - cy;
  const float dz = rz - cz;
  const float xx = dx * dx;
  const float yy = dy * dy;
  const float zz = dz * dz;
  const float xy = xx + yy;
  return xy + zz;
}

// Trim priority of a voxel: SplitMix64's output mix (Steele, Lea, Flood 2014) of
// its packed coordinate. Bijective, so priorities of distinct voxels never tie.
__device__ __forceinline__ uint64_t voxel_priority(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Table hashing: 64-bit finaliser (two multiplies) so that structured keys spread.
__device__ __forceinline__ uint32_t table_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDull;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ull;
  k ^= k >> 33;
  return static_cast<uint32_t>(k);
}

// Compare-and-swap returning the previous value.
__device__ __forceinline__ uint64_t lds_cas(uint64_t* p, uint64_t expected, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
  return expected;
}

// ------------------------------------------------------------------ block helpers

template <int kThreads>
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* s_tmp) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s_tmp[wv] = v;
  __syncthreads();
  uint32_t t = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) t += s_tmp[w];
  return t;
}

// Exclusive scan of one value per thread across the block; returns the block total.
template <int kThreads>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* excl,
                                                         uint32_t* s_tmp) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = static_cast<uint32_t>(__shfl_up(static_cast<int>(x), o, 64));
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) s_tmp[wv] = x;
  __syncthreads();
  uint32_t wbase = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wv) wbase += s_tmp[w];
    total += s_tmp[w];
  }
  *excl = wbase + x - v;
  return total;
}

}  // namespace hav
