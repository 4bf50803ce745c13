// Device-side building blocks of the HAVSampler kernels (gfx950).
//
// Every floating-point step here is one correctly rounded binary32 operation; the
// library is compiled with -ffp-contract=off so that no multiply-add is fused.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hav {

constexpr uint64_t kEmptyKey = ~0ull;  // packed voxel keys use 63 bits, never all ones
constexpr int kKeyBits = 21;           // bits per voxel coordinate in a packed key
constexpr float kKeyLimit = 2097152.0f;  // 2^21

// Monotone map from a float to uint32 (IEEE total order: -0 < +0), so that the
// bounding box can be reduced with integer atomics.
__device__ __forceinline__ uint32_t float_to_ordered(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float ordered_to_float(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// Voxel coordinate along one axis (Sec. 3.2, Eq. 2) in the stage frame:
// g = floor(fl(fl(p - origin) * inv)), with inv = fl(1 / v).
__device__ __forceinline__ uint32_t axis_coord(float p, float origin, float inv, float* r_out) {
  const float r = p - origin;
  const float q = r * inv;
  *r_out = r;
  return static_cast<uint32_t>(floorf(q));  // q in [0, 2^21): floor then exact convert
}

__device__ __forceinline__ uint64_t pack_key(uint32_t gx, uint32_t gy, uint32_t gz) {
  return static_cast<uint64_t>(gx) | (static_cast<uint64_t>(gy) << kKeyBits) |
         (static_cast<uint64_t>(gz) << (2 * kKeyBits));
}

// Squared distance of a point to its voxel centre v * (g + 0.5) (Sec. 3.2, d_i),
// in the fixed order ((dx*dx + dy*dy) + dz*dz). Never negative, so its bit pattern
// orders like its value.
__device__ __forceinline__ float centre_dist2(const float r[3], const uint32_t g[3],
                                              const float v[3]) {
  float d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float gc = static_cast<float>(g[a]) + 0.5f;
    const float centre = v[a] * gc;
    d[a] = r[a] - centre;
  }
  const float xx = d[0] * d[0];
  const float yy = d[1] * d[1];
  const float zz = d[2] * d[2];
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

// Home slot of a key in a power-of-two open-addressing table (multiplicative
// hashing, top bits).
__device__ __forceinline__ uint32_t home_slot(uint64_t key, int shift) {
  return static_cast<uint32_t>((key * 0xD6E8FEB86659FD93ull) >> shift);
}

// Insert-or-find with linear probing. Returns true if this call stored the key.
// A plain load first: a slot changes at most once (empty -> key) between clears,
// so a stale read can only show it empty, and the CAS then settles it.
__device__ __forceinline__ bool table_insert(unsigned long long* keys, uint32_t mask, int shift,
                                             uint64_t key, uint32_t* slot_out) {
  uint32_t s = home_slot(key, shift);
  while (true) {
    const unsigned long long k = keys[s];
    if (k == key) {
      *slot_out = s;
      return false;
    }
    if (k == kEmptyKey) {
      const unsigned long long prev = atomicCAS(&keys[s], kEmptyKey, key);
      if (prev == kEmptyKey) {
        *slot_out = s;
        return true;
      }
      if (prev == key) {
        *slot_out = s;
        return false;
      }
    }
    s = (s + 1) & mask;
  }
}

// Wave64 reductions.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o, 64)));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o, 64)));
  return v;
}

}  // namespace hav
