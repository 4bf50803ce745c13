// Sampling-quality context tools — TEST INFRASTRUCTURE ONLY (CPU).
//
// Farthest point sampling (arXiv 2305.14306, Sec. 3.1, Eq. 1), random point
// sampling, and the covering radius of a sample (largest distance from any cloud
// point to its nearest sampled point). The paper motivates the voxel sampler by the
// wide, even coverage of FPS (Sec. 3.1, Fig. 3) and times it against FPS and RPS
// (Sec. 4.2, Fig. 7); FPS and RPS here are the definitions the GPU comparators are
// checked against, bit for bit. Pins: FPS by a closed form on a line of equally
// spaced points and by its factor-2 bound on the k-centre optimum (brute force on
// tiny clouds); RPS by published SplitMix64 outputs.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <unordered_map>
#include <vector>

extern "C" {

// FPS (Eq. 1): start from `start`, then repeatedly take the point whose distance to
// the selected set is largest; ties go to the lowest index. Distances in double.
int32_t oracle_fps(const float* xyz, int64_t N, int64_t m, int64_t start, int32_t* out) {
  if (!xyz || !out || N < 1 || m < 1 || m > N || start < 0 || start >= N) return 1;
  std::vector<double> dist(static_cast<size_t>(N), std::numeric_limits<double>::infinity());
  int64_t cur = start;
  for (int64_t j = 0; j < m; ++j) {
    out[j] = static_cast<int32_t>(cur);
    const double cx = xyz[3 * cur], cy = xyz[3 * cur + 1], cz = xyz[3 * cur + 2];
    int64_t arg = 0;
    double best = -1.0;
    for (int64_t i = 0; i < N; ++i) {
      const double dx = xyz[3 * i] - cx, dy = xyz[3 * i + 1] - cy, dz = xyz[3 * i + 2] - cz;
      const double d = dx * dx + dy * dy + dz * dz;
      if (d < dist[i]) dist[i] = d;
      if (dist[i] > best) {
        best = dist[i];
        arg = i;
      }
    }
    cur = arg;
  }
  return 0;
}

// Random point sampling, the fast baseline of the latency comparison (Sec. 4.2,
// Fig. 7): point i gets the key splitmix64(seed + (i + 1) * golden gamma), output
// i + 1 of the SplitMix64 generator (Steele, Lea and Flood 2014) seeded with `seed`;
// the m points of smallest key are returned in ascending index order. Keys are
// distinct (the finaliser is a bijection of seed + (i+1) gamma, itself distinct for
// i < 2^64), so the set is unique.
static uint64_t sm64_finalise(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int32_t oracle_rps(int64_t N, int64_t m, uint64_t seed, int32_t* out) {
  if (!out || N < 1 || m < 1 || m > N) return 1;
  std::vector<std::pair<uint64_t, int64_t>> key(static_cast<size_t>(N));
  for (int64_t i = 0; i < N; ++i)
    key[i] = {sm64_finalise(seed + static_cast<uint64_t>(i + 1) * 0x9E3779B97F4A7C15ull), i};
  std::sort(key.begin(), key.end());
  std::vector<int64_t> pick;
  for (int64_t j = 0; j < m; ++j) pick.push_back(key[j].second);
  std::sort(pick.begin(), pick.end());
  for (int64_t j = 0; j < m; ++j) out[j] = static_cast<int32_t>(pick[j]);
  return 0;
}

// Covering radius: max over all points of the distance to the nearest point of idx.
// Exact nearest-neighbour search on a uniform grid of the sampled points, searched
// in growing shells of cells until no closer cell can remain.
double oracle_covering_radius(const float* xyz, int64_t N, const int32_t* idx, int64_t m) {
  if (!xyz || !idx || N < 1 || m < 1) return -1.0;
  double mn[3], mx[3];
  for (int a = 0; a < 3; ++a) {
    mn[a] = std::numeric_limits<double>::infinity();
    mx[a] = -std::numeric_limits<double>::infinity();
  }
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) {
      mn[a] = std::min(mn[a], static_cast<double>(xyz[3 * i + a]));
      mx[a] = std::max(mx[a], static_cast<double>(xyz[3 * i + a]));
    }
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= std::max(mx[a] - mn[a], 1e-9);
  const double h = std::max(std::cbrt(vol / static_cast<double>(m)) * 1.5, 1e-9);
  auto cell = [&](const float* p, int a) {
    return static_cast<int64_t>(std::floor((p[a] - mn[a]) / h));
  };
  auto pack = [](int64_t x, int64_t y, int64_t z) {
    return (static_cast<uint64_t>(x) & 0x1FFFFF) | ((static_cast<uint64_t>(y) & 0x1FFFFF) << 21) |
           ((static_cast<uint64_t>(z) & 0x1FFFFF) << 42);
  };
  std::unordered_map<uint64_t, std::vector<int32_t>> grid;
  int64_t cmax[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) cmax[a] = static_cast<int64_t>(std::floor((mx[a] - mn[a]) / h));
  for (int64_t j = 0; j < m; ++j) {
    const float* p = xyz + 3 * static_cast<int64_t>(idx[j]);
    grid[pack(cell(p, 0), cell(p, 1), cell(p, 2))].push_back(idx[j]);
  }
  const int64_t rmax = std::max({cmax[0], cmax[1], cmax[2]}) + 1;
  double worst = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    const float* p = xyz + 3 * i;
    const int64_t c0 = cell(p, 0), c1 = cell(p, 1), c2 = cell(p, 2);
    double best = std::numeric_limits<double>::infinity();
    for (int64_t r = 0; r <= rmax; ++r) {
      for (int64_t dx = -r; dx <= r; ++dx)
        for (int64_t dy = -r; dy <= r; ++dy)
          for (int64_t dz = -r; dz <= r; ++dz) {
            if (std::max({std::llabs(dx), std::llabs(dy), std::llabs(dz)}) != r) continue;
            const int64_t x = c0 + dx, y = c1 + dy, z = c2 + dz;
            if (x < 0 || y < 0 || z < 0 || x > cmax[0] || y > cmax[1] || z > cmax[2]) continue;
            auto it = grid.find(pack(x, y, z));
            if (it == grid.end()) continue;
            for (int32_t q : it->second) {
              const double ex = static_cast<double>(xyz[3 * q]) - p[0];
              const double ey = static_cast<double>(xyz[3 * q + 1]) - p[1];
              const double ez = static_cast<double>(xyz[3 * q + 2]) - p[2];
              best = std::min(best, ex * ex + ey * ey + ez * ez);
            }
          }
      // every sample in a ring beyond r is at least r*h away
      const double bound = static_cast<double>(r) * h;
      if (best <= bound * bound) break;
    }
    worst = std::max(worst, best);
  }
  return std::sqrt(worst);
}

}  // extern "C"
