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

// Squared distance from every query to its nearest sample, in double as
// ((ex*ex + ey*ey) + ez*ez) with ex = sample - query: brute force over all pairs.
// exclude_self: query j is sample j and does not count as its own neighbour.
void nn_d2(const float* smp, int64_t M, const float* qry, int64_t Q, int exclude_self, double* out) {
  for (int64_t i = 0; i < Q; ++i) {
    const double px = qry[3 * i], py = qry[3 * i + 1], pz = qry[3 * i + 2];
    double best = std::numeric_limits<double>::infinity();
    for (int64_t q = 0; q < M; ++q) {
      if (exclude_self && q == i) continue;
      const double ex = static_cast<double>(smp[3 * q]) - px;
      const double ey = static_cast<double>(smp[3 * q + 1]) - py;
      const double ez = static_cast<double>(smp[3 * q + 2]) - pz;
      best = std::min(best, ex * ex + ey * ey + ez * ez);
    }
    out[i] = best;
  }
}

int32_t oracle_nn_d2(const float* samples, int64_t M, const float* queries, int64_t Q,
                     int32_t exclude_self, double* out) {
  if (!samples || !queries || !out || M < 1 || Q < 1 || (exclude_self && (Q != M || M < 2))) return 1;
  nn_d2(samples, M, queries, Q, exclude_self, out);
  return 0;
}

// Ball query, the grouping step after sampling: for centre j the lowest-index points
// with d2 < r2 (float32, ((dx*dx + dy*dy) + dz*dz), dx = x_i - c_j), up to K in index
// order; the row's rest repeats its first entry, or is -1 for an empty ball; count[j]
// is the number of points inside. Brute force in index order.
int32_t oracle_ball_query(const float* xyz, int64_t N, const float* ctr, int64_t Q, float radius,
                          int32_t K, int32_t* idx, int32_t* count) {
  if (!xyz || !ctr || !idx || N < 1 || Q < 1 || K < 1 || !(radius > 0.0f)) return 1;
  const float r2 = radius * radius;
  for (int64_t j = 0; j < Q; ++j) {
    int32_t* row = idx + j * K;
    int32_t n = 0;
    int64_t total = 0;
    for (int64_t i = 0; i < N; ++i) {
      const float dx = xyz[3 * i] - ctr[3 * j];
      const float dy = xyz[3 * i + 1] - ctr[3 * j + 1];
      const float dz = xyz[3 * i + 2] - ctr[3 * j + 2];
      const float d2 = dx * dx + dy * dy + dz * dz;
      if (!(d2 < r2)) continue;
      ++total;
      if (n < K) row[n++] = static_cast<int32_t>(i);
    }
    for (int32_t t = n; t < K; ++t) row[t] = n > 0 ? row[0] : -1;
    if (count) count[j] = static_cast<int32_t>(total);
  }
  return 0;
}

// Covering radius: max over all points of the distance to the nearest point of idx
// (brute force: O(N m)).
double oracle_covering_radius(const float* xyz, int64_t N, const int32_t* idx, int64_t m) {
  if (!xyz || !idx || N < 1 || m < 1) return -1.0;
  std::vector<float> smp(static_cast<size_t>(m) * 3);
  for (int64_t j = 0; j < m; ++j)
    for (int a = 0; a < 3; ++a) smp[3 * j + a] = xyz[3 * static_cast<int64_t>(idx[j]) + a];
  std::vector<double> d(static_cast<size_t>(N));
  nn_d2(smp.data(), m, xyz, N, 0, d.data());
  double worst = 0.0;
  for (double v : d) worst = std::max(worst, v);
  return std::sqrt(worst);
}

}  // extern "C"
