// HAVSampler CPU oracle — TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded implementation of the hierarchical adaptive
// voxel-guided sampler, written from the paper (arXiv 2305.14306, Sec. 3). It is
// the definition the GPU library is checked against, bit for bit. Only the test
// suite, the smoke check and the bench's CPU-baseline leg may load it; the product
// path never does. It shares no code, header or table with the GPU library.
//
// Built with -O2 -ffp-contract=off -fno-fast-math on x86-64 (SSE arithmetic), so
// every float expression below is one correctly rounded binary32 operation.
//
// What is computed (one call = one stage):
//   1. Stage frame: per-axis min/max of the cloud; the grid origin is the min
//      corner; E = max_a (extent_a / aspect_a); hi0 = smallest power of two >= E.
//   2. Layer sizes (Sec. 3.4, Eq. 3): m_l = ratio * m_{l-1}, sum m_l = M; floor for
//      l < k, remainder to the last layer.
//   3. Per layer, on the not-yet-sampled points R:
//      a. voxel coordinates (Sec. 3.2, Eq. 2) g = floor(r * (1/v)), r = p - origin;
//      b. the voxel counter Cnt(R, v) = number of distinct voxel coordinates
//         (the hashed sparse voxelization of Sec. 3.2, and Sec. 3.3);
//      c. adaptive voxel search (Sec. 3.3): bisection on the voxel scale s until the
//         count is in [m, (1+sigma) m] or t_max evaluations have been made;
//      d. centre-closest representative per occupied voxel (the centre-closest
//         point sampling of Sec. 3.2), ties to the lowest index;
//      e. exactly m picks: trim by a fixed hash priority of the voxel coordinate
//         when there are too many representatives, pad with the lowest unsampled
//         indices when there are too few (Sec. 3.3 says the surplus or deficit has to
//         be made up or dropped without fixing how);
//      f. mask the picks out of R (Sec. 3.4).
//   4. Output: the picks of all layers in ascending index order (Sec. 3.4 gathers the
//      layer subsets; the order is this implementation's choice).
//
// Parity status of each function is stated beside it; every function here is pinned
// by the CPU test suite (closed forms on lattices, brute force on tiny clouds, a
// sort-and-unique second route, the covering bound and published SplitMix64 values).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

namespace {

// Status codes of the oracle (same meanings as the library's, defined separately).
enum : int32_t {
  OR_OK = 0,
  OR_INVALID_ARG = 1,
  OR_UNSUPPORTED = 4,
  OR_NONFINITE = 5,
};

constexpr uint32_t OR_FIXED_VOXEL = 1u;
constexpr int kMaxLayers = 8;

}  // namespace

extern "C" {

// Parameters, laid out for ctypes. Defaults: 2 layers, ratio 4, sigma 0.05,
// t_max 20 (the implementation details of Sec. 4.1; ratio from Sec. 3.4).
typedef struct {
  int32_t layers;
  int32_t layer_ratio;
  int32_t t_max;
  int32_t flags;
  double sigma;
  float aspect[3];
  float fixed_voxel[3];
  int32_t select;   // 0: centre-closest (Sec. 3.2); 1: random member (Table 6, RA);
                    // 2: voxel centre, 3: voxel mean (CE, ME; points, not indices)
  uint32_t seed;    // random member: generator seed
} OracleParams;

typedef struct {
  int32_t status;
  int32_t layers;  // number of layers that ran (m_l > 0)
  float hi0;
  float mn[3];
  float mx[3];
  int32_t m[kMaxLayers];
  float s[kMaxLayers];  // chosen voxel scale per layer (0 with a fixed voxel)
  int32_t evals[kMaxLayers];
  int32_t count[kMaxLayers];  // occupied voxels at the chosen size
  int32_t accepted[kMaxLayers];
  int32_t trimmed[kMaxLayers];
  int32_t padded[kMaxLayers];
} OracleInfo;

}  // extern "C"

namespace {

uint32_t float_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}

// a < b in IEEE total order, for finite values (-0 sorts below +0).
bool total_less(float a, float b) {
  if (a < b) return true;
  if (a > b) return false;
  return std::signbit(a) && !std::signbit(b);
}

// Voxel coordinate of one point at voxel size v (Sec. 3.2, Eq. 2), relative to the
// stage origin mn: r = p - mn, g = floor(r * fl(1/v)). Returns the three integer
// coordinates packed 21 bits each (x low). Coordinates are < 2^21 on every size the
// search or a checked fixed voxel can produce.
uint64_t voxel_key(const float* p, const float* mn, const float* inv, int32_t* g_out,
                   float* r_out) {
  uint64_t key = 0;
  for (int a = 0; a < 3; ++a) {
    const float r = p[a] - mn[a];
    const float q = r * inv[a];
    const int32_t g = static_cast<int32_t>(std::floor(q));
    if (g_out) g_out[a] = g;
    if (r_out) r_out[a] = r;
    key |= static_cast<uint64_t>(static_cast<uint32_t>(g)) << (21 * a);
  }
  return key;
}

// Squared distance from a point to the centre of its voxel, v * (g + 0.5) in the
// stage frame (Sec. 3.2, d_i). Fixed binary32 order: ((dx*dx + dy*dy) + dz*dz).
// The square root is not taken: it could merge distinct squared distances.
float centre_dist2(const float* r, const int32_t* g, const float* v) {
  float d[3];
  for (int a = 0; a < 3; ++a) {
    const float centre = v[a] * (static_cast<float>(g[a]) + 0.5f);
    d[a] = r[a] - centre;
  }
  const float xx = d[0] * d[0];
  const float yy = d[1] * d[1];
  const float zz = d[2] * d[2];
  return (xx + yy) + zz;
}

// Trim priority of a voxel: the SplitMix64 output function (Steele, Lea and Flood,
// OOPSLA 2014) applied to the packed coordinate. A bijection on 64-bit words, so
// distinct voxels never tie.
uint64_t voxel_priority(uint64_t key) {
  uint64_t z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Voxel size and its correctly rounded reciprocal for scale s: v = s * aspect.
void voxel_of_scale(float s, const float* aspect, float* v, float* inv) {
  for (int a = 0; a < 3; ++a) {
    v[a] = s * aspect[a];
    inv[a] = 1.0f / v[a];
  }
}

// Point visits of the calls made on this thread: every Cnt evaluation and every
// selection pass visits each point of R once (the O(N)-per-evaluation claim of Sec. 4.2
// and Table 1; the tests compare it with sum over layers of (evals + 1) * |R|).
thread_local int64_t g_visits = 0;

// Cnt(R, v): number of non-empty voxels among the points still in R (Sec. 3.3).
int64_t count_voxels(const float* xyz, const std::vector<int64_t>& R, const float* mn,
                     const float* inv) {
  g_visits += static_cast<int64_t>(R.size());
  std::unordered_set<uint64_t> seen;
  seen.reserve(R.size() * 2 + 16);
  for (int64_t i : R) seen.insert(voxel_key(xyz + 3 * i, mn, inv, nullptr, nullptr));
  return static_cast<int64_t>(seen.size());
}

// Smallest power of two >= E (E > 0, normal), by exponent arithmetic.
float pow2_ceil(float E) {
  int e = 0;
  const float f = std::frexp(E, &e);  // E = f * 2^e, f in [0.5, 1)
  return (f == 0.5f) ? E : std::ldexp(1.0f, e);
}

bool params_valid(const OracleParams* p) {
  if (!p) return false;
  if (p->layers < 1 || p->layers > kMaxLayers) return false;
  if (p->layer_ratio < 2 || p->layer_ratio > 16) return false;
  if (p->t_max < 1 || p->t_max > 20) return false;
  if (!std::isfinite(p->sigma) || p->sigma < 0.0 || p->sigma > 16.0) return false;
  for (int a = 0; a < 3; ++a) {
    const float as = p->aspect[a];
    if (!std::isfinite(as) || as < std::ldexp(1.0f, -16) || as > std::ldexp(1.0f, 16))
      return false;
    if (p->flags & OR_FIXED_VOXEL) {
      const float fv = p->fixed_voxel[a];
      if (!std::isfinite(fv) || fv < std::ldexp(1.0f, -100) || fv > std::ldexp(1.0f, 100))
        return false;
    }
  }
  if (p->flags & ~OR_FIXED_VOXEL) return false;
  if (p->select < 0 || p->select > 3) return false;
  return true;
}

// Layer budgets m_l (Sec. 3.4): m_l = ratio * m_{l-1} and sum m_l = M, i.e.
// m_l = M * r^(l-1) * (r-1) / (r^k - 1), floored for l < k, remainder to layer k.
void layer_budgets(int64_t M, int k, int r, int64_t* m) {
  uint64_t rk = 1;
  for (int l = 0; l < k; ++l) rk *= static_cast<uint64_t>(r);
  uint64_t rl = 1;  // r^(l-1)
  int64_t used = 0;
  for (int l = 0; l < k - 1; ++l) {
    m[l] = static_cast<int64_t>(static_cast<uint64_t>(M) * rl * static_cast<uint64_t>(r - 1) /
                                (rk - 1));
    used += m[l];
    rl *= static_cast<uint64_t>(r);
  }
  m[k - 1] = M - used;
}

// One stage: sample exactly M of the N points. idx gets M ascending indices. pt_out
// (optional, [N][3]) gets, for every voxel representative, the point that stands for
// its voxel: the representative itself, or with select 2 / 3 the voxel's centre /
// the mean of its points; a padded point stands for itself.
int32_t sample_stage(const float* xyz, int64_t N, int64_t M, const OracleParams* p,
                     int32_t* idx, OracleInfo* info, uint8_t* tag_out, float* pt_out = nullptr) {
  OracleInfo local{};
  OracleInfo& inf = info ? *info : local;
  std::memset(&inf, 0, sizeof(inf));
  if (!xyz || !idx || N < 1 || M < 1 || M > N || N >= (int64_t(1) << 31) || !params_valid(p)) {
    inf.status = OR_INVALID_ARG;
    return inf.status;
  }
  // Stage frame: bounding box and the finiteness check.
  float mn[3], mx[3];
  for (int a = 0; a < 3; ++a) mn[a] = mx[a] = xyz[a];
  for (int64_t i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) {
      const float c = xyz[3 * i + a];
      if (!std::isfinite(c)) {
        inf.status = OR_NONFINITE;
        return inf.status;
      }
      if (total_less(c, mn[a])) mn[a] = c;
      if (total_less(mx[a], c)) mx[a] = c;
    }
  }
  std::memcpy(inf.mn, mn, sizeof(mn));
  std::memcpy(inf.mx, mx, sizeof(mx));
  if (M == N) {  // every point is kept
    for (int64_t i = 0; i < N; ++i) idx[i] = static_cast<int32_t>(i);
    if (pt_out) std::memcpy(pt_out, xyz, static_cast<size_t>(N) * 3 * sizeof(float));
    if (tag_out) std::memset(tag_out, 1, static_cast<size_t>(N));
    return OR_OK;
  }
  float E = 0.0f;
  for (int a = 0; a < 3; ++a) {
    const float ext = (mx[a] - mn[a]) / p->aspect[a];
    if (!(ext <= E)) E = ext;  // also takes a NaN/inf so the check below sees it
  }
  if (!(E <= std::ldexp(1.0f, 100))) {
    inf.status = OR_UNSUPPORTED;
    return inf.status;
  }
  const float hi0 = pow2_ceil(std::max(E, std::ldexp(1.0f, -64)));
  inf.hi0 = hi0;

  const bool fixed = (p->flags & OR_FIXED_VOXEL) != 0;
  float fixed_v[3], fixed_inv[3];
  if (fixed) {
    for (int a = 0; a < 3; ++a) {
      fixed_v[a] = p->fixed_voxel[a];
      fixed_inv[a] = 1.0f / fixed_v[a];
      // the largest coordinate along this axis must fit the 21-bit field
      const float q = (mx[a] - mn[a]) * fixed_inv[a];
      if (!(q < 2097152.0f)) {
        inf.status = OR_UNSUPPORTED;
        return inf.status;
      }
    }
  }

  // Voxel mean (select 3) in fixed point, so that the sum does not depend on the
  // order of the points: along axis a, q = floor(r_a * 2^32 / H_a) with H_a the
  // smallest power of two >= the extent (r_a <= H_a, so q <= 2^32 and a sum over up
  // to 2^30 points fits 64 bits); mean = mn + (sum_q / n) * H_a * 2^-32 in double,
  // rounded to float once.
  float qscale[3];
  double qback[3];
  for (int a = 0; a < 3; ++a) {
    const float H = pow2_ceil(std::max(mx[a] - mn[a], std::ldexp(1.0f, -64)));
    qscale[a] = 4294967296.0f / H;
    qback[a] = static_cast<double>(H) / 4294967296.0;
  }

  int64_t budget[kMaxLayers];
  layer_budgets(M, p->layers, p->layer_ratio, budget);

  std::vector<uint8_t> taken(static_cast<size_t>(N), 0);
  int out_layer = 0;
  for (int l = 0; l < p->layers; ++l) {
    const int64_t m = budget[l];
    if (m == 0) continue;
    const int L = out_layer++;
    inf.m[L] = static_cast<int32_t>(m);
    std::vector<int64_t> R;
    R.reserve(static_cast<size_t>(N));
    for (int64_t i = 0; i < N; ++i)
      if (!taken[i]) R.push_back(i);

    float v[3], inv[3];
    int64_t c_final = 0;
    if (fixed) {
      std::memcpy(v, fixed_v, sizeof(v));
      std::memcpy(inv, fixed_inv, sizeof(inv));
      inf.s[L] = 0.0f;
      c_final = count_voxels(xyz, R, mn, inv);
    } else {
      // Adaptive voxel search (Sec. 3.3): bisection on s in (0, hi0].
      const int64_t upper = static_cast<int64_t>(std::floor(static_cast<double>(m) * (1.0 + p->sigma)));
      float lo = 0.0f, hi = hi0;
      int64_t c_lo = 0, c_hi = 0;
      bool accepted = false;
      float s_final = 0.0f;
      int evals = 0;
      for (int t = 0; t < p->t_max; ++t) {
        const float s = (lo + hi) * 0.5f;  // exact: lo, hi are dyadic multiples of hi0
        float vv[3], ii[3];
        voxel_of_scale(s, p->aspect, vv, ii);
        const int64_t c = count_voxels(xyz, R, mn, ii);
        ++evals;
        if (c >= m && c <= upper) {
          accepted = true;
          s_final = s;
          c_final = c;
          break;
        }
        if (c < m) {
          hi = s;
          c_hi = c;
        } else {
          lo = s;
          c_lo = c;
        }
      }
      if (!accepted) {
        // No size in the tolerance window within t_max evaluations: take the
        // finest size whose count exceeded the window (then trim) if there was
        // one, else the smallest size evaluated (then pad).
        if (lo > 0.0f) {
          s_final = lo;
          c_final = c_lo;
        } else {
          s_final = hi;
          c_final = c_hi;
        }
      }
      voxel_of_scale(s_final, p->aspect, v, inv);
      inf.s[L] = s_final;
      inf.evals[L] = evals;
      inf.accepted[L] = accepted ? 1 : 0;
    }

    // Centre-closest representative per voxel, ties to the lowest index. The random
    // variant (the "RA" selection of Table 6) ranks a voxel's points instead by the top
    // 32 bits of output i+1 of a SplitMix64 generator seeded with p->seed, ties again
    // to the lowest index.
    std::unordered_map<uint64_t, std::pair<uint32_t, int64_t>> best;
    best.reserve(R.size() * 2 + 16);
    g_visits += static_cast<int64_t>(R.size());
    for (int64_t i : R) {
      int32_t g[3];
      float r[3];
      const uint64_t key = voxel_key(xyz + 3 * i, mn, inv, g, r);
      const uint32_t d2 =
          p->select == 1
              ? static_cast<uint32_t>(voxel_priority(static_cast<uint64_t>(p->seed) +
                                                     static_cast<uint64_t>(i) * 0x9E3779B97F4A7C15ull) >> 32)
              : float_bits(centre_dist2(r, g, v));  // d2 >= 0: bits order = value order
      auto it = best.find(key);
      if (it == best.end()) {
        best.emplace(key, std::make_pair(d2, i));
      } else if (d2 < it->second.first || (d2 == it->second.first && i < it->second.second)) {
        it->second = std::make_pair(d2, i);
      }
    }
    const int64_t c = static_cast<int64_t>(best.size());
    if (pt_out) {
      // what stands for each voxel (only the kept voxels' entries are read)
      std::unordered_map<uint64_t, std::array<uint64_t, 4>> sums;
      if (p->select == 3) {
        for (int64_t i : R) {
          int32_t g[3];
          float r[3];
          const uint64_t key = voxel_key(xyz + 3 * i, mn, inv, g, r);
          auto& acc = sums[key];
          for (int a = 0; a < 3; ++a) acc[a] += static_cast<uint64_t>(r[a] * qscale[a]);
          acc[3] += 1;
        }
      }
      for (const auto& kv : best) {
        const int64_t i = kv.second.second;
        float* o = pt_out + 3 * i;
        if (p->select == 2) {
          for (int a = 0; a < 3; ++a) {
            const float ga = static_cast<float>((kv.first >> (21 * a)) & 0x1FFFFF);
            o[a] = mn[a] + v[a] * (ga + 0.5f);
          }
        } else if (p->select == 3) {
          const auto& acc = sums[kv.first];
          for (int a = 0; a < 3; ++a) {
            const double mean = static_cast<double>(acc[a]) / static_cast<double>(acc[3]);
            o[a] = static_cast<float>(static_cast<double>(mn[a]) + mean * qback[a]);
          }
        } else {
          for (int a = 0; a < 3; ++a) o[a] = xyz[3 * i + a];
        }
      }
    }
    if (c != c_final) {  // the search and the selection must see the same voxels
      inf.status = OR_INVALID_ARG;
      return inf.status;
    }
    inf.count[L] = static_cast<int32_t>(c);

    std::vector<int64_t> picks;
    if (c > m) {
      // keep the m voxels of smallest priority
      std::vector<std::pair<uint64_t, int64_t>> pr;
      pr.reserve(best.size());
      for (const auto& kv : best) pr.emplace_back(voxel_priority(kv.first), kv.second.second);
      std::sort(pr.begin(), pr.end());
      for (int64_t j = 0; j < m; ++j) picks.push_back(pr[j].second);
      inf.trimmed[L] = static_cast<int32_t>(c - m);
    } else {
      for (const auto& kv : best) picks.push_back(kv.second.second);
    }
    for (int64_t i : picks) taken[i] = static_cast<uint8_t>(L + 1);
    if (c < m) {
      // pad with the lowest-index points of R that were not picked
      int64_t need = m - c;
      for (int64_t i : R) {
        if (need == 0) break;
        if (!taken[i]) {
          taken[i] = static_cast<uint8_t>(L + 1);
          if (pt_out)
            for (int a = 0; a < 3; ++a) pt_out[3 * i + a] = xyz[3 * i + a];
          --need;
        }
      }
      inf.padded[L] = static_cast<int32_t>(m - c);
    }
  }
  inf.layers = out_layer;
  if (tag_out) std::memcpy(tag_out, taken.data(), static_cast<size_t>(N));
  int64_t w = 0;
  for (int64_t i = 0; i < N; ++i)
    if (taken[i]) idx[w++] = static_cast<int32_t>(i);
  if (w != M) {
    inf.status = OR_INVALID_ARG;
    return inf.status;
  }
  return OR_OK;
}

}  // namespace

extern "C" {

OracleParams oracle_params_default(void) {
  OracleParams p{};
  p.layers = 2;
  p.layer_ratio = 4;
  p.t_max = 20;
  p.flags = 0;
  p.sigma = 0.05;
  for (int a = 0; a < 3; ++a) {
    p.aspect[a] = 1.0f;
    p.fixed_voxel[a] = 1.0f;
  }
  p.select = 0;
  p.seed = 0;
  return p;
}

int32_t oracle_sample(const float* xyz, int64_t N, int64_t M, const OracleParams* p,
                      int32_t* idx, OracleInfo* info) {
  return sample_stage(xyz, N, M, p, idx, info, nullptr);
}

// Same as oracle_sample, and tag[i] = layer number (1-based) that picked point i,
// 0 when not picked.
int32_t oracle_sample_tags(const float* xyz, int64_t N, int64_t M, const OracleParams* p,
                           int32_t* idx, OracleInfo* info, uint8_t* tag) {
  return sample_stage(xyz, N, M, p, idx, info, tag);
}

// The stage's picks as points: xyz_out[j] stands for idx[j] (the voxel centre or mean
// with select 2 / 3, else the point itself).
int32_t oracle_sample_points(const float* xyz, int64_t N, int64_t M, const OracleParams* p,
                             int32_t* idx, float* xyz_out, OracleInfo* info) {
  if (!xyz_out || N < 1) return OR_INVALID_ARG;
  std::vector<float> pt(static_cast<size_t>(N) * 3, 0.0f);
  const int32_t st = sample_stage(xyz, N, M, p, idx, info, nullptr, pt.data());
  if (st != OR_OK) return st;
  for (int64_t j = 0; j < M; ++j)
    for (int a = 0; a < 3; ++a) xyz_out[3 * j + a] = pt[3 * static_cast<int64_t>(idx[j]) + a];
  return OR_OK;
}

// Chained stages: stage j samples Ms[j] points of the cloud stage j-1 produced
// (the gathered points, in ascending original-index order). idx_concat holds each
// stage's picks as original indices, stage after stage (sum of Ms entries).
int32_t oracle_chain(const float* xyz, int64_t N, const int64_t* Ms, int32_t n_stages,
                     const OracleParams* p, int32_t* idx_concat, OracleInfo* infos) {
  if (!xyz || !Ms || !idx_concat || n_stages < 1) return OR_INVALID_ARG;
  std::vector<float> cur(xyz, xyz + 3 * N);
  std::vector<int32_t> to_orig(static_cast<size_t>(N));
  for (int64_t i = 0; i < N; ++i) to_orig[i] = static_cast<int32_t>(i);
  int64_t n = N;
  int64_t off = 0;
  for (int32_t j = 0; j < n_stages; ++j) {
    const int64_t m = Ms[j];
    std::vector<int32_t> local(static_cast<size_t>(std::max<int64_t>(m, 1)));
    const int32_t st = sample_stage(cur.data(), n, m, p, local.data(), infos ? &infos[j] : nullptr, nullptr);
    if (st != OR_OK) return st;
    std::vector<float> next(static_cast<size_t>(3 * m));
    std::vector<int32_t> next_map(static_cast<size_t>(m));
    for (int64_t q = 0; q < m; ++q) {
      const int32_t li = local[q];
      for (int a = 0; a < 3; ++a) next[3 * q + a] = cur[3 * static_cast<size_t>(li) + a];
      next_map[q] = to_orig[li];
      idx_concat[off + q] = to_orig[li];
    }
    off += m;
    cur.swap(next);
    to_orig.swap(next_map);
    n = m;
  }
  return OR_OK;
}

// Exposed pieces, so the tests can pin them one by one.

// Cnt at voxel size v with origin mn over the points whose mask byte is 0
// (mask may be null: all points).
int64_t oracle_count(const float* xyz, int64_t N, const float* mn, const float* v,
                     const uint8_t* mask) {
  float inv[3];
  for (int a = 0; a < 3; ++a) inv[a] = 1.0f / v[a];
  std::vector<int64_t> R;
  for (int64_t i = 0; i < N; ++i)
    if (!mask || !mask[i]) R.push_back(i);
  return count_voxels(xyz, R, mn, inv);
}

// Voxel coordinates and squared centre distance of every point at size v.
void oracle_keys(const float* xyz, int64_t N, const float* mn, const float* v, int32_t* g_out,
                 uint64_t* key_out, float* d2_out) {
  float inv[3];
  for (int a = 0; a < 3; ++a) inv[a] = 1.0f / v[a];
  for (int64_t i = 0; i < N; ++i) {
    int32_t g[3];
    float r[3];
    const uint64_t key = voxel_key(xyz + 3 * i, mn, inv, g, r);
    if (g_out) std::memcpy(g_out + 3 * i, g, sizeof(g));
    if (key_out) key_out[i] = key;
    if (d2_out) d2_out[i] = centre_dist2(r, g, v);
  }
}

uint64_t oracle_priority(uint64_t key) { return voxel_priority(key); }

// Point visits made on the calling thread since the last call of this function.
int64_t oracle_take_visits(void) {
  const int64_t v = g_visits;
  g_visits = 0;
  return v;
}

float oracle_pow2_ceil(float E) { return pow2_ceil(std::max(E, std::ldexp(1.0f, -64))); }

void oracle_layer_budgets(int64_t M, int32_t k, int32_t r, int64_t* m) {
  layer_budgets(M, k, r, m);
}

}  // extern "C"
