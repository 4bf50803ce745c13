// HAVSampler for MI355X (gfx950): kernels and the C ABI of include/hav.h.
//
// One stage samples exactly M of N points (arXiv 2305.14306, Sec. 3). Pipeline, all
// on one stream, every decision taken on the device (no host round trip):
//
//   k_bbox         per-block min/max of the cloud and the non-finite check
//   k_bin_count    every block reduces the partial boxes (same bits everywhere),
//                  derives the stage frame (origin = min corner, search bracket hi0)
//                  and a 12-bit Morton cell per point; per-block cell histograms
//   k_bin_scan     exclusive scan of the (cell, block) histogram
//   k_bin_scatter  counting sort by cell into 16-byte records (r = p - origin, which
//                  is exactly what Eq. 2 consumes, and the original index), so each
//                  2048-point tile is spatially compact; one more block starts layer 1
//   per layer (Sec. 3.4, Eq. 3):
//     k_search     adaptive voxel search (Sec. 3.3), one launch: a queue of (pass,
//                  tile) tickets. A pass evaluates the voxel counter Cnt at up to
//                  `depth` sizes along the bisection path a count model predicts;
//                  steps whose count is provably below m (more voxels than grid cells
//                  is impossible) are taken without evaluation. Decisions, and so the
//                  chosen size, are exactly those of one bisection step at a time. A
//                  tile dedups its voxels in LDS as 4x4x4 bricks with 64-bit occupancy
//                  masks, then makes one find-or-claim and at most one atomicOr per
//                  distinct brick in a global table; the newly set bits are newly seen
//                  voxels. The block that completes a pass runs the bisection step and
//                  publishes the next pass.
//     k_select     centre-closest point per occupied voxel at the chosen size
//                  (Sec. 3.2): LDS min of (bits(d^2) << 32 | index), then at most one
//                  global atomicMin per tile-distinct voxel; ties go to the lowest
//                  index. Also counts voxel priorities below / inside a window around
//                  the expected trim threshold
//     k_trim_hist  (fixed voxel size only) radix rounds of the trim threshold
//     k_mark       keep the voxels below the trim bucket, queue the bucket; the last
//                  block ranks the bucket and marks up to the exact threshold; when a
//                  layer found fewer voxels than m it pads the lowest-index unsampled
//                  points (a pass in index order that ends once enough are marked), and
//                  it starts the next layer
//   k_out          ascending output indices (one pass, tiles chained in dispatch order;
//                  the last layer's pad folded in)
//
// Table hygiene: a workspace is initialised once (hav_workspace_init). Each kernel
// that fills a table records the slots it claimed and a later kernel of the same call
// empties exactly those, so every call leaves the workspace as it found it and no call
// clears whole tables.
//
// Cross-block reductions: blocks publish partial results with atomic RMWs into
// per-group accumulators (<= ~32 atomics per address), wait for them to complete
// (s_waitcnt 0), then arrive on two-level counters; the last block reads the partials
// back with RMWs. Data written with plain stores is only read by later kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>
#include <cmath>
#include <cstring>

#include "../../include/hav.h"
#include "hav_device.hpp"

namespace hav {

// Polls before a tag scan's bounded wait gives up, and before a voxel-search wait for a
// pass's publication gives up (per device; test hooks lower them).
constexpr uint32_t kScanSpinDefault = 1u << 22;
__device__ uint32_t g_scan_spin_limit = kScanSpinDefault;
constexpr uint32_t kSearchSpinDefault = 1u << 22;
__device__ uint32_t g_search_spin_limit = kSearchSpinDefault;

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 2048;                     // points per search/select tile
constexpr int kPerThread = kTile / kThreads;    // 8
constexpr int kLdsCap = 4096;                   // select: LDS voxel map entries (2x tile)
constexpr int kBrickCap = 1024;                 // search: LDS hash slots per candidate
constexpr int kCandWords = 2 * kBrickCap;        // search: LDS words per candidate (hash values
                                                 // then keys, or one box of up to this many bricks)
constexpr int kMaxCand = 7;                     // candidate scales per search pass
constexpr int kSplitTickets = 512;              // search tickets per pass up to which a tile's
                                                // candidates get tickets of their own
constexpr int kMaxDepth = kMaxCand;
constexpr int kDefaultDepth = 4;
constexpr int kGroups = 16;
constexpr int kStride = 32;                     // uint32 spacing of hot counters (128 B)
constexpr int kBinBits = 12;
constexpr int kBins = 1 << kBinBits;
constexpr int kMaxBinBlocks = 512;
constexpr int kBinChunk = 16;                   // bins per block of the histogram scan
constexpr int kBinChunks = kBins / kBinChunk;
constexpr int kMaxBBoxBlocks = 1024;
constexpr int kScanTile = 4096;                 // tag scans: 16 per thread
constexpr int kScanPer = kScanTile / kThreads;
constexpr int kSelDense = 4;                    // voxel value slots per brick-table slot (at least)
constexpr uint64_t kMagic = 0x4841565F57533031ull;
constexpr int kMaxDevices = 64;
constexpr int kTieLds = 1024;                   // trim bucket staged in LDS up to this size
constexpr float kWinSigma = 6.0f;                // default trim window half-width (std devs)
constexpr int kTieRank = 128;                   // bucket members ranked directly up to this many
constexpr int kTrimBits = 8;                    // priority digit of one trim round
constexpr int kTrimBins = 1 << kTrimBits;
constexpr int kWinBins = 1024;                  // trim window: bins of its priority histogram
constexpr int kHotCap = 4096;                   // brick grids this small use replicas
constexpr int kReps = 16;                       // replicas of a hot brick table
constexpr int kClaimCap = 2 * kTile;            // claims per tile and candidate
constexpr int kClrReg = 4;                      // search: claims a thread clears from registers
constexpr int64_t kMaxPoints = (int64_t(1) << 30) - 1;  // table slots stay below 2^31

// ----------------------------------------------------------------------------- state

struct Frame {
  int32_t status;
  int32_t bbits[3];
  float mn[3], mx[3];
  float hi0;
  float bscale[3];
  // box-counting prior of the search's count model: Cnt(s) ~ prior_c (prior_s / s)^prior_d
  float prior_s, prior_c, prior_d;
  int32_t prior_ok;
};

struct Ctrl {
  int32_t layer;
  uint32_t m, upper;
  int32_t evals, done, accepted;
  float s_final;
  float v_final[3], inv_final[3];
  int32_t set;          // table set the next search pass fills
  int32_t pend_set, pend_nc;  // table set and candidates whose claims are still to clear
  uint32_t pend_hashed;       // bit k: candidate k of that pass used a hashed table
  int32_t sel_dense;              // 1: voxel grid at the chosen size fits, index directly
  uint32_t sel_nv[2];             // voxel grid x, y extents (dense mode)
  uint32_t ncand;       // occupied voxels at the chosen size
  int32_t trim;
  uint32_t need;        // pad count
  uint32_t rank;        // rank sought inside the trim bucket
  uint64_t prefix;      // radix rounds: decided top bits of the threshold
  int32_t rounds_done;
  // trim bucket: 0 the radix prefix, 1 the priority window [blo, bhi], 2 every voxel;
  // 3: no bucket, every voxel of priority at most bhi stays (the rank is the largest of the
  // window bin that holds it)
  int32_t trim_mode;
  uint32_t c_final;     // voxels the search counted at s_final (0: no search)
  int32_t win;          // a window was set for the selection kernel to test
  int32_t wshift;       // window priority bin: (p - blo) >> wshift
  uint64_t blo, bhi;
};

// State of the voxel search between passes (Sec. 3.3): the bracket, the outcome so
// far and the next pass's candidate scales. Published as 32-bit words.
struct SState {
  float lo, hi;
  uint32_t c_hi;  // count at hi (0: hi is the initial bracket, never evaluated)
  uint32_t c_lo;  // count at lo (0: lo is 0, never evaluated)
  uint32_t c_final;  // count at s_final once done
  int32_t pdir[kMaxCand];  // predicted step after candidate k: 0 down (hi = s), 1 up (lo = s)
  int32_t evals, done, accepted;
  int32_t nc, set, prev_set, prev_nc;
  uint32_t prev_hashed;  // bit k: candidate k of the previous pass used a hashed table
  float s_final;
  float cand_s[kMaxCand];
  float cand_inv[kMaxCand][3];
  int32_t cand_dense[kMaxCand], cand_hot[kMaxCand];
  uint32_t cand_nb[kMaxCand][2];
};

struct Plan {  // per-call constants (kernel argument)
  int32_t nlayers;
  int32_t t_max;
  int32_t depth;
  int32_t fixed;
  uint32_t m[HAV_MAX_LAYERS];
  uint32_t upper[HAV_MAX_LAYERS];
  float aspect[3];
  float fixed_v[3];
  uint64_t magic;
  uint32_t cap;       // brick table slots: dense brick grids up to this size
  uint32_t sel_cap;   // voxel value slots: dense voxel grids up to this size
  float spec_mult;    // speculation budget of the search, in multiples of the window top
  float win_sigma;    // trim window half-width in standard deviations (<= 0: none)
  int32_t select;     // HAV_SELECT_CENTRE_CLOSEST or HAV_SELECT_RANDOM
  uint32_t seed;      // random member: generator seed
  int32_t identity;   // M == N: output 0..N-1, nothing else runs
  int32_t rounds[HAV_MAX_LAYERS];  // radix rounds of each layer's trim (fixed size only)
};

constexpr int kPubWords = static_cast<int>(sizeof(SState) / 4);
static_assert(sizeof(SState) % 4 == 0 && kPubWords <= kThreads, "search state words");

struct alignas(256) Header {
  uint64_t magic;
  int64_t binned_n;     // points of the stage whose sorted cloud the workspace holds (0: none)
  uint64_t pad0[14];
  uint32_t ball_next;   // grouping: the next work item, and the number of items
  uint32_t ball_items;
  uint32_t pad1[30];
  alignas(256) Frame frame;
  alignas(256) Ctrl ctrl;
  alignas(256) hav_info_t info;
  alignas(256) uint32_t sync_top[kStride];
  uint32_t sync_grp[kGroups][kStride];
  uint32_t acc[kMaxCand][kGroups][kStride];
  uint32_t hist[kGroups][kTrimBins];  // trim: priority digit histograms
  uint32_t whist[kWinBins];       // trim window: voxels per priority bin
  uint32_t tie_cur[kGroups][kStride];
  uint32_t ord[kStride];          // dispatch-order block ids of the tag scans
  uint32_t scan_bad[kStride];     // a tag-scan wait gave up
  // voxel search: double-buffered per-pass counts, tile tickets, completed tiles,
  // the pass whose candidates are published, finish and failure flags
  uint32_t sacc[2][kMaxCand][kGroups][kStride];
  uint32_t sq_ticket[kStride];
  uint32_t sq_dgrp[kGroups][kStride];
  uint32_t sq_done[kStride];
  uint32_t sq_gen[kStride];
  uint32_t sq_fin[kStride];
  uint32_t sq_err[kStride];
  alignas(256) uint32_t pub[kPubWords];
  uint32_t pub_first[HAV_MAX_LAYERS][kPubWords];  // each layer's first pass, planned at the start
};

// Device view of the workspace for one stage.
struct Ws {
  Header* h;
  float4* pts;                   // sorted: (r_x, r_y, r_z, original index as bits)
  int32_t* invp;                 // original index -> sorted position
  uint8_t* tag_s;                // sorted order: layer that picked the point (0 = none)
  uint8_t* tag_o;                // original order
  uint32_t* part;                // k_bbox partials [nbbox][8]
  uint32_t* bh;                  // cell histogram [nbb][kBins], then offsets within a cell
  uint32_t* binpre;              // [kBins] offset of a cell inside its chunk of cells
  uint32_t* bsum;                // [kBinChunks] chunk sums, then chunk offsets
  unsigned long long* ckeys;     // brick tables [2][ncmax][cap_ws]
  unsigned long long* cmasks;
  int32_t* ccl;                  // claims [2][ncmax][ntile_ws][kClaimCap]
  unsigned long long* hrep;      // hot table replicas [2][ncmax][kReps][kHotCap]
  int32_t* ccn;                  // claim counts [2][ncmax][ntile_ws]
  unsigned long long* skeys;     // voxel table [cap_ws]
  unsigned long long* svals;
  int32_t* scl;                  // claims [ntile_ws][kTile]
  int32_t* scn;                  // [ntile_ws]
  uint64_t* tie_p;               // [kGroups][tie_seg]
  int64_t* tie_o;                // (sorted slot << 32) | original index
  uint32_t* tcnt;                // scan tile counts [nscan_ws]
  float* pt_out;                 // points modes: what stands for each kept point [n_ws][3]
  unsigned long long* msum;      // mean mode: per voxel slot fixed-point sums [slots][3]
  uint32_t* mcnt;                // mean mode: per voxel slot point counts [slots]
  float* xyz_out;                // points modes: output [M][3] (null: indices only)
  int32_t pmode;                 // 0 indices, 1 voxel centres, 2 voxel means
  int64_t n;
  int64_t npad;                  // slots of the sorted arrays: ntile * kTile
  int32_t ntile, nscan, nbb, nbbox;
  uint32_t cap, cmask;           // table capacity used by this stage
  uint32_t cap_ws;
  int32_t ntile_ws, ncmax;
  int64_t tie_seg;
  const float* xyz;              // the cloud, [n][3]
  int32_t* idx;                  // output [M]
  hav_info_t* info_dev;          // caller's report or null
  int64_t M;
};

__device__ __forceinline__ unsigned long long* ctab_keys(const Ws& w, int set, int c) {
  return w.ckeys + (static_cast<size_t>(set) * w.ncmax + c) * w.cap_ws;
}
__device__ __forceinline__ unsigned long long* ctab_masks(const Ws& w, int set, int c) {
  return w.cmasks + (static_cast<size_t>(set) * w.ncmax + c) * w.cap_ws;
}
__device__ __forceinline__ int32_t* claims(const Ws& w, int set, int c, int tile) {
  return w.ccl + ((static_cast<size_t>(set) * w.ncmax + c) * w.ntile_ws + tile) * kClaimCap;
}
__device__ __forceinline__ unsigned long long* hrep_of(const Ws& w, int set, int c, int r) {
  return w.hrep + ((static_cast<size_t>(set) * w.ncmax + c) * kReps + r) * kHotCap;
}
__device__ __forceinline__ int32_t* claim_n(const Ws& w, int set, int c, int tile) {
  return w.ccn + (static_cast<size_t>(set) * w.ncmax + c) * w.ntile_ws + tile;
}

// Sorted storage is transposed inside each tile: the tile's (kPerThread*t + k)-th
// point sits in slot k*kThreads + t, so a coalesced load (lane t, rows k) hands
// thread t kPerThread neighbouring points. Slots past the cloud hold no point.
__device__ __forceinline__ int64_t slot_of(int64_t L) {
  const int64_t tile = L / kTile;
  const int j = static_cast<int>(L - tile * kTile);
  return tile * kTile + (j % kPerThread) * kThreads + j / kPerThread;
}
__device__ __forceinline__ int64_t logical_of(int64_t S) {
  const int64_t tile = S / kTile;
  const int j = static_cast<int>(S - tile * kTile);
  return tile * kTile + (j % kThreads) * kPerThread + j / kThreads;
}

// ----------------------------------------------------------------------------- clouds

// A cloud's device view and per-call constants. The single-cloud path passes it to
// every kernel by value (One); the batched path (Many) gives each kernel one grid over
// all clouds, and a block finds its cloud and its block index within that cloud's
// share of the grid in a block map built at the start of the call.
struct Cloud {
  Ws w;
  Plan P;
};

// Grid kinds: how many blocks a kernel gives a cloud of n points (kKScat: the
// binning blocks and one more, which starts layer 1 while the others scatter).
enum Kind : int { kKBBox = 0, kKBin, kKBScan, kKTile, kKOne, kKScan, kKScat, kKinds };

// Layout tuning code: the tuning field table_scale in bits 0-3, and the binning block's
// points (the tuning field bin_points) in bits 4-5: 0 = 4,096, 1 = 2,048, 2 = 8,192.
__host__ __device__ inline int tab_scale(int tcode) { return tcode & 15; }
__host__ __device__ inline int bin_shift(int tcode) {
  const int b = (tcode >> 4) & 3;
  return b == 1 ? 11 : (b == 2 ? 13 : 12);
}

// Chunks of kBinChunk cells one block of the histogram scan owns: the most (up to 8)
// that leave each thread at most kMaxBinBlocks / 16 binning blocks' counts to hold, so a
// small cloud's scan is a few blocks rather than kBinChunks nearly idle ones.
__host__ __device__ inline int scan_group(int64_t nbb) {
  int g = 1;
  while (g < 8 && nbb * (2 * g) <= kMaxBinBlocks) g *= 2;
  return g;
}

// bshift: log2 of the points of a binning block (a tuning field: the binning
// workgroup's share of the cloud).
__host__ __device__ inline int64_t blocks_of(int kind, int64_t n, int bshift = 12) {
  switch (kind) {
    case kKBBox: return n < 2048 ? 1 : (n + 2047) / 2048 < kMaxBBoxBlocks ? (n + 2047) / 2048 : kMaxBBoxBlocks;
    case kKBin: {
      const int64_t bp = int64_t(1) << bshift;
      return n < bp ? 1 : (n + bp - 1) / bp < kMaxBinBlocks ? (n + bp - 1) / bp : kMaxBinBlocks;
    }
    case kKBScan: return kBinChunks / scan_group(blocks_of(kKBin, n, bshift));
    case kKTile: return (n + kTile - 1) / kTile;
    case kKOne: return 1;
    case kKScat: return blocks_of(kKBin, n, bshift) + 1;
    default: return (n + kScanTile - 1) / kScanTile;
  }
}

struct BlockRef {
  int32_t c, b, nb, pad;  // cloud, block within the cloud's grid, the cloud's grid size
};

struct alignas(256) BatchDev {
  int32_t B;
  int32_t depth;               // speculation depth (the same for every cloud of a call)
  int32_t bshift;              // log2 points of a binning block (likewise)
  int32_t kind_off[kKinds];    // where each kind's block map starts in bmap
  int32_t kind_total[kKinds];
  int32_t nact;                // clouds searching in the current layer
  int32_t pad[1];
  Cloud* clouds;               // [B]
  BlockRef* bmap;              // [sum of kind_total]
  int32_t* act;                // [B] the searching clouds
  alignas(128) uint32_t nfin[kStride];  // searching clouds that have finished
  uint32_t err[kStride];
};

struct One {
  Cloud c;
};
struct Many {
  BatchDev* bd;
};

// Threads of a counting block (k_bin_count): a single cloud's 4,096-point blocks run at
// 512 (two waves per SIMD at one block per CU); the batched path keeps 256, which
// measured faster there, where several small blocks share a CU.
template <class Src>
struct CountThreads {
  static constexpr int value = kThreads;
};
template <>
struct CountThreads<One> {
  static constexpr int value = 2 * kThreads;
};

// The block's cloud (by reference: fields are loaded where they are used) and its
// block index and grid size within that cloud's share of the launch.
__device__ __forceinline__ const Cloud& cloud_of(const One& s, int, int& b, int& nb) {
  b = blockIdx.x;
  nb = gridDim.x;
  return s.c;
}
__device__ __forceinline__ const Cloud& cloud_of(const Many& s, int kind, int& b, int& nb) {
  const BlockRef r = s.bd->bmap[s.bd->kind_off[kind] + static_cast<int>(blockIdx.x)];
  b = r.b;
  nb = r.nb;
  return s.bd->clouds[r.c];
}

// Two-level arrival: true in exactly one block, the last to arrive. Every thread
// first waits for its own memory operations to complete, so the partial results the
// block published with atomic RMWs are in place before the arrival is counted; the
// last block reads them back with RMWs. Counters are left at zero.
__device__ bool arrive_last(Header* h, int block, int nblocks) {
  __shared__ int s_last;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = block & (kGroups - 1);
    const int gsize = (nblocks - g + kGroups - 1) / kGroups;
    const int ngroups = nblocks < kGroups ? nblocks : kGroups;
    int last = 0;
    const uint32_t a = atomicAdd(&h->sync_grp[g][0], 1u);
    if (a == static_cast<uint32_t>(gsize - 1)) {
      atomicExch(&h->sync_grp[g][0], 0u);
      const uint32_t b = atomicAdd(&h->sync_top[0], 1u);
      if (b == static_cast<uint32_t>(ngroups - 1)) {
        atomicExch(&h->sync_top[0], 0u);
        last = 1;
      }
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// Read-and-reset of an accumulator other blocks filled with atomics; plain read.
__device__ __forceinline__ uint32_t take(uint32_t* p) { return atomicExch(p, 0u); }
__device__ __forceinline__ uint32_t peek(uint32_t* p) { return atomicAdd(p, 0u); }

// ----------------------------------------------------------------------------- search plan

// Largest voxel coordinate per axis at reciprocal size inv: the coordinate of the
// cloud's max corner (r = mx - mn), the largest r any point has.
__device__ __forceinline__ void max_coords(const Frame& fr, const float* inv, uint32_t* mk) {
  for (int ax = 0; ax < 3; ++ax) mk[ax] = axis_coord(fr.mx[ax] - fr.mn[ax], inv[ax]);
}

// Candidates of the next pass: the next P.depth steps of the bisection as a model
// predicts them. Candidate 0 is the midpoint of the bracket [lo, hi]; candidate k+1
// is the midpoint of the half the model expects step k to keep (down, to [lo, s], when
// the count at s looks below m; up otherwise), computed with the same arithmetic as
// bisection itself. A candidate counts as an evaluation only if every step before it
// went the predicted way (search_step), so results are those of plain bisection; a
// good model just gets several steps out of one pass. The model is a power law
// Cnt(s) = c_ref (s_ref / s)^D through the counts known at the bracket ends (D fitted
// when both are known, else 2); the chain stops early where it predicts acceptance.
//
// Steps whose outcome is certain are taken without a count: at size s no point has a
// voxel coordinate above that of the max corner, so Cnt(s) is at most the number of
// grid cells up to it, and when that is below m the step goes down. Such a step still
// counts as an evaluation (the bisection is the same); the last step of the budget
// is always counted.
__device__ void plan_search(SState* st, const Plan& P, const Frame& fr, uint32_t m, uint32_t upper) {
  while (st->evals + 1 < P.t_max) {
    const float s = (st->lo + st->hi) * 0.5f;
    float inv[3];
    for (int ax = 0; ax < 3; ++ax) {
      const float v = s * P.aspect[ax];
      inv[ax] = 1.0f / v;
    }
    uint32_t mk[3];
    max_coords(fr, inv, mk);
    const double cells = (double(mk[0]) + 1.0) * (double(mk[1]) + 1.0) * (double(mk[2]) + 1.0);
    if (!(cells < static_cast<double>(m))) break;
    st->hi = s;
    st->evals += 1;
  }
  const int left = P.t_max - st->evals;
  const int D = left < P.depth ? left : P.depth;
  // the model: through the counts at both bracket ends when known; else through the
  // one known count with the binning's box-counting dimension; else the box-counting
  // prior itself (or one voxel at hi0, dimension 2, when the binning gave none)
  const float dim0 = fr.prior_ok ? fr.prior_d : 2.0f;
  float sref, cref, dim = dim0;
  if (st->c_lo && st->c_hi && st->lo > 0.0f && st->c_lo > st->c_hi) {
    sref = st->hi;
    cref = static_cast<float>(st->c_hi);
    dim = __logf(static_cast<float>(st->c_lo) / static_cast<float>(st->c_hi)) / __logf(st->hi / st->lo);
  } else if (st->c_hi) {
    sref = st->hi;
    cref = static_cast<float>(st->c_hi);
  } else if (st->c_lo) {
    sref = st->lo;
    cref = static_cast<float>(st->c_lo);
  } else if (fr.prior_ok) {
    sref = fr.prior_s;
    cref = fr.prior_c;
  } else {
    sref = fr.hi0;
    cref = 1.0f;
    dim = 2.0f;
  }
  float lo = st->lo, hi = st->hi;
  int nc = 0;
  for (int k = 0; k < D; ++k) {
    const float s = (lo + hi) * 0.5f;
    st->cand_s[k] = s;
    for (int ax = 0; ax < 3; ++ax) {
      const float v = s * P.aspect[ax];
      st->cand_inv[k][ax] = 1.0f / v;
    }
    const float pred = cref * __expf(dim * __logf(sref / s));
    // a speculative candidate predicted far finer than the window's scale would cost
    // a lot (its count, and so its table work, is large): end the chain before it
    if (k > 0 && pred > P.spec_mult * static_cast<float>(upper)) break;
    uint32_t mk[3];
    max_coords(fr, st->cand_inv[k], mk);
    const uint64_t nbx = (mk[0] >> kBrickShift) + 1, nby = (mk[1] >> kBrickShift) + 1,
                   nbz = (mk[2] >> kBrickShift) + 1;
    const uint64_t nb = nbx * nby * nbz;
    st->cand_dense[k] = nb <= P.cap ? 1 : 0;
    st->cand_hot[k] = nb <= static_cast<uint64_t>(kHotCap) ? 1 : 0;
    st->cand_nb[k][0] = static_cast<uint32_t>(nbx);
    st->cand_nb[k][1] = static_cast<uint32_t>(nby);
    nc = k + 1;
    if (pred >= static_cast<float>(m) && pred <= static_cast<float>(upper)) break;
    st->pdir[k] = pred < static_cast<float>(m) ? 0 : 1;
    if (st->pdir[k] == 0)
      hi = s;
    else
      lo = s;
  }
  st->nc = nc;
}

// The bisection steps of a pass, on its counts: candidate k is used only while the
// steps before it went the predicted way; then the next pass's candidates, or the
// final scale.
__device__ void search_step(SState* st, const uint32_t* cnt, const Plan& P, const Frame& fr,
                            uint32_t m, uint32_t upper) {
  st->prev_set = st->set;
  st->prev_nc = st->nc;
  uint32_t hm = 0;
  for (int k = 0; k < st->nc; ++k) hm |= static_cast<uint32_t>(st->cand_dense[k] == 0) << k;
  st->prev_hashed = hm;
  st->set ^= 1;
  for (int k = 0; k < st->nc; ++k) {
    const uint32_t cc = cnt[k];
    const float s = st->cand_s[k];
    st->evals += 1;
    if (cc >= m && cc <= upper) {
      st->accepted = 1;
      st->done = 1;
      st->s_final = s;
      st->c_final = cc;
      return;
    }
    const int dir = cc < m ? 0 : 1;
    if (dir == 0) {
      st->hi = s;
      st->c_hi = cc;
    } else {
      st->lo = s;
      st->c_lo = cc;
    }
    if (st->evals >= P.t_max) break;
    if (k + 1 < st->nc && dir != st->pdir[k]) break;  // the rest of the chain is off the path
  }
  if (st->evals >= P.t_max) {
    // no size in the window: the finest size with too many voxels if there was one
    // (then trim), else the smallest size evaluated (then pad)
    st->done = 1;
    st->s_final = st->lo > 0.0f ? st->lo : st->hi;
    // lo is always evaluated; hi is too when lo is 0 (the budget's last step is)
    st->c_final = st->lo > 0.0f ? st->c_lo : st->c_hi;
    return;
  }
  plan_search(st, P, fr, m, upper);
}

__device__ void set_select_grid(Ctrl* c, const Plan& P, const Frame& fr) {
  uint32_t mk[3];
  max_coords(fr, c->inv_final, mk);
  const uint64_t nv = (uint64_t(mk[0]) + 1) * (uint64_t(mk[1]) + 1) * (uint64_t(mk[2]) + 1);
  c->sel_dense = nv <= P.sel_cap ? 1 : 0;
  c->sel_nv[0] = mk[0] + 1;
  c->sel_nv[1] = mk[1] + 1;
}

__device__ void set_final(Ctrl* c, float s, const Plan& P, const Frame& fr) {
  c->s_final = s;
  for (int ax = 0; ax < 3; ++ax) {
    c->v_final[ax] = s * P.aspect[ax];
    c->inv_final[ax] = 1.0f / c->v_final[ax];
  }
  set_select_grid(c, P, fr);
}

// Trim window: with c voxels of which the m of smallest priority stay, the threshold
// is the m-th smallest of c priorities. SplitMix64 spreads keys evenly over 64 bits,
// so that order statistic lies near the fraction m / (c + 1) of the range, with
// standard deviation sqrt(x (1 - x) / (c + 2)). The window spans `sig` of them (by
// default kWinSigma) on each side; the selection kernel counts the voxels below and
// inside it and uses it as the trim bucket only if the threshold is proven to lie
// inside (any input stays exact: otherwise the bucket is every voxel).
__device__ void set_window(Ctrl* c, float sig) {
  c->win = 0;
  const uint32_t cf = c->c_final, m = c->m;
  if (cf <= m || m == 0 || !(sig > 0.0f)) return;
  const double kWin = sig;
  const double x = static_cast<double>(m) / (static_cast<double>(cf) + 1.0);
  const double sd = sqrt(x * (1.0 - x) / (static_cast<double>(cf) + 2.0));
  const double lo = (x - kWin * sd) * 0x1p64, hi = (x + kWin * sd) * 0x1p64;
  c->blo = lo <= 0.0 ? 0ull : (lo >= 0x1p64 ? ~0ull : static_cast<uint64_t>(lo));
  c->bhi = hi >= 0x1p64 ? ~0ull : (hi <= 0.0 ? 0ull : static_cast<uint64_t>(hi));
  int sh = 0;
  while (((c->bhi - c->blo) >> sh) >= static_cast<uint64_t>(kWinBins)) ++sh;
  c->wshift = sh;
  c->win = 1;
}

__device__ void layer_init_ctrl(Header* h, const Plan& P, int L);

// Start layer L; all threads of the block call it. The bulk clearing is spread over
// the block, the controller is thread 0's. (The layer's first search pass was planned
// when the call started: first_plans.)
__device__ void layer_init(Header* h, const Plan& P, int L) {
  for (int i = threadIdx.x; i < 2 * kMaxCand * kGroups; i += blockDim.x)
    h->sacc[i / (kMaxCand * kGroups)][(i / kGroups) % kMaxCand][i % kGroups][0] = 0;
  if (threadIdx.x < kGroups) h->sq_dgrp[threadIdx.x][0] = 0;
  if (threadIdx.x == 0) layer_init_ctrl(h, P, L);
}

// The first search pass of every layer, one thread per layer, into the header. A
// layer's first pass depends only on the frame (with the binning's prior) and the
// layer's budget: it starts from the whole bracket [0, hi0] and uses table set 0 (the
// tables of both sets are empty between layers, as at the start of a call).
__device__ void first_plans(Header* h, const Plan& P, const Frame& frame_in) {
  __shared__ SState s_pl[HAV_MAX_LAYERS];
  if (P.fixed) return;
  const int L = threadIdx.x;
  if (L < P.nlayers) {
    const Frame fl = frame_in;
    SState* s0 = &s_pl[L];
    s0->lo = 0.0f;
    s0->hi = fl.hi0;
    s0->c_hi = 0;
    s0->c_lo = 0;
    s0->evals = 0;
    s0->done = 0;
    s0->accepted = 0;
    s0->set = 0;
    s0->prev_set = 0;
    s0->prev_nc = 0;
    s0->prev_hashed = 0;
    s0->s_final = 0.0f;
    s0->c_final = 0;
    plan_search(s0, P, fl, P.m[L], P.upper[L]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P.nlayers * kPubWords; i += blockDim.x)
    h->pub_first[i / kPubWords][i % kPubWords] =
        reinterpret_cast<const uint32_t*>(&s_pl[i / kPubWords])[i % kPubWords];
}

__device__ void layer_init_ctrl(Header* h, const Plan& P, int L) {
  Ctrl* c = &h->ctrl;
  c->layer = L;
  c->m = P.m[L];
  c->upper = P.upper[L];
  c->evals = 0;
  c->accepted = 0;
  c->ncand = 0;
  c->trim = 0;
  c->need = 0;
  c->rank = 0;
  c->prefix = 0;
  c->rounds_done = 0;
  c->trim_mode = 0;
  c->c_final = 0;
  c->win = 0;
  h->info.m[L] = static_cast<int32_t>(P.m[L]);
  h->info.layers = L + 1;
  h->sq_ticket[0] = 0;
  h->sq_done[0] = 0;
  h->sq_gen[0] = 0;
  h->sq_fin[0] = 0;
  h->sq_err[0] = 0;
  if (P.fixed) {
    const Frame fl = h->frame;
    c->done = 1;
    c->s_final = 0.0f;
    for (int ax = 0; ax < 3; ++ax) {
      c->v_final[ax] = P.fixed_v[ax];
      c->inv_final[ax] = 1.0f / P.fixed_v[ax];
    }
    set_select_grid(c, P, fl);
  } else {
    c->done = 0;
  }
}

// ----------------------------------------------------------------------------- frame

template <class Src>
__global__ void __launch_bounds__(kThreads) k_bbox(Src src) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKBBox, bx, gx);
  const Ws& w = cd.w;
  const float* __restrict__ xyz = w.xyz;
  if (bx == 0 && threadIdx.x == 0) w.h->binned_n = 0;  // (set again once this call has binned)
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
  uint32_t hi[3] = {0u, 0u, 0u};
  uint32_t bad = 0;
  const int64_t n = w.n;
  // a contiguous share of the cloud per block, eight points per thread per round with
  // their loads in flight together; an index past the share reads its last point again
  // (no effect on a min, a max or an or), so every load and its use are unconditional
  constexpr int kBB = 8;
  const int64_t chunk = (n + gx - 1) / gx;
  const int64_t beg = bx * chunk, end = min(n, beg + chunk);
  for (int64_t i0 = beg; i0 < end; i0 += static_cast<int64_t>(kBB) * kThreads) {
    float c[kBB][3];
#pragma unroll
    for (int k = 0; k < kBB; ++k) {
      const int64_t i = min(end - 1, i0 + threadIdx.x + static_cast<int64_t>(k) * kThreads);
#pragma unroll
      for (int a = 0; a < 3; ++a) c[k][a] = xyz[3 * i + a];
    }
#pragma unroll
    for (int k = 0; k < kBB; ++k)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bad |= !isfinite(c[k][a]);
        const uint32_t o = float_to_ordered(c[k][a]);
        lo[a] = min(lo[a], o);
        hi[a] = max(hi[a], o);
      }
  }
  // tags cleared 16 at a time (both arrays start 256-byte aligned; tag_o's region is
  // padded to a multiple of 256 bytes, tag_s holds whole tiles)
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  const int64_t stride = static_cast<int64_t>(gx) * kThreads;
  for (int64_t q = bx * static_cast<int64_t>(kThreads) + threadIdx.x; q < (n + 15) / 16; q += stride)
    reinterpret_cast<uint4*>(w.tag_o)[q] = z4;
  for (int64_t q = bx * static_cast<int64_t>(kThreads) + threadIdx.x; q < w.npad / 16; q += stride) {
    const int64_t S0 = 16 * q;
    if ((S0 / kTile + 1) * kTile <= n) {  // a whole tile of points: every slot holds one
      reinterpret_cast<uint4*>(w.tag_s)[q] = z4;
    } else {
      uint32_t v[4] = {0u, 0u, 0u, 0u};
      for (int b = 0; b < 16; ++b)
        if (logical_of(S0 + b) >= n) v[b >> 2] |= 0xFFu << (8 * (b & 3));  // 0xFF: empty slot
      reinterpret_cast<uint4*>(w.tag_s)[q] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  }
  __shared__ uint32_t s_v[7][kThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t vals[7] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], bad};
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    uint32_t v = vals[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t y = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o, 64));
      v = (k < 3) ? min(v, y) : ((k < 6) ? max(v, y) : (v | y));
    }
    if (lane == 0) s_v[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    uint32_t v = s_v[k][0];
    for (int q = 1; q < kThreads / 64; ++q)
      v = (k < 3) ? min(v, s_v[k][q]) : ((k < 6) ? max(v, s_v[k][q]) : (v | s_v[k][q]));
    w.part[bx * 8 + k] = v;
  }
}

// Reduce the k_bbox partials and derive the stage frame. Every block of the calling
// kernel does this itself and gets the same bits; only block 0 publishes them.
// Returns the status.
template <int NT>
__device__ int frame_from_partials(const Ws& w, const Plan& P, Frame* fr, int identity) {
  __shared__ uint32_t s_v[7][NT / 64];
  uint32_t v[7] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u, 0u};
  const uint64_t magic = w.h->magic;  // in flight with the partials
  // every thread's partials (nbbox <= kMaxBBoxBlocks) in one round trip
  constexpr int kJ = (kMaxBBoxBlocks + NT - 1) / NT;
  const uint4* p4 = reinterpret_cast<const uint4*>(w.part);
  uint4 pa[kJ], pb[kJ];
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    const int b = threadIdx.x + j * NT;
    if (b < w.nbbox) {
      pa[j] = p4[2 * b];
      pb[j] = p4[2 * b + 1];
    } else {
      pa[j] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u);
      pb[j] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
#pragma unroll
  for (int j = 0; j < kJ; ++j) {
    v[0] = min(v[0], pa[j].x);
    v[1] = min(v[1], pa[j].y);
    v[2] = min(v[2], pa[j].z);
    v[3] = max(v[3], pa[j].w);
    v[4] = max(v[4], pb[j].x);
    v[5] = max(v[5], pb[j].y);
    v[6] |= pb[j].z;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    uint32_t x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t y = static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), o, 64));
      x = (k < 3) ? min(x, y) : ((k < 6) ? max(x, y) : (x | y));
    }
    if (lane == 0) s_v[k][wv] = x;
  }
  __syncthreads();
  for (int k = 0; k < 7; ++k) {
    uint32_t x = s_v[k][0];
    for (int q = 1; q < NT / 64; ++q)
      x = (k < 3) ? min(x, s_v[k][q]) : ((k < 6) ? max(x, s_v[k][q]) : (x | s_v[k][q]));
    v[k] = x;
  }
  __syncthreads();
  int status = HAV_OK;
  if (magic != P.magic) status = HAV_ERR_WORKSPACE_NOT_INIT;
  else if (v[6]) status = HAV_ERR_NONFINITE;
  float E = 0.0f;
  for (int a = 0; a < 3; ++a) {
    fr->mn[a] = ordered_to_float(v[a]);
    fr->mx[a] = ordered_to_float(v[3 + a]);
    const float ext = fr->mx[a] - fr->mn[a];
    const float e = ext / P.aspect[a];
    if (!(e <= E)) E = e;
  }
  fr->hi0 = 0.0f;
  if (status == HAV_OK && !identity) {
    if (!(E <= 0x1p100f)) {
      status = HAV_ERR_UNSUPPORTED;
    } else {
      const float Ec = E < 0x1p-64f ? 0x1p-64f : E;
      const uint32_t bits = __float_as_uint(Ec);
      fr->hi0 = (bits & 0x7FFFFFu) ? __uint_as_float((bits & 0x7F800000u) + 0x00800000u) : Ec;
      if (P.fixed) {
        for (int a = 0; a < 3; ++a) {
          const float inv = 1.0f / P.fixed_v[a];
          const float q = (fr->mx[a] - fr->mn[a]) * inv;
          if (!(q < kKeyLimit)) status = HAV_ERR_UNSUPPORTED;
        }
      }
    }
  }
  // spatial binning: 12 Morton bits shared out by extent (affects speed only)
  float ext[3];
  int bb[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) ext[a] = fr->mx[a] - fr->mn[a];
  for (int k = 0; k < kBinBits; ++k) {
    int best = 0;
    float bv = -1.0f;
    for (int a = 0; a < 3; ++a) {
      const float q = ldexpf(ext[a], -bb[a]);  // (exact: a power-of-two scaling)
      if (q > bv) {
        bv = q;
        best = a;
      }
    }
    bb[best] += 1;
  }
  for (int a = 0; a < 3; ++a) {
    fr->bbits[a] = bb[a];
    fr->bscale[a] = ext[a] > 0.0f ? static_cast<float>(1 << bb[a]) / ext[a] : 0.0f;
    if (!isfinite(fr->bscale[a])) fr->bscale[a] = 0.0f;
  }
  fr->prior_s = fr->prior_c = fr->prior_d = 0.0f;
  fr->prior_ok = 0;  // (set by the binning's scan)
  fr->status = status;
  return status;
}

__device__ void publish_frame(const Ws& w, const Frame& fr, int block) {
  if (block != 0 || threadIdx.x != 0) return;
  w.h->frame = fr;
  hav_info_t* info = &w.h->info;
  int32_t* z = reinterpret_cast<int32_t*>(info);
  for (int i = 0; i < static_cast<int>(sizeof(hav_info_t) / 4); ++i) z[i] = 0;
  info->status = fr.status;
  info->hi0 = fr.hi0;
  for (int a = 0; a < 3; ++a) {
    info->mn[a] = fr.mn[a];
    info->mx[a] = fr.mx[a];
  }
}

// The cell numbering of a frame, in registers: per axis the scale, the top cell, the
// bit count and the 4-bit positions of its bits in the cell number (packed), so that
// numbering a point touches no memory.
struct CellCoder {
  float scale[3];
  uint32_t lim[3];
  int bb[3];
  uint64_t pos[3];
};

__device__ __forceinline__ CellCoder make_coder(const Frame& fr) {
  CellCoder k;
  for (int a = 0; a < 3; ++a) {
    k.scale[a] = fr.bscale[a];
    k.bb[a] = fr.bbits[a];
    k.lim[a] = (1u << k.bb[a]) - 1u;
    k.pos[a] = 0ull;
  }
  uint32_t p = 0;
  for (int j = 0; j < kBinBits; ++j)
    for (int a = 0; a < 3; ++a)
      if (j < k.bb[a]) k.pos[a] |= static_cast<uint64_t>(p++) << (4 * j);
  return k;
}

// The cell index of offset r along axis a: floor(r * scale), clamped to the top cell
// (and to 0 below: a point's r is never negative, a bound of a search range can be).
// Non-decreasing in r.
__device__ __forceinline__ uint32_t cell_index(float r, const CellCoder& k, int a) {
  // (fmaxf takes 0 for a NaN product; the clamped value converts exactly)
  return static_cast<uint32_t>(fminf(fmaxf(r * k.scale[a], 0.0f), static_cast<float>(k.lim[a])));
}
// The cell number of cell indices (cx, cy, cz): their bits interleaved (Morton order).
// Index bits at or above an axis's bit count are 0 (cell_index clamps) and their position
// nibbles are 0, so every bit is deposited unconditionally.
__device__ __forceinline__ uint32_t cell_code_of(const uint32_t (&c)[3], const CellCoder& k) {
  uint32_t code = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int j = 0; j < kBinBits; ++j)
      code |= ((c[a] >> j) & 1u) << ((k.pos[a] >> (4 * j)) & 15u);
  }
  return code;
}
// The cell number of offset (rx, ry, rz).
__device__ __forceinline__ uint32_t cell_code_k(float rx, float ry, float rz, const CellCoder& k) {
  const uint32_t c[3] = {cell_index(rx, k, 0), cell_index(ry, k, 1), cell_index(rz, k, 2)};
  return cell_code_of(c, k);
}

// The same numbering by table lookup, for the binning's per-point loops: per axis, the
// deposited bits of the low and of the high six bits of a cell index (12 bits at most),
// so a point costs six LDS reads instead of a deposit of every index bit.
struct CellLut {
  uint32_t d[3][2][64];
};
// All threads call; the table is complete after the block's next barrier.
__device__ __forceinline__ void build_lut(CellLut& L, const CellCoder& k) {
  static_assert(kBinBits <= 12, "two six-bit halves per cell index");
  for (int e = threadIdx.x; e < 3 * 2 * 64; e += blockDim.x) {
    const int a = e >> 7, hf = (e >> 6) & 1, v = e & 63;
    uint32_t code = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) code |= ((v >> j) & 1u) << ((k.pos[a] >> (4 * (6 * hf + j))) & 15u);
    L.d[a][hf][v] = code;
  }
}
__device__ __forceinline__ uint32_t cell_code_lut(float rx, float ry, float rz, const CellCoder& k,
                                                  const CellLut& L) {
  const uint32_t cx = cell_index(rx, k, 0), cy = cell_index(ry, k, 1), cz = cell_index(rz, k, 2);
  return L.d[0][0][cx & 63u] | L.d[0][1][cx >> 6] | L.d[1][0][cy & 63u] | L.d[1][1][cy >> 6] |
         L.d[2][0][cz & 63u] | L.d[2][1][cz >> 6];
}


template <class Src>
__global__ void __launch_bounds__(kThreads) k_identity(Src src) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKScan, bx, gx);
  const Ws& w = cd.w;
  const Plan& P = cd.P;
  if (!P.identity) return;
  int32_t* idx = w.idx;
  hav_info_t* info_dev = w.info_dev;
  __shared__ Frame fr;
  Frame f;
  const int st = frame_from_partials<kThreads>(w, P, &f, 1);
  if (threadIdx.x == 0) fr = f;
  __syncthreads();
  if (bx == 0 && threadIdx.x == 0) {
    publish_frame(w, fr, bx);
    if (info_dev) *info_dev = w.h->info;
  }
  if (st != HAV_OK) return;
  for (int64_t i = bx * static_cast<int64_t>(kThreads) + threadIdx.x; i < w.n;
       i += static_cast<int64_t>(gx) * kThreads) {
    idx[i] = static_cast<int32_t>(i);
    if (w.xyz_out)
      for (int a = 0; a < 3; ++a) w.xyz_out[3 * i + a] = w.xyz[3 * i + a];
  }
}

// ----------------------------------------------------------------------------- binning

template <class Src>
__global__ void __launch_bounds__(CountThreads<Src>::value) k_bin_count(Src src) {
  constexpr int kCountThreads = CountThreads<Src>::value;
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKBin, bx, gx);
  const Ws& w = cd.w;
  const Plan& P = cd.P;
  if (P.identity) return;
  const float* __restrict__ xyz = w.xyz;
  __shared__ Frame fr;
  __shared__ uint32_t hist[kBins];
  const int64_t chunk = (w.n + w.nbb - 1) / w.nbb;
  const int64_t beg = bx * chunk, end = min(w.n, beg + chunk);
  // 4,096 points per block and round, all loads in flight together; the first round's
  // loads are issued before the frame's partials, so the two round trips overlap
  constexpr int kBP = 4096 / kCountThreads;
  float px[kBP], py[kBP], pz[kBP];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int k = 0; k < kBP; ++k) {
      const int64_t i = i0 + threadIdx.x + static_cast<int64_t>(k) * kCountThreads;
      if (i < end) {
        px[k] = xyz[3 * i];
        py[k] = xyz[3 * i + 1];
        pz[k] = xyz[3 * i + 2];
      }
    }
  };
  load(beg);
  Frame f;
  const int st = frame_from_partials<kCountThreads>(w, P, &f, 0);  // (the same frame in every thread)
  if (threadIdx.x == 0) fr = f;
  for (int i = threadIdx.x; i < kBins; i += kCountThreads) hist[i] = 0;
  const CellCoder kc = make_coder(f);
  __shared__ CellLut lut;
  build_lut(lut, kc);
  __syncthreads();
  publish_frame(w, fr, bx);
  if (st != HAV_OK) return;
  const float m0 = f.mn[0], m1 = f.mn[1], m2 = f.mn[2];
  for (int64_t i0 = beg; i0 < end; i0 += static_cast<int64_t>(kBP) * kCountThreads) {
    // (every earlier load has landed: the compiler need not wait before each new one)
    if (i0 != beg) {
      __builtin_amdgcn_s_waitcnt(0);
      load(i0);
    }
#pragma unroll
    for (int k = 0; k < kBP; ++k) {
      const int64_t i = i0 + threadIdx.x + static_cast<int64_t>(k) * kCountThreads;
      if (i < end) atomicAdd(&hist[cell_code_lut(px[k] - m0, py[k] - m1, pz[k] - m2, kc, lut)], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += kCountThreads)
    w.bh[static_cast<size_t>(bx) * kBins + b] = hist[b];
}

// Offsets of every (block, cell) run of the counting sort. Block c of this kernel owns
// the ncell = 16 G cells from c ncell on (G = scan_group(nbb)): kThreads / ncell threads
// per cell scan its counts over the binning blocks (an equal share of them each), then
// each 16-cell chunk is scanned within a 16-lane segment; the last block scans the
// chunk totals.
template <class Src>
__global__ void __launch_bounds__(kThreads) k_bin_scan(Src src) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKBScan, bx, gx);
  const Ws& w = cd.w;
  const Plan& P = cd.P;
  if (P.identity) return;
  if (w.h->frame.status != HAV_OK) return;
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint32_t s_q[kThreads];
  __shared__ uint32_t s_tot[kThreads];
  const int ncell = scan_group(w.nbb) * kBinChunk;
  const int parts = kThreads / ncell;
  const int lb = threadIdx.x & (ncell - 1);
  const int q = threadIdx.x / ncell;
  const int bin = bx * ncell + lb;
  const int nq = (w.nbb + parts - 1) / parts;
  const int b0 = q * nq, b1 = min(w.nbb, b0 + nq);
  // this thread's counts (at most 32: scan_group keeps nbb * G <= kMaxBinBlocks) in
  // registers, one round trip
  constexpr int kQ = kMaxBinBlocks / (kThreads / kBinChunk);
  uint32_t v[kQ];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kQ; ++j) v[j] = b0 + j < b1 ? w.bh[static_cast<size_t>(b0 + j) * kBins + bin] : 0u;
#pragma unroll
  for (int j = 0; j < kQ; ++j) sum += v[j];
  s_q[threadIdx.x] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int qq = 0; qq < q; ++qq) run += s_q[qq * ncell + lb];
  if (q == parts - 1) s_tot[lb] = run + sum;
#pragma unroll
  for (int j = 0; j < kQ; ++j) {
    if (b0 + j < b1) w.bh[static_cast<size_t>(b0 + j) * kBins + bin] = run;
    run += v[j];
  }
  __syncthreads();
  const bool mine = static_cast<int>(threadIdx.x) < ncell;
  const uint32_t x = mine ? s_tot[threadIdx.x] : 0u;
  // box counting for the search's prior: occupied cells, and occupied groups of 8
  // consecutive cells (the parent cells, each axis halved, when every axis has cell
  // bits: the lowest three bits of a cell number are one bit of each axis). A wave
  // holds whole groups; one packed atomic per wave.
  static_assert(kBinChunk % 8 == 0, "whole parent groups per chunk");
  {
    const uint64_t occ = __ballot(mine && x != 0u);
    if ((threadIdx.x & 63) == 0 && occ) {
      uint32_t groups = 0;
#pragma unroll
      for (int g = 0; g < 8; ++g) groups += ((occ >> (8 * g)) & 0xFFull) ? 1u : 0u;
      atomicAdd(&w.h->acc[3][(bx * (kThreads / 64) + (threadIdx.x >> 6)) & (kGroups - 1)][0],
                (groups << 16) | static_cast<uint32_t>(__popcll(occ)));
    }
  }
  // each chunk's inclusive scan within its 16-lane segment
  const int lc = threadIdx.x & (kBinChunk - 1);
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < kBinChunk; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, kBinChunk);
    if (lc >= d) inc += y;
  }
  if (mine) {
    w.binpre[bx * ncell + threadIdx.x] = inc - x;
    if (lc == kBinChunk - 1) atomicExch(&w.bsum[bx * (ncell / kBinChunk) + (threadIdx.x / kBinChunk)], inc);
  }
  if (!arrive_last(w.h, bx, gx)) return;
  static_assert(kBinChunks <= kThreads, "one chunk total per thread");
  const uint32_t y = threadIdx.x < kBinChunks ? peek(&w.bsum[threadIdx.x]) : 0u;
  uint32_t ey;
  block_exclusive_scan<kThreads>(y, &ey, s_tmp);
  if (threadIdx.x < kBinChunks) w.bsum[threadIdx.x] = ey;
}

// The search's prior from the binning's occupancy counts, the controller's reset and
// the start of layer 1 (one block; the frame is complete once the scan has run).
__device__ void start_search(const Ws& w, const Plan& P) {
  __shared__ uint32_t s_occ[2];
  if (threadIdx.x < 2) s_occ[threadIdx.x] = 0u;
  __syncthreads();
  if (threadIdx.x < kGroups) {
    const uint32_t v = take(&w.h->acc[3][threadIdx.x][0]);
    if (v) {
      atomicAdd(&s_occ[0], v & 0xFFFFu);
      atomicAdd(&s_occ[1], v >> 16);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // prior: occupied cells at the binning cell size (geometric mean over the axes that
    // have cells), dimension from the parent level; not when the cells are nearly all
    // occupied (the fine level is saturated and says nothing about finer scales)
    Frame* f = &w.h->frame;
    const uint32_t o12 = s_occ[0], o9 = s_occ[1];
    int bbl[3];
    float bsl[3];
    for (int a = 0; a < 3; ++a) {  // loads first, all in flight
      bbl[a] = f->bbits[a];
      bsl[a] = f->bscale[a];
    }
    float lsum = 0.0f;
    int na = 0;
    for (int a = 0; a < 3; ++a)
      if (bbl[a] > 0 && bsl[a] > 0.0f) {
        lsum += __logf(1.0f / bsl[a]);
        ++na;
      }
    f->prior_ok = 0;
    if (na > 0 && o9 > 0 && o12 > 0 && o12 <= static_cast<uint32_t>(kBins) * 3u / 4u) {
      const float d = __log2f(static_cast<float>(o12) / static_cast<float>(o9));
      f->prior_d = d < 1.0f ? 1.0f : (d > 3.0f ? 3.0f : d);
      f->prior_s = __expf(lsum / static_cast<float>(na));
      f->prior_c = static_cast<float>(o12);
      f->prior_ok = isfinite(f->prior_s) && f->prior_s > 0.0f ? 1 : 0;
    }
  }
  if (threadIdx.x == 0) {
    Ctrl* c = &w.h->ctrl;
    c->set = 0;
    c->pend_nc = 0;
    c->pend_set = 0;
    c->pend_hashed = 0;
    w.h->binned_n = w.n;  // the sorted cloud (scattered by this launch) stays for grouping
  }
  __shared__ Frame s_fr;
  if (threadIdx.x == 0) s_fr = w.h->frame;  // (thread 0 wrote the prior above)
  __syncthreads();
  layer_init(w.h, P, 0);
  first_plans(w.h, P, s_fr);
}

// NT: 512 for a single cloud of at most 256 binning blocks (one per CU), else 256 (at
// two or more blocks per CU, and in a batch, 512-thread blocks measured slower).
template <class Src, int NT>
__global__ void __launch_bounds__(NT) k_bin_scatter(Src src) {
  constexpr int kScatThreads = NT;
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKScat, bx, gx);
  const Ws& w = cd.w;
  if (cd.P.identity) return;
  const float* __restrict__ xyz = w.xyz;
  if (w.h->frame.status != HAV_OK) return;
  if (bx == gx - 1) {  // the extra block
    start_search(w, cd.P);
    return;
  }
  __shared__ Frame fr;
  __shared__ uint32_t off[kBins];
  // The chunk this block sorts. Workgroups go to the eight XCDs in turn, so the blocks one
  // XCD runs are every eighth; up to one binning block per CU they take consecutive
  // chunks. A cell's run holds the chunks' points in chunk order, so each of its lines is
  // then mostly written through one XCD's L2 instead of in parts through eight (the
  // scatter 21 -> 18 us at 1M points; with more blocks it measured no faster).
  int cb = bx;
  if (w.nbb <= 256) {
    cb = 0;
    for (int y = 0; y < (bx & 7); ++y) cb += (w.nbb - y + 7) >> 3;
    cb += bx >> 3;
  }
  const int64_t chunk = (w.n + w.nbb - 1) / w.nbb;
  const int64_t beg = cb * chunk, end = min(w.n, beg + chunk);
  constexpr int kBP = 4096 / kScatThreads;  // points per thread per round
  float px[kBP], py[kBP], pz[kBP];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int k = 0; k < kBP; ++k) {
      const int64_t i = i0 + threadIdx.x + static_cast<int64_t>(k) * kScatThreads;
      if (i < end) {
        px[k] = xyz[3 * i];
        py[k] = xyz[3 * i + 1];
        pz[k] = xyz[3 * i + 2];
      }
    }
  };
  load(beg);  // (in flight with the frame and the offsets)
  if (threadIdx.x == 0) fr = w.h->frame;
  static_assert(kBins % kScatThreads == 0, "cells per thread");
#pragma unroll
  for (int j = 0; j < kBins / kScatThreads; ++j) {
    const int b = threadIdx.x + j * kScatThreads;
    off[b] = w.bh[static_cast<size_t>(cb) * kBins + b] + w.binpre[b] + w.bsum[b / kBinChunk];
  }
  __syncthreads();
  const CellCoder kc = make_coder(fr);
  __shared__ CellLut lut;
  build_lut(lut, kc);
  __syncthreads();
  const float m0 = fr.mn[0], m1 = fr.mn[1], m2 = fr.mn[2];
  for (int64_t i0 = beg; i0 < end; i0 += static_cast<int64_t>(kBP) * kScatThreads) {
    // (every earlier load has landed: the compiler need not wait before each new one)
    if (i0 != beg) {
      __builtin_amdgcn_s_waitcnt(0);
      load(i0);
    }
#pragma unroll
    for (int k = 0; k < kBP; ++k) {
      const int64_t i = i0 + threadIdx.x + static_cast<int64_t>(k) * kScatThreads;
      if (i >= end) continue;
      const float rx = px[k] - m0;
      const float ry = py[k] - m1;
      const float rz = pz[k] - m2;
      const uint32_t pos = atomicAdd(&off[cell_code_lut(rx, ry, rz, kc, lut)], 1u);
      if (pos < w.n) {
        const int64_t S = slot_of(pos);
        w.pts[S] = make_float4(rx, ry, rz, __int_as_float(static_cast<int32_t>(i)));
        w.invp[i] = static_cast<int32_t>(S);
      }
    }
  }
}

// ----------------------------------------------------------------------------- search

template <typename T>
__device__ __forceinline__ T ld_agent(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Empty the table words one tile claimed in a search pass over `nc` candidates of
// table set `set`, leaving the tables as initialised. A claim is a brick table slot
// (>= 0), or -(1 + r * kHotCap + slot) for a word of hot replica r. Bit k of
// `hashed` marks candidates whose brick table is hashed (its keys are cleared too).
// Uses block-shared s_cn[kMaxCand + 1]; all threads call it.
__device__ void clear_claims(const Ws& w, int set, int k0, int k1, uint32_t hashed, int tile, int* s_cn) {
  const int nk = k1 > k0 ? k1 - k0 : 0;
  if (static_cast<int>(threadIdx.x) < nk) s_cn[threadIdx.x + 1] = ld_agent(claim_n(w, set, k0 + threadIdx.x, tile));
  __syncthreads();
  if (threadIdx.x == 0) {
    s_cn[0] = 0;
    for (int j = 0; j < nk; ++j) s_cn[j + 1] += s_cn[j];
  }
  __syncthreads();
  const int total = s_cn[nk];
  for (int e = threadIdx.x; e < total; e += kThreads) {
    int j = 0;
    while (e >= s_cn[j + 1]) ++j;
    const int k = k0 + j;
    const int32_t id = ld_agent(claims(w, set, k, tile) + (e - s_cn[j]));
    if (id >= 0) {
      if ((hashed >> k) & 1u) atomicExch(ctab_keys(w, set, k) + id, static_cast<unsigned long long>(kEmptyKey));
      atomicExch(ctab_masks(w, set, k) + id, 0ull);
    } else {
      const int32_t q = -1 - id;
      atomicExch(hrep_of(w, set, k, q / kHotCap) + (q % kHotCap), 0ull);
    }
  }
  __syncthreads();
}

// The claims of the search's last pass, for one tile.
__device__ void clear_pending(const Ws& w, const Ctrl* c, int tile) {
  __shared__ int s_cn[kMaxCand + 1];
  clear_claims(w, c->pend_set, 0, c->pend_nc, c->pend_hashed, tile, s_cn);
}

// Whether a cloud has work in layer L (batched grids skip the others).
__device__ __forceinline__ bool layer_due(const Cloud& cd, int L) {
  return !cd.P.identity && L < cd.P.nlayers && cd.w.h->frame.status == HAV_OK;
}

constexpr float kSpecMult = 16.0f;

struct EvalShared {
  int ncl[kMaxCand];
  uint32_t fresh[kMaxCand];
  uint32_t box[kMaxCand][6];  // brick box: lo x,y,z, extent x,y, volume (0: hash)
  uint32_t boxm[kMaxCand][2]; // exact-division multipliers of the box extents x, y
  int nu;                     // flush units: a candidate, or each half of a box above kBrickCap
  int unit_c[2 * kMaxCand], unit_h[2 * kMaxCand];
  uint32_t red[kThreads / 64][6];
  uint32_t tb[6];             // tile's min (0..2) and max (3..5) offset bits per axis
};

// Inside the search launch, memory that another block writes (tables, claim lists,
// counts, the published state) is only written with atomics and read with
// agent-scope atomic loads: a plain load could return a line this compute die's L2
// cached in an earlier pass.

// OR `bits` into the brick table entry of `key` (hashed table); returns the number
// of bits that were not set before. Each probe step is one CAS, which both finds the
// key and claims an empty slot; a tile that claims a slot records it.
__device__ __forceinline__ uint32_t global_or(unsigned long long* keys, unsigned long long* masks,
                                                uint32_t cmask, uint64_t key, uint64_t bits,
                                                int32_t* list, int* s_ncl) {
  uint32_t s = table_hash(key) & cmask;
  while (true) {
    const unsigned long long prev = atomicCAS(&keys[s], kEmptyKey, static_cast<unsigned long long>(key));
    if (prev == kEmptyKey || prev == key) {
      if (prev == kEmptyKey) st_agent(&list[atomicAdd(s_ncl, 1)], static_cast<int32_t>(s));
      const unsigned long long old = atomicOr(&masks[s], static_cast<unsigned long long>(bits));
      return static_cast<uint32_t>(__popcll(bits & ~old));
    }
    s = (s + 1) & cmask;
  }
}

// Dense brick table: `bits` ORed into word `slot`; the tile whose atomic finds the
// word empty records it.
__device__ __forceinline__ uint32_t dense_or(unsigned long long* masks, uint32_t slot,
                                             uint64_t bits, int32_t* list, int* s_ncl) {
  const unsigned long long old = atomicOr(&masks[slot], static_cast<unsigned long long>(bits));
  if (old == 0ull) st_agent(&list[atomicAdd(s_ncl, 1)], static_cast<int32_t>(slot));
  return static_cast<uint32_t>(__popcll(bits & ~old));
}

// a / d for a < 2^11 and 1 <= d <= 2^11, with m = div_magic(d): m = floor((2^32 - 1) / d)
// + 1 exceeds 2^32 / d by less than 1 (equals it for a power of two), so a * m / 2^32 exceeds
// a / d by less than 2^-21, below the distance 1/d of a non-multiple to the next integer.
__device__ __forceinline__ uint32_t div_magic(uint32_t d) { return d <= 1u ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ uint32_t box_div(uint32_t a, uint32_t m) { return m ? __umulhi(a, m) : a; }

// Issue the loads of a tile's points (thread t: the tile's points 8t..8t+7) and
// their layer tags; every slot of a tile exists, so no load depends on another.
__device__ __forceinline__ void issue_tile(const Ws& w, int tile, float4 (&pt)[kPerThread],
                                           uint32_t (&tg)[kPerThread]) {
  const int64_t base = static_cast<int64_t>(tile) * kTile + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t S = base + k * kThreads;
    tg[k] = w.tag_s[S];
    pt[k] = w.pts[S];
  }
}

// Keep the live points (tag 0) and reduce the tile's offset range: each wave's share into
// sh.red (finish_tile_a), then, after a barrier, the tile's into sh.tb (finish_tile_b).
__device__ __forceinline__ void finish_tile_a(float4 (&pt)[kPerThread], const uint32_t (&tg)[kPerThread],
                                              uint32_t& live, EvalShared& sh) {
  live = 0;
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const bool ok = tg[k] == 0;
    if (!ok) pt[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) {
      live |= 1u << k;
      // offsets are >= +0, so their bit patterns order like their values
      const uint32_t bx = __float_as_uint(pt[k].x), by = __float_as_uint(pt[k].y),
                     bz = __float_as_uint(pt[k].z);
      lo[0] = min(lo[0], bx); lo[1] = min(lo[1], by); lo[2] = min(lo[2], bz);
      hi[0] = max(hi[0], bx); hi[1] = max(hi[1], by); hi[2] = max(hi[2], bz);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t r[6];
  for (int a = 0; a < 3; ++a) {
    r[a] = __ockl_wfred_min_u32(lo[a]);
    r[3 + a] = __ockl_wfred_max_u32(hi[a]);
  }
  if (lane == 0)
    for (int q = 0; q < 6; ++q) sh.red[wv][q] = r[q];
}
__device__ __forceinline__ void finish_tile_b(EvalShared& sh) {
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    uint32_t v = q < 3 ? 0xFFFFFFFFu : 0u;
    for (int j = 0; j < kThreads / 64; ++j) v = q < 3 ? min(v, sh.red[j][q]) : max(v, sh.red[j][q]);
    sh.tb[q] = v;
  }
}

// Cnt contributions of one loaded tile at the pass's candidates, added to sh.fresh.
// Each candidate has kCandWords LDS words (from lvals, in the order of the launch's
// candidates): a box of up to kCandWords brick words, or kBrickCap hash values followed by
// kBrickCap hash keys (stored as key + 1, so that an empty slot reads 0). All are 0 on
// entry and left 0.
// `mid` runs (all threads) between the LDS phase and the global flush.
template <class Mid>
__device__ __forceinline__ void eval_loaded(const Ws& w, int tile, const SState& st,
                                            EvalShared& sh, uint64_t* lvals, uint64_t* lkeys,
                                            const float4 (&pt)[kPerThread], uint32_t live, int cb,
                                            int ce, int lb, Mid&& mid) {
  const int set = st.set;
  if (cb + static_cast<int>(threadIdx.x) < ce) {
    const int k = cb + threadIdx.x;
    sh.ncl[k] = 0;
    uint32_t l[3], u[3];
    for (int a = 0; a < 3; ++a) {
      uint32_t mn = sh.tb[a], mx = sh.tb[3 + a];
      if (mn > mx) { mn = 0; mx = 0; }  // no live point
      l[a] = axis_coord(__uint_as_float(mn), st.cand_inv[k][a]) >> kBrickShift;
      u[a] = axis_coord(__uint_as_float(mx), st.cand_inv[k][a]) >> kBrickShift;
    }
    const uint64_t dx = u[0] - l[0] + 1, dy = u[1] - l[1] + 1, dz = u[2] - l[2] + 1;
    const uint64_t vol = dx * dy * dz;
    sh.box[k][0] = l[0];
    sh.box[k][1] = l[1];
    sh.box[k][2] = l[2];
    sh.box[k][3] = static_cast<uint32_t>(dx);
    sh.box[k][4] = static_cast<uint32_t>(dy);
    sh.box[k][5] = vol <= static_cast<uint64_t>(kCandWords) ? static_cast<uint32_t>(vol) : 0u;
    sh.boxm[k][0] = div_magic(static_cast<uint32_t>(dx));
    sh.boxm[k][1] = div_magic(static_cast<uint32_t>(dy));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nu = 0;
    for (int ci = cb; ci < ce; ++ci) {
      sh.unit_c[nu] = ci;
      sh.unit_h[nu++] = 0;
      if (sh.box[ci][5] > static_cast<uint32_t>(kBrickCap)) {
        sh.unit_c[nu] = ci;
        sh.unit_h[nu++] = 1;
      }
    }
    sh.nu = nu;
  }
  for (int ci = cb; ci < ce; ++ci) {
    const float ix = st.cand_inv[ci][0], iy = st.cand_inv[ci][1], iz = st.cand_inv[ci][2];
    uint64_t* tv = lvals + (ci - lb) * kCandWords;
    if (sh.box[ci][5] != 0) {
      const uint32_t bl0 = sh.box[ci][0], bl1 = sh.box[ci][1], bl2 = sh.box[ci][2];
      const uint32_t bdx = sh.box[ci][3], bdy = sh.box[ci][4];
      uint32_t cur = 0xFFFFFFFFu;
      uint64_t cb = 0ull;
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if (!(live & (1u << k))) continue;
        const uint32_t gx = axis_coord(pt[k].x, ix);
        const uint32_t gy = axis_coord(pt[k].y, iy);
        const uint32_t gz = axis_coord(pt[k].z, iz);
        const uint32_t loc = ((gx >> kBrickShift) - bl0) +
                             bdx * (((gy >> kBrickShift) - bl1) + bdy * ((gz >> kBrickShift) - bl2));
        const uint64_t bit = brick_bit(gx, gy, gz);
        if (loc == cur) {
          cb |= bit;
        } else {
          if (cur != 0xFFFFFFFFu)
            __hip_atomic_fetch_or(&tv[cur], cb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          cur = loc;
          cb = bit;
        }
      }
      if (cur != 0xFFFFFFFFu)
        __hip_atomic_fetch_or(&tv[cur], cb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      continue;
    }
    // sparse tile: the brick ids go through three direct-mapped LDS levels (keys in
    // lkeys, bits in lvals). A run stores its key in its level-1 slot and, after a
    // barrier, ORs its bits in if the slot holds its key (the runs of one key all
    // do); the others try a level-2 slot (other bits of the hash) the same way, then
    // level 3, and the few left go straight to the global table. A key sits in at most
    // one slot, and no run probes, so there are no chains of LDS round trips. The
    // thread's runs are formed first (run q ends before point q).
    const int dense = st.cand_dense[ci];
    const uint64_t nbx = st.cand_nb[ci][0], nby = st.cand_nb[ci][1];
    uint64_t* tk = tv + kBrickCap;  // keys + 1
    uint64_t rk[kPerThread + 1], rb[kPerThread + 1];
    uint32_t pend = 0;
    {
      uint64_t cur = kEmptyKey, cb = 0ull;
#pragma unroll
      for (int k = 0; k <= kPerThread; ++k) {
        uint64_t key = kEmptyKey, bit = 0ull;
        if (k < kPerThread) {
          if (!(live & (1u << k))) continue;
          const uint32_t gx = axis_coord(pt[k].x, ix);
          const uint32_t gy = axis_coord(pt[k].y, iy);
          const uint32_t gz = axis_coord(pt[k].z, iz);
          key = dense ? (static_cast<uint64_t>(gx >> kBrickShift) +
                         nbx * (static_cast<uint64_t>(gy >> kBrickShift) + nby * (gz >> kBrickShift)))
                      : brick_key(gx, gy, gz);
          bit = brick_bit(gx, gy, gz);
          if (key == cur) {
            cb |= bit;
            continue;
          }
        }
        if (cur != kEmptyKey) {
          rk[k] = cur;
          rb[k] = cb;
          pend |= 1u << k;
        }
        cur = key;
        cb = bit;
      }
    }
    // levels: slots [0, 512) on hash bits 0-8, [512, 768) on bits 12-19, [768, 1024)
    // on bits 22-29
    static_assert(kBrickCap == 1024, "direct-mapped levels of the LDS brick table");
    uint32_t hh[kPerThread + 1];
#pragma unroll
    for (int q = 0; q <= kPerThread; ++q) hh[q] = ((pend >> q) & 1u) ? table_hash(rk[q]) : 0u;
#pragma unroll
    for (int lv = 0; lv < 3; ++lv) {
      const uint32_t base = lv == 0 ? 0u : (lv == 1 ? 512u : 768u);
      const uint32_t mask = lv == 0 ? 511u : 255u;
      const int shift = lv == 0 ? 0 : (lv == 1 ? 12 : 22);
#pragma unroll
      for (int q = 0; q <= kPerThread; ++q)
        if ((pend >> q) & 1u)
          __hip_atomic_store(&tk[base + ((hh[q] >> shift) & mask)], rk[q] + 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
      __syncthreads();
#pragma unroll
      for (int q = 0; q <= kPerThread; ++q) {
        const uint32_t e = base + ((hh[q] >> shift) & mask);
        if (((pend >> q) & 1u) &&
            __hip_atomic_load(&tk[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == rk[q] + 1ull) {
          __hip_atomic_fetch_or(&tv[e], rb[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          pend &= ~(1u << q);
        }
      }
    }
    if (pend) {
      uint32_t f = 0;
#pragma unroll
      for (int q = 0; q <= kPerThread; ++q) {
        if (!((pend >> q) & 1u)) continue;
        f += dense ? dense_or(ctab_masks(w, set, ci), static_cast<uint32_t>(rk[q]), rb[q],
                              claims(w, set, ci, tile), &sh.ncl[ci])
                   : global_or(ctab_keys(w, set, ci), ctab_masks(w, set, ci), w.cmask, rk[q], rb[q],
                               claims(w, set, ci, tile), &sh.ncl[ci]);
      }
      if (f) atomicAdd(&sh.fresh[ci], f);
    }
  }
  __syncthreads();
  mid();
  // One global update per distinct brick of the tile, LDS entries emptied as read.
  // The flush goes by units of kBrickCap entries (a candidate, or each half of a box
  // above kBrickCap bricks); thread t owns entries t + j*kThreads (j < 4) of a unit, and
  // the updates of up to three units are issued together so that their round trips overlap. A hot
  // table (a brick grid of at most kHotCap words, shared by very many tiles) is first
  // ORed into the tile's replica (one of kReps, so a word sees a 1/kReps share of the
  // tiles) and only the bits new to the replica go on to the table; every bit still
  // reaches the table, so the fresh count stays exact.
  static_assert(kBrickCap == 4 * kThreads, "four flush entries per thread");
  constexpr int kGrp = 3;
  const int rep = tile & (kReps - 1);
  const int nu = sh.nu;
  for (int u0 = 0; u0 < nu; u0 += kGrp) {
    uint32_t slot[4 * kGrp];
    uint64_t bits[4 * kGrp], hkey[4 * kGrp];
    uint32_t valid = 0, hot = 0, hm = 0;
    uint32_t f[kGrp] = {};
    int uc[kGrp];
#pragma unroll
    for (int k = 0; k < kGrp; ++k) uc[k] = u0 + k < nu ? sh.unit_c[u0 + k] : cb;
#pragma unroll
    for (int q = 0; q < 4 * kGrp; ++q) {
      const int u = u0 + q / 4;
      slot[q] = 0;
      bits[q] = 0ull;
      if (u >= nu) continue;
      const int ci = uc[q / 4];
      const int le = sh.unit_h[u] * kBrickCap + (q % 4) * kThreads + threadIdx.x;
      uint64_t* R = lvals + (ci - lb) * kCandWords;
      const uint32_t vol = sh.box[ci][5];
      const int dense = st.cand_dense[ci];
      uint64_t key, b;
      if (vol) {
        if (le >= static_cast<int>(vol)) continue;
        b = R[le];
        if (!b) continue;
        R[le] = 0ull;
        const uint32_t bdx = sh.box[ci][3], bdy = sh.box[ci][4];
        const uint32_t t2 = box_div(static_cast<uint32_t>(le), sh.boxm[ci][0]);
        const uint32_t t3 = box_div(t2, sh.boxm[ci][1]);
        const uint32_t bx = sh.box[ci][0] + (static_cast<uint32_t>(le) - t2 * bdx);
        const uint32_t by = sh.box[ci][1] + (t2 - t3 * bdy);
        const uint32_t bz = sh.box[ci][2] + t3;
        key = dense ? (bx + static_cast<uint64_t>(st.cand_nb[ci][0]) *
                                (by + static_cast<uint64_t>(st.cand_nb[ci][1]) * bz))
                    : (static_cast<uint64_t>(bx) | (static_cast<uint64_t>(by) << kBrickCoordBits) |
                       (static_cast<uint64_t>(bz) << (2 * kBrickCoordBits)));
      } else {
        const uint64_t k1 = R[kBrickCap + le];
        if (k1 == 0ull) continue;
        key = k1 - 1ull;
        b = R[le];
        R[kBrickCap + le] = 0ull;
        R[le] = 0ull;
      }
      if (!dense) {  // hashed table: the slot is found below
        slot[q] = table_hash(key) & w.cmask;
        hkey[q] = key;
        bits[q] = b;
        hm |= 1u << q;
        continue;
      }
      slot[q] = static_cast<uint32_t>(key);
      bits[q] = b;
      valid |= 1u << q;
      if (st.cand_hot[ci]) hot |= 1u << q;
    }
    // hashed tables: the entries probe in lockstep, one CAS round trip per probe step for
    // all of them (the CAS both looks the slot up and claims it when empty; a claim is
    // recorded), then join the table updates below (tables hold at most half their
    // slots in keys, so every probe ends)
    const uint32_t hashed = hm;
    while (hm) {
      unsigned long long kk[4 * kGrp];
#pragma unroll
      for (int q = 0; q < 4 * kGrp; ++q)
        kk[q] = ((hm >> q) & 1u) ? atomicCAS(ctab_keys(w, set, uc[q / 4]) + slot[q], kEmptyKey,
                                             static_cast<unsigned long long>(hkey[q]))
                                 : 0ull;
#pragma unroll
      for (int q = 0; q < 4 * kGrp; ++q) {
        if (!((hm >> q) & 1u)) continue;
        if (kk[q] == kEmptyKey)
          st_agent(claims(w, set, uc[q / 4], tile) + atomicAdd(&sh.ncl[uc[q / 4]], 1),
                   static_cast<int32_t>(slot[q]));
        if (kk[q] == kEmptyKey || kk[q] == hkey[q]) {
          hm &= ~(1u << q);
          valid |= 1u << q;
        } else {
          slot[q] = (slot[q] + 1) & w.cmask;
        }
      }
    }
    // hot words: the tile's replica first
    uint64_t old[4 * kGrp];
#pragma unroll
    for (int q = 0; q < 4 * kGrp; ++q)
      old[q] = ((hot >> q) & 1u)
                   ? atomicOr(hrep_of(w, set, uc[q / 4], rep) + slot[q],
                              static_cast<unsigned long long>(bits[q]))
                   : 0ull;
#pragma unroll
    for (int q = 0; q < 4 * kGrp; ++q) {
      if (!((hot >> q) & 1u)) continue;
      if (old[q] == 0ull)
        st_agent(claims(w, set, uc[q / 4], tile) + atomicAdd(&sh.ncl[uc[q / 4]], 1),
                 static_cast<int32_t>(-1 - (rep * kHotCap + static_cast<int32_t>(slot[q]))));
      bits[q] &= ~old[q];
      if (!bits[q]) valid &= ~(1u << q);
    }
    // the tables
#pragma unroll
    for (int q = 0; q < 4 * kGrp; ++q)
      old[q] = ((valid >> q) & 1u)
                   ? atomicOr(ctab_masks(w, set, uc[q / 4]) + slot[q],
                              static_cast<unsigned long long>(bits[q]))
                   : ~0ull;
#pragma unroll
    for (int q = 0; q < 4 * kGrp; ++q) {
      if (!((valid >> q) & 1u)) continue;
      f[q / 4] += static_cast<uint32_t>(__popcll(bits[q] & ~old[q]));
      if (old[q] == 0ull && !((hashed >> q) & 1u))  // (a hashed slot was recorded when claimed)
        st_agent(claims(w, set, uc[q / 4], tile) + atomicAdd(&sh.ncl[uc[q / 4]], 1),
                 static_cast<int32_t>(slot[q]));
    }
#pragma unroll
    for (int k = 0; k < kGrp; ++k)
      if (f[k]) atomicAdd(&sh.fresh[uc[k]], f[k]);
  }
  __syncthreads();
  if (cb + static_cast<int>(threadIdx.x) < ce)
    st_agent(claim_n(w, set, cb + threadIdx.x, tile), static_cast<int32_t>(sh.ncl[cb + threadIdx.x]));
}

// Block-shared state of the search kernels.
struct SearchShared {
  SState st;
  EvalShared sh;
  uint32_t cnt[kMaxCand];
  int cn[kMaxCand + 1];
  int cloud, pass, tile, go, last;
  int rank, part;  // the ticket's place in its pass, and its candidate (-1: all of them)
};

enum TicketResult : int { kTicketDone = 0, kTicketPublished = 1, kTicketFinished = 2 };

// One ticket of a cloud's search: tile `tile` of pass `p`, whose state S.st holds and
// whose loads are in flight in pt/tg. Clears the tile's claims of the previous pass,
// counts the tile at the pass's candidates and adds the counts; the block that
// completes the pass runs the bisection step and publishes the next pass
// (kTicketPublished; S.st is then that pass's state) or the end of the search
// (kTicketFinished; the controller and report are written for the following kernels).
__device__ __forceinline__ int run_ticket(const Ws& w, const Plan& P, SearchShared& S,
                                          uint64_t* lvals, uint64_t* lkeys,
                                          float4 (&pt)[kPerThread], const uint32_t (&tg)[kPerThread],
                                          int p, int tile, int rank, int ntk, int part) {
  Header* h = w.h;
  SState& st = S.st;
  const int nc = st.nc;
  // this ticket's candidates: all of the pass's, or candidate `part` alone (then the
  // LDS holds one candidate's tables); the previous pass's claims likewise
  const int cb = part < 0 ? 0 : part, ce = part < 0 ? nc : (part < nc ? part + 1 : part);
  const int pb = part < 0 ? 0 : part;
  const int pe = part < 0 ? st.prev_nc : (part < st.prev_nc ? part + 1 : part);
  // The previous pass's claims of this tile are cleared in three steps whose round trips
  // overlap the tile's own work (the two passes use different table sets): the claim
  // counts load with the tile's bounds reduction, the claims (up to kClrReg per thread
  // in registers) with the box setup and LDS phase, and the exchanges are issued
  // before the flush without being waited for (the ticket's final wait covers them).
  const int nk = pe > pb ? pe - pb : 0;
  const int pset = st.prev_set;
  const uint32_t phashed = st.prev_hashed;
  int32_t ccount = 0;
  if (static_cast<int>(threadIdx.x) < nk) ccount = ld_agent(claim_n(w, pset, pb + threadIdx.x, tile));
  if (cb + static_cast<int>(threadIdx.x) < ce) S.sh.fresh[cb + threadIdx.x] = 0;
  uint32_t live = 0;
  if (cb < ce) finish_tile_a(pt, tg, live, S.sh);
  if (static_cast<int>(threadIdx.x) < nk) S.cn[threadIdx.x + 1] = ccount;
  __syncthreads();
  if (cb < ce) finish_tile_b(S.sh);
  if (threadIdx.x == 0) {
    S.cn[0] = 0;
    for (int j = 0; j < nk; ++j) S.cn[j + 1] += S.cn[j];
  }
  __syncthreads();
  const int ctotal = S.cn[nk];
  int32_t cid[kClrReg];
  int ck[kClrReg];
#pragma unroll
  for (int q = 0; q < kClrReg; ++q) {
    const int e = static_cast<int>(threadIdx.x) + q * kThreads;
    ck[q] = -1;
    cid[q] = 0;
    if (e < ctotal) {
      int j = 0;
      while (e >= S.cn[j + 1]) ++j;
      ck[q] = pb + j;
      cid[q] = ld_agent(claims(w, pset, pb + j, tile) + (e - S.cn[j]));
    }
  }
  auto clear_one = [&](int k, int32_t id) {
    if (id >= 0) {
      if ((phashed >> k) & 1u) atomicExch(ctab_keys(w, pset, k) + id, static_cast<unsigned long long>(kEmptyKey));
      atomicExch(ctab_masks(w, pset, k) + id, 0ull);
    } else {
      const int32_t q = -1 - id;
      atomicExch(hrep_of(w, pset, k, q / kHotCap) + (q % kHotCap), 0ull);
    }
  };
  auto clear_issue = [&]() {
#pragma unroll
    for (int q = 0; q < kClrReg; ++q)
      if (ck[q] >= 0) clear_one(ck[q], cid[q]);
    for (int e = static_cast<int>(threadIdx.x) + kClrReg * kThreads; e < ctotal; e += kThreads) {
      int j = 0;
      while (e >= S.cn[j + 1]) ++j;
      clear_one(pb + j, ld_agent(claims(w, pset, pb + j, tile) + (e - S.cn[j])));
    }
  };
  if (cb < ce)
    eval_loaded(w, tile, st, S.sh, lvals, lkeys, pt, live, cb, ce, part < 0 ? 0 : part, clear_issue);
  else
    clear_issue();
  __syncthreads();
  if (cb + static_cast<int>(threadIdx.x) < ce && S.sh.fresh[cb + threadIdx.x])
    atomicAdd(&h->sacc[p & 1][cb + threadIdx.x][rank & (kGroups - 1)][0], S.sh.fresh[cb + threadIdx.x]);
  // this tile's clears, table updates and counts are complete before it counts as done
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    // two-level completion count: a pass's tickets of group g = rank % kGroups, then the
    // groups (every pass adds exactly gsize and ngroups)
    const int g = rank & (kGroups - 1);
    const uint32_t gsize = static_cast<uint32_t>((ntk - g + kGroups - 1) / kGroups);
    const uint32_t ngroups = static_cast<uint32_t>(ntk < kGroups ? ntk : kGroups);
    int last = 0;
    const uint32_t d = atomicAdd(&h->sq_dgrp[g][0], 1u);
    if (d % gsize == gsize - 1) {
      const uint32_t e = atomicAdd(&h->sq_done[0], 1u);
      last = (e % ngroups) == ngroups - 1;
    }
    S.last = last;
  }
  __syncthreads();
  if (!S.last) return kTicketDone;
  // ---- last tile of pass p: bisection step, then publish pass p + 1 or the end
  if (threadIdx.x < nc) S.cnt[threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x < nc * kGroups) {
    const uint32_t v = atomicExch(&h->sacc[p & 1][threadIdx.x / kGroups][threadIdx.x % kGroups][0], 0u);
    if (v) atomicAdd(&S.cnt[threadIdx.x / kGroups], v);
  }
  __syncthreads();
  Ctrl* c = &h->ctrl;
  if (threadIdx.x == 0) {
    const Frame fl = h->frame;  // one round trip, then the step's arithmetic waits on nothing
    search_step(&st, S.cnt, P, fl, c->m, c->upper);
  }
  __syncthreads();
  if (st.done) {
    if (threadIdx.x == 0) {
      c->evals = st.evals;
      c->accepted = st.accepted;
      c->done = 1;
      c->set = st.set;
      c->pend_set = st.prev_set;
      c->pend_nc = st.prev_nc;
      c->pend_hashed = st.prev_hashed;
      set_final(c, st.s_final, P, h->frame);
      c->c_final = st.c_final;
      set_window(c, P.win_sigma);
      const int Lc = c->layer;
      h->info.evals[Lc] = st.evals;
      h->info.accepted[Lc] = st.accepted;
      h->info.s[Lc] = st.s_final;
      atomicExch(&h->sq_fin[0], 1u);
    }
    __syncthreads();
    return kTicketFinished;
  }
  if (threadIdx.x < kPubWords)
    st_agent(&h->pub[threadIdx.x], reinterpret_cast<const uint32_t*>(&st)[threadIdx.x]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) atomicExch(&h->sq_gen[0], static_cast<uint32_t>(p + 1));
  return kTicketPublished;
}

// Wait (thread 0) until pass p of the cloud behind `h` is published. 1: go on; 0: the
// cloud's search has ended (drop the ticket); -1: a wait gave up (error flag raised).
// (Measured: sleeping longer between polls makes the launch slower, since a publication
// is noticed late.)
__device__ int wait_pass(Header* h, int p, uint32_t* err) {
  uint32_t spins = 0;
  const uint32_t limit = g_search_spin_limit;
  while (ld_agent(&h->sq_gen[0]) < static_cast<uint32_t>(p)) {
    if (ld_agent(&h->sq_fin[0])) return 0;
    if (ld_agent(&h->sq_err[0]) || (err && ld_agent(err))) return -1;
    if (++spins > limit) {
      atomicOr(&h->sq_err[0], 1u);
      if (err) atomicOr(err, 1u);
      return -1;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return 1;
}

__device__ __forceinline__ void search_lds_init(uint64_t* lds, int depth, uint64_t*& lvals,
                                                uint64_t*& lkeys) {
  const int ncap = depth;
  lvals = lds;
  lkeys = nullptr;  // (keys live in each candidate's words)
  for (int e = threadIdx.x; e < ncap * kCandWords; e += kThreads) lvals[e] = 0ull;
}

// A wait gave up: tables may hold claims nobody cleared, so the workspace needs
// hav_workspace_init again.
__device__ void mark_search_failed(Header* h) {
  h->frame.status = HAV_ERR_HIP;
  h->info.status = HAV_ERR_HIP;
  h->magic = 0;
}

// The adaptive voxel search of a layer (Sec. 3.3) in one launch. The passes' work is
// a queue of tickets: ticket t is tile t % ntile of pass t / ntile. A block takes a
// ticket, waits until that pass's candidates are published and runs it (run_ticket).
// A block only ever waits for tiles that running blocks hold, so the launch needs no
// co-resident grid and no kernel boundary per pass. (The one ticket counter also
// staggers the blocks' starts a little, which spreads their bursts of table atomics:
// measured, static first tickets per block made the launch slower, not faster.)
__global__ void __launch_bounds__(kThreads) k_search(One src, int L, int split) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKTile, bx, gx);
  const Ws& w = cd.w;
  const Plan& P = cd.P;
  Header* h = w.h;
  if (cd.P.identity || L >= cd.P.nlayers) return;
  extern __shared__ uint64_t lds[];
  __shared__ SearchShared S;
  __shared__ uint32_t s_first;
  const uint32_t pub0 = threadIdx.x < kPubWords ? ld_agent(&h->pub_first[L][threadIdx.x]) : 0u;
  if (threadIdx.x == 0) {
    const int status = h->frame.status;
    const int done = h->ctrl.done;
    s_first = atomicAdd(&h->sq_ticket[0], 1u);
    S.go = status == HAV_OK && !done ? 1 : 0;
  }
  uint64_t *lvals, *lkeys;
  search_lds_init(lds, split > 1 ? 1 : P.depth, lvals, lkeys);
  __syncthreads();
  if (!S.go) return;
  const int ntile = w.ntile;
  const int ntk = ntile * split;  // tickets of a pass
  int cur = -1;  // pass whose state S.st holds
  bool first = true;
  float4 pt[kPerThread];
  while (true) {
    __syncthreads();  // every thread has read the previous ticket's shared fields
    if (threadIdx.x == 0) {
      const uint32_t t = first ? s_first : atomicAdd(&h->sq_ticket[0], 1u);
      const int p = static_cast<int>(t / static_cast<uint32_t>(ntk));
      const int r = static_cast<int>(t - static_cast<uint32_t>(p) * static_cast<uint32_t>(ntk));
      S.pass = p;
      S.rank = r;
      S.tile = r % ntile;
      S.part = split > 1 ? r / ntile : -1;
    }
    __syncthreads();
    const int p = S.pass, tile = S.tile, rank = S.rank, part = S.part;
    if (p >= P.t_max) break;  // every pass makes at least one evaluation
    uint32_t tg[kPerThread];
    issue_tile(w, tile, pt, tg);  // in flight during the wait and the state and claim reads
    if (first && p == 0) {
      if (threadIdx.x < kPubWords) reinterpret_cast<uint32_t*>(&S.st)[threadIdx.x] = pub0;
      __syncthreads();
      cur = 0;
    } else if (p != cur) {
      if (threadIdx.x == 0) S.go = wait_pass(h, p, nullptr);
      __syncthreads();
      if (S.go <= 0) break;
      if (threadIdx.x < kPubWords)
        reinterpret_cast<uint32_t*>(&S.st)[threadIdx.x] = ld_agent(&h->pub[threadIdx.x]);
      __syncthreads();
      cur = p;
    }
    first = false;
    const int r = run_ticket(w, P, S, lvals, lkeys, pt, tg, p, tile, rank, ntk, part);
    if (r == kTicketFinished) break;
    if (r == kTicketPublished) cur = p + 1;
  }
  if (threadIdx.x == 0 && ld_agent(&h->sq_err[0])) mark_search_failed(h);
}

// ----------------------------------------------------------------------------- select

// Packed voxel coordinate of a selection-table slot (dense: decoded from the slot).
__device__ __forceinline__ uint64_t sel_key(const Ws& w, const Ctrl* c, int32_t slot) {
  if (!c->sel_dense) return w.skeys[slot];
  const uint32_t nx = c->sel_nv[0], ny = c->sel_nv[1];
  const uint32_t u = static_cast<uint32_t>(slot);
  const uint32_t gx = u % nx, t = u / nx;
  return pack_key(gx, t % ny, t / ny);
}

// LDS voxel map insert of one (key, value) run: linear probing from the key's hash slot
// (an empty slot is claimed by CAS); the slot's value takes the minimum.
__device__ __forceinline__ bool lds_try_min(uint64_t* tk, uint64_t* tv, uint64_t key, uint64_t v) {
  uint32_t hs = table_hash(key) & (kLdsCap - 1);
  for (int pr = 0; pr < kLdsCap; ++pr) {
    uint64_t kk = tk[hs];
    if (kk == kEmptyKey) kk = lds_cas(&tk[hs], kEmptyKey, key);
    if (kk == kEmptyKey || kk == key) {
      __hip_atomic_fetch_min(&tv[hs], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return true;
    }
    hs = (hs + 1) & (kLdsCap - 1);
  }
  return false;  // unreachable: the map holds twice the tile's points
}

// The digit whose bucket holds rank (0-based) in a 256-bin histogram, and the rank
// inside that bucket: one bin per thread and a block scan. Every thread gets both.
__device__ void find_digit(const uint32_t* hist, uint32_t rank, int* digit, uint32_t* rest) {
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ int s_d;
  __shared__ uint32_t s_r;
  const uint32_t v = threadIdx.x < 256 ? hist[threadIdx.x] : 0u;
  if (threadIdx.x == 0) {
    s_d = 255;
    s_r = 0;
  }
  uint32_t ex;
  block_exclusive_scan<kThreads>(v, &ex, s_tmp);
  if (threadIdx.x < 256 && rank >= ex && rank < ex + v) {
    s_d = threadIdx.x;
    s_r = rank - ex;
  }
  __syncthreads();
  *digit = s_d;
  *rest = s_r;
  __syncthreads();
}

// Centre-closest point of every occupied voxel at the chosen size (Sec. 3.2): the
// tile's minimum of (bits(d^2) << 32 | index) per voxel in LDS (a dense box array
// when the tile's voxels fit one), then one global atomicMin per voxel of the tile.
template <class Src>
__global__ void __launch_bounds__(kThreads) k_select(Src src, int L) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKTile, bx, gx);
  if (!layer_due(cd, L)) return;
  const Ws& w = cd.w;
  Header* h = w.h;
  Ctrl* c = &h->ctrl;
  const int tile = bx;
  extern __shared__ uint64_t lds[];
  uint64_t* lvals = lds;
  uint64_t* lkeys = lds + kLdsCap;
  __shared__ int s_ncl;
  __shared__ uint32_t s_red[kThreads / 64][6];
  __shared__ uint32_t s_box[6];
  __shared__ uint32_t s_below, s_inwin;
  const float vx = c->v_final[0], vy = c->v_final[1], vz = c->v_final[2];
  const float ix = c->inv_final[0], iy = c->inv_final[1], iz = c->inv_final[2];
  const int dense = c->sel_dense;
  const uint64_t nx = c->sel_nv[0], ny = c->sel_nv[1];
  const bool rnd = cd.P.select == HAV_SELECT_RANDOM;
  const uint64_t seed = cd.P.seed;
  for (int e = threadIdx.x; e < kLdsCap; e += kThreads) {
    lkeys[e] = kEmptyKey;
    lvals[e] = ~0ull;
  }
  if (threadIdx.x == 0) {
    s_ncl = 0;
    s_below = 0;
    s_inwin = 0;
  }
  // trim window test of a voxel this tile claimed first (every voxel has one such tile)
  const int win = c->win;
  const uint64_t blo = c->blo, bhi = c->bhi;
  const int wshift = c->wshift;
  uint32_t* whist = h->whist;
  auto wcount = [&](uint64_t pk) {
    const uint64_t p = voxel_priority(pk);
    if (p < blo) {
      atomicAdd(&s_below, 1u);
    } else if (p <= bhi) {
      atomicAdd(&s_inwin, 1u);
      atomicAdd(&whist[(p - blo) >> wshift], 1u);
    }
  };
  auto unpack = [&](uint64_t key) -> uint64_t {
    if (!dense) return key;
    const uint32_t u = static_cast<uint32_t>(key);
    const uint32_t t = u / static_cast<uint32_t>(nx);
    return pack_key(u % static_cast<uint32_t>(nx), t % static_cast<uint32_t>(ny), t / static_cast<uint32_t>(ny));
  };
  const int64_t base = static_cast<int64_t>(tile) * kTile + threadIdx.x;
  float4 pt[kPerThread];
  uint32_t live = 0;
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  uint32_t tg[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {  // tags and points in one round trip
    const int64_t S = base + k * kThreads;
    tg[k] = w.tag_s[S];
    pt[k] = w.pts[S];
  }
  // the search's last pass's claims in this tile, cleared while the tile loads are in
  // flight (the search tables are not the selection's)
  clear_pending(w, c, tile);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const bool ok = tg[k] == 0;
    if (!ok) pt[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok) {
      live |= 1u << k;
      const uint32_t bx = __float_as_uint(pt[k].x), by = __float_as_uint(pt[k].y),
                     bz = __float_as_uint(pt[k].z);
      lo[0] = min(lo[0], bx); lo[1] = min(lo[1], by); lo[2] = min(lo[2], bz);
      hi[0] = max(hi[0], bx); hi[1] = max(hi[1], by); hi[2] = max(hi[2], bz);
    }
  }
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t r[6];
    for (int a = 0; a < 3; ++a) {
      r[a] = __ockl_wfred_min_u32(lo[a]);
      r[3 + a] = __ockl_wfred_max_u32(hi[a]);
    }
    if (lane == 0)
      for (int q = 0; q < 6; ++q) s_red[wv][q] = r[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float inv[3] = {ix, iy, iz};
    uint32_t l[3], u[3];
    for (int a = 0; a < 3; ++a) {
      uint32_t mn = 0xFFFFFFFFu, mx = 0u;
      for (int q = 0; q < kThreads / 64; ++q) {
        mn = min(mn, s_red[q][a]);
        mx = max(mx, s_red[q][3 + a]);
      }
      if (mn > mx) { mn = 0; mx = 0; }
      l[a] = axis_coord(__uint_as_float(mn), inv[a]);
      u[a] = axis_coord(__uint_as_float(mx), inv[a]);
    }
    const uint64_t dx = u[0] - l[0] + 1, dy = u[1] - l[1] + 1, dz = u[2] - l[2] + 1;
    const uint64_t vol = dx * dy * dz;
    s_box[0] = l[0];
    s_box[1] = l[1];
    s_box[2] = l[2];
    s_box[3] = static_cast<uint32_t>(dx);
    s_box[4] = static_cast<uint32_t>(dy);
    s_box[5] = vol <= static_cast<uint64_t>(kLdsCap) ? static_cast<uint32_t>(vol) : 0u;
  }
  __syncthreads();
  const uint32_t bl0 = s_box[0], bl1 = s_box[1], bl2 = s_box[2], bdx = s_box[3], bdy = s_box[4];
  const uint32_t vol = s_box[5];
  {
    // runs of equal voxels among the thread's points merge (min) in registers
    uint64_t cur = kEmptyKey, cv = ~0ull;
    for (int k = 0; k <= kPerThread; ++k) {
      uint64_t key = kEmptyKey, val = ~0ull;
      if (k < kPerThread) {
        if (!(live & (1u << k))) continue;
        const float4 p = pt[k];
        const uint32_t gx = axis_coord(p.x, ix), gy = axis_coord(p.y, iy), gz = axis_coord(p.z, iz);
        const uint32_t orig = static_cast<uint32_t>(__float_as_int(p.w));
        uint32_t rank;
        if (rnd) {
          // random member: top half of SplitMix64 output orig + 1 for the seed
          rank = static_cast<uint32_t>(
              voxel_priority(seed + static_cast<uint64_t>(orig) * 0x9E3779B97F4A7C15ull) >> 32);
        } else {
          rank = __float_as_uint(centre_dist2(p.x, p.y, p.z, gx, gy, gz, vx, vy, vz));
        }
        val = (static_cast<uint64_t>(rank) << 32) | orig;
        key = vol ? static_cast<uint64_t>((gx - bl0) + bdx * ((gy - bl1) + bdy * (gz - bl2)))
                  : (dense ? gx + nx * (gy + ny * gz) : pack_key(gx, gy, gz));
        if (key == cur) {
          cv = val < cv ? val : cv;
          continue;
        }
      }
      if (cur != kEmptyKey) {
        if (vol)
          __hip_atomic_fetch_min(&lvals[cur], cv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
          lds_try_min(lkeys, lvals, cur, cv);
      }
      cur = key;
      cv = val;
    }
  }
  __syncthreads();
  int32_t* list = w.scl + static_cast<size_t>(tile) * kTile;
  // The occupied map entries (at most kTile: each holds a point) move to the front of
  // the map with their voxel keys, so that the table updates below take one round.
  uint32_t tot = 0;
  {
    __shared__ uint32_t s_cmp[kThreads / 64];
    constexpr int kSP = kLdsCap / kThreads;
    uint64_t ck[kSP], cv[kSP];
    uint32_t occ = 0;
#pragma unroll
    for (int j = 0; j < kSP; ++j) {
      const int e = j * kThreads + static_cast<int>(threadIdx.x);
      cv[j] = lvals[e];
      ck[j] = 0ull;
      if (cv[j] == ~0ull || (vol && e >= static_cast<int>(vol))) continue;
      if (vol) {
        const uint32_t gx = bl0 + static_cast<uint32_t>(e) % bdx;
        const uint32_t t2 = static_cast<uint32_t>(e) / bdx;
        const uint32_t gy = bl1 + t2 % bdy, gz = bl2 + t2 / bdy;
        ck[j] = dense ? gx + nx * (gy + ny * gz) : pack_key(gx, gy, gz);
      } else {
        ck[j] = lkeys[e];
      }
      occ |= 1u << j;
    }
    uint32_t ex;
    tot = block_exclusive_scan<kThreads>(static_cast<uint32_t>(__popc(occ)), &ex, s_cmp);
    // (every thread read its entries before the scan's barrier)
#pragma unroll
    for (int j = 0; j < kSP; ++j) {
      if (!((occ >> j) & 1u)) continue;
      const uint32_t pos = ex + static_cast<uint32_t>(__popc(occ & ((1u << j) - 1u)));
      lkeys[pos] = ck[j];
      lvals[pos] = cv[j];
    }
    __syncthreads();
  }
  // thread t owns entries t + j*kThreads; a dense table's minima are issued together, so
  // that their round trips overlap (the atomic's old value says whether this tile is the
  // voxel's first, which then records the slot)
  constexpr int kQ = kTile / kThreads;
  const int ntot = static_cast<int>(tot);
  for (int e0 = 0; e0 < ntot; e0 += kQ * kThreads) {
    uint64_t key[kQ], val[kQ];
    uint32_t has = 0;
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      const int e = e0 + j * kThreads + static_cast<int>(threadIdx.x);
      key[j] = 0ull;
      val[j] = ~0ull;
      if (e >= ntot) continue;
      key[j] = lkeys[e];
      val[j] = lvals[e];
      has |= 1u << j;
    }
    if (!has) continue;
    if (!dense) {
      // hashed table: the entries probe in lockstep, one CAS round trip per probe step
      // for all of them (the CAS both looks the slot up and, when empty, claims the voxel)
      uint32_t sl[kQ];
      uint32_t pend = has;
#pragma unroll
      for (int j = 0; j < kQ; ++j) sl[j] = ((has >> j) & 1u) ? table_hash(key[j]) & w.cmask : 0u;
      while (pend) {
        unsigned long long kk[kQ];
#pragma unroll
        for (int j = 0; j < kQ; ++j)
          kk[j] = ((pend >> j) & 1u)
                      ? atomicCAS(&w.skeys[sl[j]], kEmptyKey, static_cast<unsigned long long>(key[j]))
                      : 0ull;
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
          if (!((pend >> j) & 1u) || kk[j] != kEmptyKey) continue;
          list[atomicAdd(&s_ncl, 1)] = static_cast<int32_t>(sl[j]);
          if (win) wcount(key[j]);
          kk[j] = key[j];
        }
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
          if (!((pend >> j) & 1u)) continue;
          if (kk[j] == key[j]) {
            atomicMin(&w.svals[sl[j]], static_cast<unsigned long long>(val[j]));
            pend &= ~(1u << j);
          } else {
            sl[j] = (sl[j] + 1) & w.cmask;
          }
        }
      }
      continue;
    }
    uint64_t old[kQ];
#pragma unroll
    for (int j = 0; j < kQ; ++j)
      old[j] = ((has >> j) & 1u) ? atomicMin(&w.svals[static_cast<uint32_t>(key[j])],
                                             static_cast<unsigned long long>(val[j]))
                                 : 0ull;
#pragma unroll
    for (int j = 0; j < kQ; ++j) {
      if (((has >> j) & 1u) && old[j] == ~0ull) {
        list[atomicAdd(&s_ncl, 1)] = static_cast<int32_t>(key[j]);
        if (win) wcount(unpack(key[j]));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = tile & (kGroups - 1);
    w.scn[tile] = s_ncl;
    if (s_ncl) atomicAdd(&h->acc[0][g][0], static_cast<uint32_t>(s_ncl));
    if (s_below) atomicAdd(&h->acc[1][g][0], s_below);
    if (s_inwin) atomicAdd(&h->acc[2][g][0], s_inwin);
  }
  if (!arrive_last(h, bx, gx)) return;
  __shared__ uint32_t s_sum[3];
  __shared__ int s_mode;
  __shared__ uint32_t s_rank, s_bin, s_brank, s_top;
  __shared__ uint32_t s_tmp2[kThreads / 64];
  if (threadIdx.x < 3) s_sum[threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x < 3 * kGroups) {
    const uint32_t v = take(&h->acc[threadIdx.x / kGroups][threadIdx.x % kGroups][0]);
    if (v) atomicAdd(&s_sum[threadIdx.x / kGroups], v);
  }
  // the window's priority histogram, read and emptied (thread t: bins 4t .. 4t+3)
  constexpr int kWB = kWinBins / kThreads;
  static_assert(kWinBins % kThreads == 0, "window bins per thread");
  uint32_t hv[kWB];
#pragma unroll
  for (int j = 0; j < kWB; ++j) hv[j] = win ? ld_agent(&whist[threadIdx.x * kWB + j]) : 0u;
  // (emptied with plain stores: the next writers are a later launch's)
  if (win)
#pragma unroll
    for (int j = 0; j < kWB; ++j) whist[threadIdx.x * kWB + j] = 0u;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nvox = s_sum[0], below = s_sum[1], inwin = s_sum[2];
    c->pend_nc = 0;
    c->ncand = nvox;
    c->trim = nvox > c->m ? 1 : 0;
    c->need = nvox < c->m ? c->m - nvox : 0u;
    c->prefix = 0;
    c->rank = c->m - 1;
    c->rounds_done = 0;
    c->trim_mode = 0;
    if (c->trim && !cd.P.fixed) {
      // the window holds the threshold iff fewer than m voxels lie below it and at
      // least m lie below or inside it
      if (win && nvox == c->c_final && below < c->m && c->m <= below + inwin) {
        c->trim_mode = 1;
        c->rank = c->m - 1 - below;
      } else {
        c->trim_mode = 2;
      }
    }
    s_mode = c->trim_mode;
    s_rank = c->rank;
    s_bin = 0;
    s_brank = 0;
    s_top = 0;
    const int Lc = c->layer;
    h->info.count[Lc] = static_cast<int32_t>(nvox);
    h->info.trimmed[Lc] = nvox > c->m ? static_cast<int32_t>(nvox - c->m) : 0;
    h->info.padded[Lc] = static_cast<int32_t>(c->need);
    h->info.s[Lc] = c->s_final;
  }
  __syncthreads();
  if (s_mode != 1) return;
  // the bin of the window holding the threshold (the rank-th smallest in-window
  // priority): the bucket narrows to that bin, and the rank to the rank inside it
  uint32_t t = 0;
#pragma unroll
  for (int j = 0; j < kWB; ++j) t += hv[j];
  uint32_t ex;
  block_exclusive_scan<kThreads>(t, &ex, s_tmp2);
  const uint32_t rank = s_rank;
  if (rank >= ex && rank < ex + t) {
    uint32_t e = ex;
#pragma unroll
    for (int j = 0; j < kWB; ++j) {
      if (rank >= e && rank < e + hv[j]) {
        s_bin = threadIdx.x * kWB + j;
        s_brank = rank - e;
        s_top = rank - e + 1 == hv[j] ? 1u : 0u;
      }
      e += hv[j];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t lo_b = blo + (static_cast<uint64_t>(s_bin) << wshift);
    const uint64_t span = (wshift >= 64 ? ~0ull : ((1ull << wshift) - 1ull));
    c->blo = lo_b;
    c->bhi = (bhi - lo_b > span) ? lo_b + span : bhi;
    c->rank = s_brank;
    if (s_top) c->trim_mode = 3;  // the bin's members all stay: nothing to settle
  }
}

// ----------------------------------------------------------------------------- trim

// One radix round of the trim (keep the m voxels of smallest priority): histogram of
// the next 8 priority bits of the voxels still in the bucket, then the last block
// fixes the digit holding the rank.
template <class Src>
__global__ void __launch_bounds__(kThreads) k_trim_hist(Src src, int L, int round) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKTile, bx, gx);
  if (!layer_due(cd, L) || round >= cd.P.rounds[L]) return;
  const Ws& w = cd.w;
  Header* h = w.h;
  Ctrl* c = &h->ctrl;
  if (!c->trim || c->trim_mode != 0) return;
  __shared__ uint32_t lh[kTrimBins];
  for (int i = threadIdx.x; i < kTrimBins; i += kThreads) lh[i] = 0;
  __syncthreads();
  const int tile = bx;
  const int n = w.scn[tile];
  const int32_t* list = w.scl + static_cast<size_t>(tile) * kTile;
  const int dshift = 64 - kTrimBits * (round + 1);
  const uint64_t pref = c->prefix;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const uint64_t p = voxel_priority(sel_key(w, c, list[i]));
    if (round > 0 && (p >> (dshift + kTrimBits)) != (pref >> (dshift + kTrimBits))) continue;
    atomicAdd(&lh[(p >> dshift) & (kTrimBins - 1)], 1u);
  }
  __syncthreads();
  const int g = tile & (kGroups - 1);
  for (int i = threadIdx.x; i < kTrimBins; i += kThreads)
    if (lh[i]) atomicAdd(&h->hist[g][i], lh[i]);
  if (!arrive_last(h, bx, gx)) return;
  // last block: the total histogram (emptied as read), then the digit holding rank
  for (int i = threadIdx.x; i < kTrimBins; i += kThreads) {
    uint32_t v[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) v[q] = take(&h->hist[q][i]);  // all in flight at once
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < kGroups; ++q) t += v[q];
    lh[i] = t;
  }
  __syncthreads();
  int b;
  uint32_t rest;
  find_digit(lh, c->rank, &b, &rest);
  if (threadIdx.x == 0) {
    c->rank = rest;
    c->prefix |= static_cast<uint64_t>(b) << dshift;
    c->rounds_done = round + 1;
  }
}

// ----------------------------------------------------------------------------- points modes

// Fixed-point scale of the voxel mean along each axis: q = floor(r * 2^32 / H) with H
// the smallest power of two >= the cloud's extent (r <= H, so q <= 2^32 and a sum over
// 2^30 points fits 64 bits); sums are exact, so the mean does not depend on the order
// the points arrive in.
__device__ __forceinline__ float mean_extent(float ext) {
  const float e = ext < 0x1p-64f ? 0x1p-64f : ext;
  const uint32_t bits = __float_as_uint(e);
  return (bits & 0x7FFFFFu) ? __uint_as_float((bits & 0x7F800000u) + 0x00800000u) : e;
}

// The slot of voxel (gx, gy, gz) in the selection table at the chosen size (it exists:
// the selection inserted every voxel of R); -1 if the probe runs out.
__device__ __forceinline__ int64_t sel_slot(const Ws& w, const Ctrl* c, uint32_t gx, uint32_t gy,
                                            uint32_t gz) {
  if (c->sel_dense)
    return static_cast<int64_t>(gx) + static_cast<int64_t>(c->sel_nv[0]) *
                                          (gy + static_cast<int64_t>(c->sel_nv[1]) * gz);
  const uint64_t key = pack_key(gx, gy, gz);
  uint32_t sl = table_hash(key) & w.cmask;
  for (uint32_t pr = 0; pr <= w.cmask; ++pr) {
    if (w.skeys[sl] == key) return sl;
    sl = (sl + 1) & w.cmask;
  }
  return -1;
}

// Voxel means ("ME" of Table 6): every unsampled point adds its fixed-point
// coordinates and a count to its voxel's slot.
__global__ void __launch_bounds__(kThreads) k_mean(One src, int L) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKTile, bx, gx);
  if (!layer_due(cd, L)) return;
  const Ws& w = cd.w;
  const Ctrl* c = &w.h->ctrl;
  const Frame& fr = w.h->frame;
  float qs[3];
  for (int a = 0; a < 3; ++a) qs[a] = 4294967296.0f / mean_extent(fr.mx[a] - fr.mn[a]);
  const float ix = c->inv_final[0], iy = c->inv_final[1], iz = c->inv_final[2];
  const int64_t base = static_cast<int64_t>(bx) * kTile + threadIdx.x;
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t S = base + k * kThreads;
    if (w.tag_s[S] != 0) continue;
    const float4 p = w.pts[S];
    const int64_t sl = sel_slot(w, c, axis_coord(p.x, ix), axis_coord(p.y, iy), axis_coord(p.z, iz));
    if (sl < 0) continue;
    atomicAdd(&w.msum[3 * sl], static_cast<unsigned long long>(p.x * qs[0]));
    atomicAdd(&w.msum[3 * sl + 1], static_cast<unsigned long long>(p.y * qs[1]));
    atomicAdd(&w.msum[3 * sl + 2], static_cast<unsigned long long>(p.z * qs[2]));
    atomicAdd(&w.mcnt[sl], 1u);
  }
}

// What stands for voxel `key` (selection slot s) whose representative is point orig:
// its centre mn + v (g + 0.5) ("CE" of Table 6) or the mean of its points ("ME"), in
// the cloud's coordinates; the mean's sums are emptied as read.
__device__ void stand_in(const Ws& w, const Ctrl* c, const Frame& fr, int32_t s, uint64_t key,
                         int32_t orig) {
  float o[3];
  if (w.pmode == 1) {
    for (int a = 0; a < 3; ++a) {
      const float ga = static_cast<float>((key >> (kKeyBits * a)) & ((1ull << kKeyBits) - 1ull));
      o[a] = fr.mn[a] + c->v_final[a] * (ga + 0.5f);
    }
  } else {
    const double n = static_cast<double>(w.mcnt[s]);
    for (int a = 0; a < 3; ++a) {
      const double back = static_cast<double>(mean_extent(fr.mx[a] - fr.mn[a])) / 4294967296.0;
      const double mean = static_cast<double>(w.msum[3 * static_cast<int64_t>(s) + a]) / n;
      o[a] = static_cast<float>(static_cast<double>(fr.mn[a]) + mean * back);
      w.msum[3 * static_cast<int64_t>(s) + a] = 0ull;
    }
    w.mcnt[s] = 0u;
  }
  for (int a = 0; a < 3; ++a) w.pt_out[3 * static_cast<int64_t>(orig) + a] = o[a];
}

// The last block of k_mark: the rank-th smallest priority inside the bucket, then
// mark every queued voxel up to it. The bucket's members, less the bucket's base, fit
// in its bit width; radix rounds of 8 bits narrow them (from LDS when the bucket fits
// there, else from the queue in global memory) until at most kTieRank remain, which
// are ranked directly (priorities are distinct). The queue was written in the same
// launch, so it is read with agent-scope atomic loads.
__device__ void settle_ties(const Ws& w, Header* h) {
  Ctrl* c = &h->ctrl;
  __shared__ uint32_t cnt_g[kGroups + 1];  // exclusive prefix over groups
  __shared__ uint32_t hst[256];
  __shared__ uint64_t s_pfx, s_thr;
  __shared__ uint32_t s_rank, s_remain, s_nm;
  __shared__ uint64_t lp[kTieLds];
  __shared__ uint64_t ls[kTieRank];
  // the groups' queue lengths, read and reset in parallel (one round trip)
  if (threadIdx.x < kGroups) {
    const uint32_t t = take(&h->tie_cur[threadIdx.x][0]);
    cnt_g[threadIdx.x + 1] = t < w.tie_seg ? t : static_cast<uint32_t>(w.tie_seg);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int q = 0; q < kGroups; ++q) {
      const uint32_t t = cnt_g[q + 1];
      cnt_g[q] = acc;
      acc += t;
    }
    cnt_g[kGroups] = acc;
    s_rank = c->rank;
    s_pfx = 0;
    s_thr = 0;
    s_remain = acc;
    s_nm = 0;
  }
  __syncthreads();
  if (!c->trim) return;
  const uint32_t total = cnt_g[kGroups];
  const bool staged = total <= static_cast<uint32_t>(kTieLds);
  // item j of the bucket: group q with cnt_g[q] <= j < cnt_g[q+1]
  auto locate = [&](uint32_t j) -> int64_t {
    int q = 0;
    while (j >= cnt_g[q + 1]) ++q;
    return static_cast<int64_t>(q) * w.tie_seg + (j - cnt_g[q]);
  };
  // a staged bucket: a thread's members (at most kTP) loaded in one round trip, the
  // priorities copied to LDS for the radix rounds, both kept in registers for the marking
  constexpr int kTP = kTieLds / kThreads;
  static_assert(kTieLds % kThreads == 0, "staged members per thread");
  uint64_t rp[kTP];
  int64_t ro[kTP];
  if (staged) {
    int64_t at[kTP];
#pragma unroll
    for (int q = 0; q < kTP; ++q) {
      const uint32_t j = threadIdx.x + q * kThreads;
      at[q] = j < total ? locate(j) : -1;
    }
#pragma unroll
    for (int q = 0; q < kTP; ++q) {
      rp[q] = ~0ull;
      ro[q] = -1;
      if (at[q] >= 0) {
        rp[q] = ld_agent(&w.tie_p[at[q]]);
        ro[q] = ld_agent(&w.tie_o[at[q]]);
      }
    }
#pragma unroll
    for (int q = 0; q < kTP; ++q)
      if (at[q] >= 0) lp[threadIdx.x + q * kThreads] = rp[q];
    __syncthreads();
  }
  auto prio = [&](uint32_t j) -> uint64_t { return staged ? lp[j] : ld_agent(&w.tie_p[locate(j)]); };
  uint64_t base = 0;
  int hi = 64;
  if (c->trim_mode == 0) {
    hi = 64 - kTrimBits * c->rounds_done;  // bits below the decided prefix
    base = c->prefix;
  } else if (c->trim_mode == 1) {
    base = c->blo;
    const uint64_t width = c->bhi - c->blo;
    hi = width ? 64 - __clzll(static_cast<long long>(width)) : 0;
  }
  while (s_remain > static_cast<uint32_t>(kTieRank) && hi > 0) {
    const int wdt = hi >= 8 ? 8 : hi;
    const int sh = hi - wdt;
    for (int i = threadIdx.x; i < 256; i += kThreads) hst[i] = 0;
    __syncthreads();
    const uint64_t pfx = s_pfx;
    for (uint32_t j = threadIdx.x; j < total; j += kThreads) {
      const uint64_t r = prio(j) - base;
      if (hi < 64 && (r >> hi) != (pfx >> hi)) continue;
      atomicAdd(&hst[(r >> sh) & ((1u << wdt) - 1u)], 1u);
    }
    __syncthreads();
    int b;
    uint32_t rest;
    find_digit(hst, s_rank, &b, &rest);
    if (threadIdx.x == 0) {
      s_rank = rest;
      s_pfx = pfx | (static_cast<uint64_t>(b) << sh);
      s_remain = hst[b];
    }
    __syncthreads();
    hi = sh;
  }
  // the members left: gathered, then the one of rank s_rank among them
  {
    const uint64_t pfx = s_pfx;
    for (uint32_t j = threadIdx.x; j < total; j += kThreads) {
      const uint64_t p = prio(j);
      const uint64_t r = p - base;
      if (hi >= 64 || (r >> hi) == (pfx >> hi)) {
        const uint32_t k = atomicAdd(&s_nm, 1u);
        if (k < static_cast<uint32_t>(kTieRank)) ls[k] = p;
      }
    }
  }
  __syncthreads();
  const uint32_t nm = s_nm < static_cast<uint32_t>(kTieRank) ? s_nm : static_cast<uint32_t>(kTieRank);
  for (uint32_t j = threadIdx.x; j < nm; j += kThreads) {
    const uint64_t pj = ls[j];
    uint32_t r = 0;
    for (uint32_t i = 0; i < nm; ++i) r += ls[i] < pj ? 1u : 0u;
    if (r == s_rank) s_thr = pj;
  }
  __syncthreads();
  const uint64_t thr = s_thr;  // the rank-th smallest priority of the bucket
  const uint8_t lt = static_cast<uint8_t>(c->layer + 1);
  auto pick = [&](int64_t v) {
    const int32_t orig = static_cast<int32_t>(v & 0xFFFFFFFFll);
    const int64_t slot = v >> 32;  // -1 in a cloud's last layer (no sorted tag is kept)
    if (orig >= 0 && orig < w.n) {
      st_agent(&w.tag_o[orig], lt);  // (read back with agent-scope loads when the layer pads)
      if (slot >= 0 && slot < w.npad) w.tag_s[slot] = lt;
    }
  };
  if (staged) {
#pragma unroll
    for (int q = 0; q < kTP; ++q)
      if (threadIdx.x + q * kThreads < total && rp[q] <= thr) pick(ro[q]);
  } else {
    for (uint32_t j = threadIdx.x; j < total; j += kThreads) {
      const int64_t at = locate(j);
      if (ld_agent(&w.tie_p[at]) <= thr) pick(ld_agent(&w.tie_o[at]));
    }
  }
}

// Pad a layer that found fewer voxels than m, in the marking launch's last block: the
// `need` lowest-index points still unsampled get the layer's tag (Sec. 3.3 leaves the
// top-up open; this is the reading both the oracle and the library take). One block
// walks the original-order tags a scan tile at a time and stops as soon as enough are
// marked; the tags the launch's other blocks wrote are read with agent-scope loads.
__device__ __forceinline__ void load_tags_agent(uint8_t* tag, int64_t base, int64_t n,
                                                uint8_t (&t)[kScanPer]) {
  uint32_t* w4 = reinterpret_cast<uint32_t*>(tag + base);  // (base is a multiple of 16)
#pragma unroll
  for (int j = 0; j < kScanPer / 4; ++j) {
    const uint32_t v = base + 4 * j < n ? ld_agent(w4 + j) : 0x01010101u;  // (the region is whole words)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      t[4 * j + b] = base + 4 * j + b < n ? static_cast<uint8_t>(v >> (8 * b)) : static_cast<uint8_t>(1);
  }
}

__device__ void pad_lowest(const Ws& w, int L, uint32_t need) {
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ uint32_t s_before;
  const uint8_t lt = static_cast<uint8_t>(L + 1);
  if (threadIdx.x == 0) s_before = 0u;
  __syncthreads();
  for (int64_t b0 = 0; b0 < w.n; b0 += kScanTile) {
    const uint32_t before = s_before;
    if (before >= need) break;
    const int64_t base = b0 + static_cast<int64_t>(threadIdx.x) * kScanPer;
    uint8_t t[kScanPer];
    load_tags_agent(w.tag_o, base, w.n, t);
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) cnt += (t[k] == 0);
    uint32_t ex;
    const uint32_t tot = block_exclusive_scan<kThreads>(cnt, &ex, s_tmp);
    uint32_t r = before + ex;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (t[k] != 0) continue;
      if (r < need) {
        const int64_t i = base + k;
        w.tag_o[i] = lt;
        w.tag_s[w.invp[i]] = lt;
        if (w.pmode)
          for (int a = 0; a < 3; ++a) w.pt_out[3 * i + a] = w.xyz[3 * i + a];
      }
      ++r;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_before = before + tot;
    __syncthreads();
  }
}

// Keep the representatives below the prefix bucket, queue the bucket's members (the
// last block then settles the bucket), and empty the selection table.
template <class Src>
__global__ void __launch_bounds__(kThreads) k_mark(Src src, int L) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKTile, bx, gx);
  if (!layer_due(cd, L)) return;
  const Ws& w = cd.w;
  Header* h = w.h;
  const Ctrl* c = &h->ctrl;
  const int tile = bx;
  const int n = w.scn[tile];
  const int32_t* list = w.scl + static_cast<size_t>(tile) * kTile;
  const int trim = c->trim;
  const int mode = c->trim_mode;
  const uint64_t blo = c->blo, bhi = c->bhi;
  const int dense = c->sel_dense;
  const int shift = 64 - kTrimBits * c->rounds_done;  // bits below the decided prefix
  const uint64_t pref_hi = shift >= 64 ? 0ull : (c->prefix >> shift);
  const uint8_t lt = static_cast<uint8_t>(c->layer + 1);
  const int g = tile & (kGroups - 1);
  // no later layer reads the sorted-order tags after a cloud's last layer (the output
  // scan reads the original-order ones): the picks' sorted slots are not looked up
  const bool last_layer = L + 1 >= cd.P.nlayers;
  __shared__ uint32_t s_base;
  __shared__ uint32_t s_tmp[kThreads / 64];
  // A tile owns at most kTile voxels: each thread takes its (up to kMP) list entries in
  // one go, so every step's loads are in flight together (list, then table words, then
  // the kept points' sorted slots) instead of one dependent chain per entry.
  constexpr int kMP = kTile / kThreads;
  int32_t sl[kMP];
#pragma unroll
  for (int k = 0; k < kMP; ++k) {
    const int i = static_cast<int>(threadIdx.x) + k * kThreads;
    sl[k] = i < n ? list[i] : -1;
  }
  uint64_t sv[kMP], sk[kMP];
#pragma unroll
  for (int k = 0; k < kMP; ++k) {
    sv[k] = sl[k] >= 0 ? w.svals[sl[k]] : ~0ull;
    sk[k] = (sl[k] >= 0 && !dense) ? w.skeys[sl[k]] : 0ull;
  }
  const uint32_t nx = c->sel_nv[0], ny = c->sel_nv[1];
  int32_t orig[kMP];
  uint64_t pr[kMP];
  uint32_t keepm = 0, tiem = 0;
#pragma unroll
  for (int k = 0; k < kMP; ++k) {
    orig[k] = -1;
    pr[k] = 0;
    if (sl[k] < 0) continue;
    const int32_t s = sl[k];
    uint64_t key = sk[k];
    if (dense) {
      const uint32_t u = static_cast<uint32_t>(s), t = u / nx;
      key = pack_key(u % nx, t % ny, t / ny);
    }
    orig[k] = static_cast<int32_t>(sv[k] & 0xFFFFFFFFull);
    if (!dense) w.skeys[s] = kEmptyKey;
    w.svals[s] = ~0ull;
    if (w.pmode && orig[k] >= 0 && orig[k] < w.n) stand_in(w, c, h->frame, s, key, orig[k]);
    bool keep = true, tie = false;
    if (trim) {
      const uint64_t p = voxel_priority(key);
      pr[k] = p;
      if (mode == 0) {
        const uint64_t hi = shift >= 64 ? 0ull : (p >> shift);
        keep = hi < pref_hi;
        tie = hi == pref_hi;
      } else if (mode == 1) {
        keep = p < blo;
        tie = !keep && p <= bhi;
      } else if (mode == 3) {
        keep = p <= bhi;
      } else {
        keep = false;
        tie = true;
      }
    }
    if (keep && orig[k] >= 0 && orig[k] < w.n) keepm |= 1u << k;
    if (tie) tiem |= 1u << k;
  }
  // the bucket's members go to the group's queue (positions by a block scan and one
  // atomic per block); the atomic and the sorted-slot loads of the kept points and of
  // the bucket's members are in flight together
  uint32_t ex;
  const uint32_t tot = block_exclusive_scan<kThreads>(static_cast<uint32_t>(__popc(tiem)), &ex, s_tmp);
  const uint32_t qb = (threadIdx.x == 0 && tot) ? atomicAdd(&h->tie_cur[g][0], tot) : 0u;
  int32_t ip[kMP];
#pragma unroll
  for (int k = 0; k < kMP; ++k)
    ip[k] = !last_layer && (((keepm | tiem) >> k) & 1u) && orig[k] >= 0 && orig[k] < w.n ? w.invp[orig[k]]
                                                                                       : -1;
  if (threadIdx.x == 0) s_base = qb;
#pragma unroll
  for (int k = 0; k < kMP; ++k) {
    if (!((keepm >> k) & 1u)) continue;  // (kept: orig is a point of the cloud)
    // a layer before the last may pad in this launch's last block, which reads the
    // original-order tags of every block: those are stored at agent scope
    if (last_layer) w.tag_o[orig[k]] = lt;
    else st_agent(&w.tag_o[orig[k]], lt);
    if (ip[k] >= 0) w.tag_s[ip[k]] = lt;
  }
  __syncthreads();
  uint32_t pos = s_base + ex;
#pragma unroll
  for (int k = 0; k < kMP; ++k) {
    if (!((tiem >> k) & 1u)) continue;
    if (pos < w.tie_seg) {
      st_agent(&w.tie_p[g * w.tie_seg + pos], pr[k]);
      st_agent(&w.tie_o[g * w.tie_seg + pos],
               static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(ip[k])) << 32) |
                                    static_cast<uint32_t>(orig[k])));
    }
    ++pos;
  }
  if (threadIdx.x == 0) w.scn[tile] = 0;
  if (!arrive_last(h, bx, gx)) return;
  if (trim && mode != 3) settle_ties(w, h);  // (no member was queued otherwise)
  __syncthreads();
  if (L + 1 < cd.P.nlayers) {  // (a cloud's last layer is padded by the output scan)
    if (c->need > 0) pad_lowest(w, L, c->need);
    layer_init(h, cd.P, L + 1);
  }
}

// ----------------------------------------------------------------------------- scans over tag_o

// Tag scans in one pass: a block takes its scan tile in dispatch order (an atomic
// ticket), counts its tile, publishes the count (slot = count + 1, agent-scope atomic
// store) and adds up the slots of the tiles before it, which belong to blocks that
// started earlier, so every wait ends; the wait is still bounded. The last block
// empties the slots and the ticket for the next scan. Returns the exclusive prefix
// (all threads), or ~0u if a wait gave up.
__device__ uint32_t scan_prefix(const Ws& w, uint32_t mine, int lb) {
  __shared__ uint32_t s_tmp[kThreads / 64];
  __shared__ int s_bad;
  if (threadIdx.x == 0) {
    st_agent(&w.tcnt[lb], mine + 1u);
    s_bad = 0;
  }
  __syncthreads();
  const uint32_t limit = g_scan_spin_limit;
  uint32_t sum = 0;
  for (int i = threadIdx.x; i < lb; i += kThreads) {
    uint32_t v, spins = 0;
    while ((v = ld_agent(&w.tcnt[i])) == 0u) {
      if (++spins > limit) {
        s_bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (v) sum += v - 1u;
  }
  const uint32_t tot = block_sum_u32<kThreads>(sum, s_tmp);
  return s_bad ? ~0u : tot;
}

__device__ __forceinline__ int scan_ticket(Header* h) {
  __shared__ int s_lb;
  if (threadIdx.x == 0) s_lb = static_cast<int>(atomicAdd(&h->ord[0], 1u));
  __syncthreads();
  return s_lb;
}

// The last block of a scan: empty the slots and the ticket.
__device__ void scan_reset(const Ws& w, Header* h, int nb) {
  for (int i = threadIdx.x; i < nb; i += kThreads) st_agent(&w.tcnt[i], 0u);
  if (threadIdx.x == 0) atomicExch(&h->ord[0], 0u);
}

// A thread's kScanPer consecutive tags (from `base`), one 16-byte load where the run is
// whole and aligned; past the end a tag reads as 1 (sampled: neither counted nor padded).
__device__ __forceinline__ void load_tags(const uint8_t* __restrict__ tag, int64_t base, int64_t n,
                                          uint8_t (&t)[kScanPer]) {
  static_assert(kScanPer == 16, "one 16-byte load per thread");
  if (base + kScanPer <= n && (reinterpret_cast<uintptr_t>(tag + base) & 15u) == 0) {
    const uint4 v = *reinterpret_cast<const uint4*>(tag + base);
    const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) t[k] = static_cast<uint8_t>(wv[k >> 2] >> (8 * (k & 3)));
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) t[k] = base + k < n ? tag[base + k] : 1;
  }
}

// Ascending output: every picked point's index, in index order.
template <class Src>
__global__ void __launch_bounds__(kThreads) k_out(Src src) {
  int bx, gx;
  const Cloud& cd = cloud_of(src, kKScan, bx, gx);
  const Ws& w = cd.w;
  if (cd.P.identity) return;
  Header* h = w.h;
  int32_t* idx = w.idx;
  const int64_t M = w.M;
  if (h->frame.status != HAV_OK) {
    if (bx == 0 && threadIdx.x == 0 && w.info_dev) *w.info_dev = h->info;
    return;
  }
  __shared__ uint32_t s_tmp[kThreads / 64];
  // the last layer's pad is done here, in the same scan: with zb unsampled points before
  // point i, a sampled point goes to (i - zb) + min(zb, need) and an unsampled one is
  // padded (to position i) while zb < need
  const uint32_t need = h->ctrl.need;
  const int lb = scan_ticket(h);
  const int64_t base = lb * static_cast<int64_t>(kScanTile) + threadIdx.x * kScanPer;
  uint8_t t[kScanPer];
  load_tags(w.tag_o, base, w.n, t);
  uint32_t cz = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) cz += (t[k] == 0);
  uint32_t ex;
  const uint32_t tot = block_exclusive_scan<kThreads>(cz, &ex, s_tmp);
  const uint32_t before = scan_prefix(w, tot, lb);
  // a point's output position is the number of outputs before it, so the block's outputs
  // fill the range [r0, r1): staged in LDS, then written out coalesced
  __shared__ int32_t s_o[kScanTile];
  const int64_t t0 = lb * static_cast<int64_t>(kScanTile);
  const int64_t t1 = min(w.n, t0 + kScanTile);
  const int64_t r0 = (t0 - before) + min(before, need);
  const int64_t r1 = (t1 - (before + tot)) + min(before + tot, need);
  if (before != ~0u) {
    uint32_t zb = before + ex;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int64_t i = base + k;
      if (i >= w.n) continue;
      int64_t r = -1;
      bool padded = false;
      if (t[k]) {
        r = (i - zb) + (zb < need ? zb : need);
      } else {
        if (zb < need) {
          r = i;
          padded = true;
        }
        ++zb;
      }
      if (r >= 0 && r < M) {
        s_o[r - r0] = static_cast<int32_t>(i);
        if (w.xyz_out) {
          // centre / mean modes: what stands for the point; else (and for a padded
          // point) the point itself
          const float* src = (w.pmode && !padded ? w.pt_out : w.xyz) + 3 * i;
          for (int a = 0; a < 3; ++a) w.xyz_out[3 * r + a] = src[a];
        }
      }
    }
  } else if (threadIdx.x == 0) {
    atomicOr(&h->scan_bad[0], 1u);
  }
  __syncthreads();
  if (before != ~0u)
    for (int64_t j = threadIdx.x; r0 + j < min(r1, M); j += kThreads) idx[r0 + j] = s_o[j];
  if (!arrive_last(h, bx, gx)) return;
  scan_reset(w, h, gx);
  // the report: its words and the scan's failure flag load in one round trip, one word a
  // thread, then go to the caller
  constexpr int kInfoWords = static_cast<int>(sizeof(hav_info_t) / 4);
  static_assert(kInfoWords <= kThreads, "report words per thread");
  __shared__ uint32_t s_bad;
  int32_t* iw = reinterpret_cast<int32_t*>(&h->info);
  const int32_t word = threadIdx.x < kInfoWords ? iw[threadIdx.x] : 0;
  if (threadIdx.x == 0) s_bad = take(&h->scan_bad[0]);
  __syncthreads();
  if (threadIdx.x < kInfoWords) {
    // (status is the report's first word)
    const int32_t v = (threadIdx.x == 0 && s_bad) ? static_cast<int32_t>(HAV_ERR_HIP) : word;
    if (threadIdx.x == 0 && s_bad) iw[0] = v;
    if (w.info_dev) reinterpret_cast<int32_t*>(w.info_dev)[threadIdx.x] = v;
  }
}

// ----------------------------------------------------------------------------- workspace init

// keep_if: a workspace whose magic already equals it is left as it is (every block reads
// the magic before any block could clear it, and a clearing block only zeroes it, so all
// blocks take the same decision); 0 clears unconditionally.
__global__ void __launch_bounds__(kThreads) k_ws_init(Ws w, size_t nct, size_t ncn, size_t nst,
                                                      size_t nsv, size_t nsn, size_t nhr, size_t nsc,
                                                      size_t nms, uint64_t keep_if) {
  if (keep_if != 0 && w.h->magic == keep_if) return;
  const size_t stride = static_cast<size_t>(gridDim.x) * kThreads;
  const size_t t0 = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x;
  for (size_t i = t0; i < nct; i += stride) {
    w.ckeys[i] = kEmptyKey;
    w.cmasks[i] = 0ull;
  }
  for (size_t i = t0; i < ncn; i += stride) w.ccn[i] = 0;
  for (size_t i = t0; i < nhr; i += stride) w.hrep[i] = 0ull;
  for (size_t i = t0; i < nsc; i += stride) w.tcnt[i] = 0u;
  for (size_t i = t0; i < nms; i += stride) {
    w.msum[3 * i] = 0ull;
    w.msum[3 * i + 1] = 0ull;
    w.msum[3 * i + 2] = 0ull;
    w.mcnt[i] = 0u;
  }
  for (size_t i = t0; i < nst; i += stride) w.skeys[i] = kEmptyKey;
  for (size_t i = t0; i < nsv; i += stride) w.svals[i] = ~0ull;
  for (size_t i = t0; i < nsn; i += stride) w.scn[i] = 0;
  uint32_t* hz = reinterpret_cast<uint32_t*>(w.h);
  for (size_t i = t0; i < sizeof(Header) / 4; i += stride) hz[i] = 0;
}

// The magic is written by a later kernel than the clearing, so it is only seen set
// once everything else is.
__global__ void k_ws_seal(Header* h, uint64_t magic) {
  if (threadIdx.x == 0) h->magic = magic;
}

// ----------------------------------------------------------------------------- chain helpers

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

// ----------------------------------------------------------------------------- grouping

// Ball query on the sampler's own spatial structure (the grouping that follows sampling
// in a set-abstraction block, Sec. 3.1): after a call on this workspace, the cloud sits
// counting-sorted by binning cell (pts, with invp from each point to its slot and the
// cell offsets of the scan), so the points near a centre are the points of the few cells
// its ball overlaps. No second sort of the cloud is made: the centres are bucketed by the
// tile holding them (in the selection's per-tile lists, free once a call has ended); a
// tile's centres form work items of at most a group each, and resident blocks take the
// items in turn. A block stages the cells its group's balls overlap through LDS in cell
// order, a buffer at a time, and a wave tests 64 staged points against one centre per
// step.
constexpr int kBallMaxK = 64;
constexpr int kBallBuf = 2048;        // points staged in LDS per fill
constexpr int kBallFill = 64;         // cells (or parts of one) per fill: one per lane
constexpr int kBallRowWords = 5120;   // LDS words for the group's sorted rows
constexpr int kBallThreads = 512;     // threads of a grouping block
constexpr int kBallGroup = 256;       // centres per group at most
static_assert(kBins / 64 == 64, "one word of the needed-cell bitmap per lane");
static_assert(kBallBuf % kBallThreads == 0, "staged points per thread");
static_assert(kBallGroup <= kBallThreads, "a thread per centre while a group loads");

__device__ __forceinline__ bool ball_ready(const Ws& w) {
  return w.h->binned_n == w.n && w.h->frame.status == HAV_OK;
}

__device__ __forceinline__ uint32_t cell_start(const Ws& w, uint32_t code) {
  return code >= static_cast<uint32_t>(kBins) ? static_cast<uint32_t>(w.n)
                                              : w.binpre[code] + w.bsum[code / kBinChunk];
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

__device__ __forceinline__ int32_t lane_of(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Bucket each centre j (point idx[j]) by the tile holding its sorted slot. A centre
// that is not a point of the cloud, or any centre when the workspace does not hold this
// cloud's sorted points, gets an empty row (-1) and count -1.
__global__ void __launch_bounds__(kThreads) k_ball_bucket(Ws w, const int32_t* __restrict__ idx, int64_t M,
                                                         int32_t K, int32_t* out, int32_t* count) {
  const bool ready = ball_ready(w);
  for (int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; j < M;
       j += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int32_t i = idx[j];
    bool ok = ready && i >= 0 && i < w.n;
    if (ok) {
      const int64_t t = w.invp[i] / kTile;
      const int pos = atomicAdd(&w.scn[t], 1);
      if (pos < kTile) w.scl[t * kTile + pos] = static_cast<int32_t>(j);
      else ok = false;  // (more than a tile's points: the centres were not distinct)
    }
    if (!ok) {
      for (int q = 0; q < K; ++q) out[j * K + q] = -1;
      if (count) count[j] = -1;
    }
  }
}

// The grouping's work items: each tile's centres in groups of at most G (as many rows
// as fit in LDS), as (tile << 32 | first centre << 16 | centres), listed in the trim
// queue's storage (written and read within a sampling call, so free between calls);
// the tiles' centre counts go back to zero for the selection. The list is ordered by an
// estimate of the item's work, largest first, so that the blocks taking items in turn
// end together: the centres times the points of the binning cell at the tile's middle
// (a centre scans the few cells around it), in classes of powers of two.
constexpr int kBallCostClasses = 48;
__global__ void __launch_bounds__(kBallThreads) k_ball_plan(Ws w, int32_t G) {
  if (!ball_ready(w)) return;
  __shared__ uint32_t s_tmp[kBallThreads / 64];
  __shared__ uint32_t s_cls[kBallCostClasses];
  __shared__ CellCoder s_kc;
  if (threadIdx.x < kBallCostClasses) s_cls[threadIdx.x] = 0u;
  if (threadIdx.x == 0) s_kc = make_coder(w.h->frame);
  __syncthreads();
  const CellCoder kc = s_kc;
  int64_t* tmp = w.tie_o;  // (the items in tile order, with their class in bits 56..61)
  uint32_t base = 0u;
  for (int t0 = 0; t0 < w.ntile; t0 += kBallThreads) {
    const int t = t0 + static_cast<int>(threadIdx.x);
    uint32_t nc = 0u, ng = 0u, dens = 1u;
    if (t < w.ntile) {
      nc = min(static_cast<uint32_t>(w.scn[t]), static_cast<uint32_t>(kTile));
      ng = (nc + G - 1) / G;
      w.scn[t] = 0;
      if (nc) {
        const int64_t mid = min(static_cast<int64_t>(t) * kTile + kTile / 2, w.n - 1);
        const float4 rec = w.pts[slot_of(mid)];
        const uint32_t code = cell_code_k(rec.x, rec.y, rec.z, kc);
        dens = max(1u, cell_start(w, code + 1) - cell_start(w, code));
      }
    }
    uint32_t ex;
    const uint32_t tot = block_exclusive_scan<kBallThreads>(ng, &ex, s_tmp);
    for (uint32_t g = 0; g < ng; ++g) {
      const uint32_t g0 = g * G;
      const uint32_t cnt = min(static_cast<uint32_t>(G), nc - g0);
      const uint64_t cost = static_cast<uint64_t>(cnt) * dens;
      const int cls = 63 - __clzll(static_cast<long long>(cost));  // (cost >= 1)
      atomicAdd(&s_cls[cls], 1u);
      tmp[base + ex + g] = static_cast<int64_t>((static_cast<uint64_t>(cls) << 56) | (static_cast<uint64_t>(t) << 32) |
                                                (static_cast<uint64_t>(g0) << 16) | cnt);
    }
    base += tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // class offsets, largest class first
    uint32_t run = 0u;
    for (int c = kBallCostClasses - 1; c >= 0; --c) {
      const uint32_t v = s_cls[c];
      s_cls[c] = run;
      run += v;
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < base; i += kBallThreads) {
    const uint64_t v = static_cast<uint64_t>(tmp[i]);
    const int cls = static_cast<int>(v >> 56);
    w.tie_p[atomicAdd(&s_cls[cls], 1u)] = v & ((uint64_t(1) << 56) - 1);
  }
  if (threadIdx.x == 0) {
    w.h->ball_items = base;
    w.h->ball_next = 0u;
  }
}

// Blocks take work items until none is left. Per item, for each centre of its group:
// the K lowest indices i with d2 < r2, d2 in float32 as ((dx dx + dy dy) + dz dz) of the
// original coordinates (dx = x_i - c), the rest of a row repeating its first entry;
// count = points inside. A centre needs the cells whose index range covers its
// coordinate offset +- the radius widened by 1e-3 of itself and by 1e-6 of the offset
// (more than the rounding of d2, of dx and of the offsets r = fl(p - origin) the cells
// were assigned by); cell_index is non-decreasing in r, so every point inside the ball
// lies in a needed cell.
//
// For a group the block marks the needed cells in a 4,096-bit map, then walks the map in
// cell order: wave 0 lists the next needed cells and cuts them to the buffer (a cell
// larger than the buffer is taken in parts), every thread stages its share of the
// points (the sorted record for the original index, then the original coordinates), and
// each wave takes every eighth centre of the group: the fill's cells inside the centre's
// cell box are found with one ballot (a cell per lane), and their points are tested 64
// at a time. A centre's row of the K lowest indices so far lives one entry per lane
// while its wave works on it (insertion: every lane above the new index takes its lower
// neighbour's entry, a one-lane DPP shift) and in LDS between fills. Each point of a
// needed cell is staged once per group, so no index enters a row twice.
__global__ void __launch_bounds__(kBallThreads) k_ball_group(Ws w, const float* __restrict__ xyz,
                                                        const int32_t* __restrict__ idx, float radius,
                                                        float r2, int32_t K, int32_t* out, int32_t* count) {
  if (!ball_ready(w)) return;  // (then the lists were not touched, and may be laid out otherwise)
  const uint32_t nitems = w.h->ball_items;
  __shared__ uint32_t s_cs[kBins + 1];
  __shared__ float4 s_buf[kBallBuf];
  __shared__ int32_t s_row[kBallRowWords];
  __shared__ float4 s_cen[kBallGroup];
  __shared__ uint32_t s_box[3][kBallGroup];
  __shared__ uint32_t s_tot[kBallGroup];
  __shared__ unsigned long long s_need[kBins / 64];
  __shared__ uint32_t s_list[kBallFill];
  __shared__ uint32_t s_fxy[kBallFill], s_fz[kBallFill], s_foff[kBallFill], s_flen[kBallFill],
      s_fbeg[kBallFill];
  __shared__ int s_nf, s_ntot, s_cur, s_more;
  __shared__ uint32_t s_curoff;
  __shared__ CellCoder s_kc;
  __shared__ float s_mn[3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int kWaves = kBallThreads / 64;
  if (threadIdx.x == 0) {
    const Frame f = w.h->frame;
    s_kc = make_coder(f);
    for (int a = 0; a < 3; ++a) s_mn[a] = f.mn[a];
  }
  for (int c = threadIdx.x; c <= kBins; c += kBallThreads) s_cs[c] = cell_start(w, c);
  __syncthreads();
  const CellCoder kc = s_kc;
  __shared__ uint32_t s_it;
  for (;;) {
    if (threadIdx.x == 0) s_it = atomicAdd(&w.h->ball_next, 1u);
    __syncthreads();
    const uint32_t it = s_it;
    if (it >= nitems) break;
    const uint64_t item = w.tie_p[it];
    const int t = static_cast<int>(item >> 32);
    const int g0 = static_cast<int>((item >> 16) & 0xFFFFu);
    const int ng = static_cast<int>(item & 0xFFFFu);
    if (threadIdx.x < kBins / 64) s_need[threadIdx.x] = 0ull;
    for (int q = threadIdx.x; q < ng * K; q += kBallThreads) s_row[q] = INT32_MAX;
    if (threadIdx.x == 0) {
      s_cur = 0;
      s_curoff = 0u;
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < ng) {
      const int c = threadIdx.x;
      const int32_t j = w.scl[static_cast<int64_t>(t) * kTile + g0 + c];
      const int64_t ci = idx[j];
      float cx[3];
      uint32_t lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        cx[a] = xyz[3 * ci + a];
        const float rc = cx[a] - s_mn[a];
        const float rad = radius * 1.001f + 1e-6f * (fabsf(rc) + radius);
        lo[a] = cell_index(rc - rad, kc, a);
        hi[a] = cell_index(rc + rad, kc, a);
        s_box[a][c] = lo[a] | (hi[a] << 16);
      }
      s_cen[c] = make_float4(cx[0], cx[1], cx[2], __int_as_float(j));
      s_tot[c] = 0u;
      for (uint32_t iz = lo[2]; iz <= hi[2]; ++iz)
        for (uint32_t iy = lo[1]; iy <= hi[1]; ++iy)
          for (uint32_t ix = lo[0]; ix <= hi[0]; ++ix) {
            const uint32_t cc[3] = {ix, iy, iz};
            const uint32_t code = cell_code_of(cc, kc);
            atomicOr(&s_need[code >> 6], 1ull << (code & 63));
          }
    }
    __syncthreads();
    for (;;) {
      // wave 0: the next needed cells in cell order (a lane per bitmap word)
      const int cur = s_cur;
      const uint32_t curoff = s_curoff;
      uint32_t tot_codes = 0u;
      if (wv == 0) {
        unsigned long long wd = s_need[lane];
        const int cw = cur >> 6;
        if (lane < cw) wd = 0ull;
        else if (lane == cw) wd &= ~0ull << (cur & 63);
        const uint32_t cnt = static_cast<uint32_t>(__popcll(wd));
        const uint32_t inc = wave_incl_scan(cnt);
        tot_codes = static_cast<uint32_t>(__shfl(static_cast<int>(inc), 63, 64));
        uint32_t r = inc - cnt;
        while (wd && r < static_cast<uint32_t>(kBallFill)) {
          s_list[r++] = static_cast<uint32_t>(lane * 64 + __ffsll(static_cast<long long>(wd)) - 1);
          wd &= wd - 1;
        }
      }
      __syncthreads();
      if (wv == 0) {
        // cut the listed cells to the buffer: a lane per cell
        const int nl = static_cast<int>(min(tot_codes, static_cast<uint32_t>(kBallFill)));
        uint32_t code = 0u, base = 0u, cs = 0u, sz = 0u;
        if (lane < nl) {
          code = s_list[lane];
          base = s_cs[code];
          cs = base + (static_cast<int>(code) == cur ? curoff : 0u);
          sz = s_cs[code + 1] - cs;
        }
        const uint32_t incl = wave_incl_scan(sz);
        const uint32_t exs = incl - sz;
        const uint32_t take = exs >= static_cast<uint32_t>(kBallBuf) ? 0u : min(sz, kBallBuf - exs);
        const unsigned long long hasm = __ballot(take > 0u);
        if (take > 0u) {
          const int e = __popcll(hasm & ((1ull << lane) - 1ull));
          uint32_t cc[3] = {0u, 0u, 0u};
          for (int a = 0; a < 3; ++a)
            for (int j = 0; j < kBinBits; ++j)
              if (j < kc.bb[a]) cc[a] |= ((code >> ((kc.pos[a] >> (4 * j)) & 15u)) & 1u) << j;
          s_fxy[e] = cc[0] | (cc[1] << 16);
          s_fz[e] = cc[2];
          s_foff[e] = exs;
          s_flen[e] = take;
          s_fbeg[e] = cs;
        }
        const unsigned long long short_m = __ballot(lane < nl && take < sz);
        const int p = short_m ? __ffsll(static_cast<long long>(short_m)) - 1 : (nl > 0 ? nl - 1 : 0);
        const uint32_t code_p = static_cast<uint32_t>(lane_of(static_cast<int32_t>(code), p));
        const uint32_t off_p = static_cast<uint32_t>(lane_of(static_cast<int32_t>(cs - base + take), p));
        const uint32_t all = static_cast<uint32_t>(lane_of(static_cast<int32_t>(incl), 63));
        if (lane == 0) {
          s_nf = __popcll(hasm);
          s_ntot = static_cast<int>(min(all, static_cast<uint32_t>(kBallBuf)));
          if (short_m) {
            s_cur = static_cast<int>(code_p);  // (the buffer ran out in or before this cell)
            s_curoff = off_p;
            s_more = 1;
          } else if (nl > 0) {
            s_cur = static_cast<int>(code_p) + 1;
            s_curoff = 0u;
            s_more = tot_codes > static_cast<uint32_t>(nl) ? 1 : 0;
          } else {
            s_more = 0;
          }
        }
      }
      __syncthreads();
      const int nf = s_nf, ntot = s_ntot;
      const bool more = s_more != 0;
      // stage: the sorted records of the fill's cells, then their original coordinates
      {
        int32_t o[kBallBuf / kBallThreads];
#pragma unroll
        for (int k = 0; k < kBallBuf / kBallThreads; ++k) {
          const int q = k * kBallThreads + static_cast<int>(threadIdx.x);
          o[k] = -1;
          if (q < ntot) {
            int lo = 0, hi = nf - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (static_cast<int>(s_foff[mid]) <= q) lo = mid;
              else hi = mid - 1;
            }
            const int64_t L = static_cast<int64_t>(s_fbeg[lo]) + (q - static_cast<int>(s_foff[lo]));
            o[k] = __float_as_int(w.pts[slot_of(L)].w);
          }
        }
#pragma unroll
        for (int k = 0; k < kBallBuf / kBallThreads; ++k) {
          const int q = k * kBallThreads + static_cast<int>(threadIdx.x);
          if (o[k] >= 0) {
            const int64_t oi = o[k];
            s_buf[q] = make_float4(xyz[3 * oi], xyz[3 * oi + 1], xyz[3 * oi + 2], __int_as_float(o[k]));
          }
        }
      }
      __syncthreads();
      // test: the fill's cells one per lane, each wave every kWaves-th centre
      uint32_t fx = 0xFFFFFFFFu, fy = 0xFFFFFFFFu, fz = 0xFFFFFFFFu, foff = 0u, flen = 0u;
      if (lane < nf) {
        const uint32_t xy = s_fxy[lane];
        fx = xy & 0xFFFFu;
        fy = xy >> 16;
        fz = s_fz[lane];
        foff = s_foff[lane];
        flen = s_flen[lane];
      }
      for (int c = wv; c < ng; c += kWaves) {
        const uint32_t bx = s_box[0][c], by = s_box[1][c], bz = s_box[2][c];
        unsigned long long cm = __ballot(lane < nf && fx >= (bx & 0xFFFFu) && fx <= (bx >> 16) &&
                                         fy >= (by & 0xFFFFu) && fy <= (by >> 16) &&
                                         fz >= (bz & 0xFFFFu) && fz <= (bz >> 16));
        if (!cm) continue;
        const float4 ce = s_cen[c];
        int32_t rv = lane < K ? s_row[c * K + lane] : INT32_MAX;
        uint32_t tot = 0u;
        while (cm) {
          const int e = __ffsll(static_cast<long long>(cm)) - 1;
          cm &= cm - 1ull;
          const int off = lane_of(static_cast<int32_t>(foff), e);
          const int len = lane_of(static_cast<int32_t>(flen), e);
          auto insert = [&](bool hit, int32_t id) {
            // candidates below the K-th entry; inserting one that an earlier insert pushed
            // past it only touches lanes >= K, which hold the row's overflow in order
            unsigned long long im = __ballot(hit && id < lane_of(rv, K - 1));
            while (im) {
              const int l = __ffsll(static_cast<long long>(im)) - 1;
              im &= im - 1ull;
              const int32_t nid = lane_of(id, l);
              const int32_t up = __builtin_amdgcn_update_dpp(INT32_MIN, rv, 0x138, 0xF, 0xF, false);
              rv = rv > nid ? (up > nid ? up : nid) : rv;
            }
          };
          for (int b = 0; b < len; b += 128) {
            const bool v0 = b + lane < len, v1 = b + 64 + lane < len;
            float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f), p1 = p0;
            if (v0) p0 = s_buf[off + b + lane];
            if (v1) p1 = s_buf[off + b + 64 + lane];
            bool hit0 = false, hit1 = false;
            if (v0) {
              const float dx = p0.x - ce.x, dy = p0.y - ce.y, dz = p0.z - ce.z;
              const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
              hit0 = ((xx + yy) + zz) < r2;
            }
            if (v1) {
              const float dx = p1.x - ce.x, dy = p1.y - ce.y, dz = p1.z - ce.z;
              const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
              hit1 = ((xx + yy) + zz) < r2;
            }
            const unsigned long long hm0 = __ballot(hit0), hm1 = __ballot(hit1);
            if (!(hm0 | hm1)) continue;
            tot += static_cast<uint32_t>(__popcll(hm0) + __popcll(hm1));
            if (hm0) insert(hit0, __float_as_int(p0.w));
            if (hm1) insert(hit1, __float_as_int(p1.w));
          }
        }
        if (lane < K) s_row[c * K + lane] = rv;
        if (lane == 0) s_tot[c] += tot;
      }
      __syncthreads();
      if (!more) break;
    }
    // the group's rows are final
    for (int c = wv; c < ng; c += kWaves) {
      const int64_t j = __float_as_int(s_cen[c].w);
      const int32_t rv = lane < K ? s_row[c * K + lane] : INT32_MAX;
      const int n = __popcll(__ballot(lane < K && rv != INT32_MAX));
      const int32_t first = lane_of(rv, 0);
      if (lane < K) out[j * K + lane] = lane < n ? rv : (n > 0 ? first : -1);
      if (lane == 0 && count) count[j] = static_cast<int32_t>(min(s_tot[c], 0x7FFFFFFFu));
    }
    __syncthreads();
  }
}

// ============================================================================ host side

constexpr size_t kAlign = 256;
__host__ __device__ inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int depth_of(const hav_params_t* p) {
  return p->spec_depth == 0 ? kDefaultDepth : p->spec_depth;
}
int bin_code(int32_t bin_points) { return bin_points == 2048 ? 1 : (bin_points == 8192 ? 2 : 0); }
int tscale_of(const hav_params_t* p) { return p->table_scale | (bin_code(p->bin_points) << 4); }

// Table slots for a stage of n points: a power of two >= n, and >= min(8n, 2^20), times
// 2^tscale (the tuning field table_scale), at most 2^31. A table never holds more keys
// than the stage has points, so with at least n slots every probe ends (a key is found
// or claims an empty slot). The 8n floor matters for small clouds of large extent
// (LiDAR sweeps): their brick and voxel grids at the fine sizes are far larger than n,
// and a bigger table keeps more candidates on the dense (unprobed) path and the hashed
// ones sparse.
constexpr uint64_t kMinTableCap = uint64_t(1) << 20;
constexpr uint64_t kTableFloorMult = 8;
__host__ __device__ inline uint32_t table_cap(int64_t n, int tscale) {
  const uint64_t nn = static_cast<uint64_t>(n);
  const uint64_t floor_cap = kTableFloorMult * nn < kMinTableCap ? kTableFloorMult * nn : kMinTableCap;
  const uint64_t want = nn > floor_cap ? nn : floor_cap;
  uint64_t cap = 1;
  while (cap < want) cap <<= 1;
  cap <<= tscale;
  return static_cast<uint32_t>(cap < (uint64_t(1) << 31) ? cap : (uint64_t(1) << 31));
}

// Voxel value slots of the selection table: kSelDense per brick-table slot and at least
// a power of two >= 8n (times 2^tscale), at most 2^31. A voxel grid at the chosen size
// that fits is indexed directly (no probing); at scene density the grid of the last
// layer is a few times the point count.
__host__ __device__ inline uint32_t sel_cap_of(int64_t n, int tscale) {
  uint64_t want = static_cast<uint64_t>(table_cap(n, tscale)) * kSelDense;
  uint64_t c = 1;
  while (c < 8 * static_cast<uint64_t>(n)) c <<= 1;
  c <<= tscale;
  if (c > want) want = c;
  return static_cast<uint32_t>(want < (uint64_t(1) << 31) ? want : (uint64_t(1) << 31));
}

struct Layout {
  size_t hdr, pts, invp, tag_s, tag_o, part, bh, binpre, bsum, ckeys, cmasks, ccl, hrep, ccn, skeys, svals, scl,
      scn, tie_p, tie_o, tcnt, pto, msum, mcnt, total;
  int64_t n_ws;
  int32_t pmode, tscale;
  uint32_t cap_ws, sel_ws;
  int32_t ntile_ws, nscan_ws, ncmax;
  int64_t tie_seg;
};

__host__ __device__ inline Layout make_layout(int64_t n, int depth, int tscale, int pmode = 0) {
  Layout L;
  L.n_ws = n;
  L.pmode = pmode;
  L.tscale = tscale;
  L.cap_ws = table_cap(n, tab_scale(tscale));
  L.sel_ws = sel_cap_of(n, tab_scale(tscale));
  L.ntile_ws = static_cast<int32_t>((n + kTile - 1) / kTile);
  L.nscan_ws = static_cast<int32_t>((n + kScanTile - 1) / kScanTile);
  L.ncmax = depth;
  L.tie_seg = static_cast<int64_t>((L.ntile_ws + kGroups - 1) / kGroups) * kTile;
  const size_t N = static_cast<size_t>(n);
  const size_t NP = static_cast<size_t>(L.ntile_ws) * kTile;
  const size_t tabs = 2 * static_cast<size_t>(L.ncmax);
  size_t o = 0;
  L.hdr = o;    o = align_up(o + sizeof(Header));
  L.pts = o;    o = align_up(o + NP * 16);
  L.invp = o;   o = align_up(o + N * 4);
  L.tag_s = o;  o = align_up(o + NP);
  L.tag_o = o;  o = align_up(o + N);
  L.part = o;   o = align_up(o + static_cast<size_t>(kMaxBBoxBlocks) * 8 * 4);
  L.bh = o;     o = align_up(o + static_cast<size_t>(kBins) * blocks_of(kKBin, n, bin_shift(tscale)) * 4);
  L.binpre = o; o = align_up(o + static_cast<size_t>(kBins) * 4);
  L.bsum = o;   o = align_up(o + static_cast<size_t>(kBinChunks) * 4);
  L.ckeys = o;  o = align_up(o + tabs * L.cap_ws * 8);
  L.cmasks = o; o = align_up(o + tabs * L.cap_ws * 8);
  L.ccl = o;    o = align_up(o + tabs * L.ntile_ws * kClaimCap * 4);
  L.hrep = o;   o = align_up(o + tabs * kReps * kHotCap * 8);
  L.ccn = o;    o = align_up(o + tabs * L.ntile_ws * 4);
  L.skeys = o;  o = align_up(o + static_cast<size_t>(L.cap_ws) * 8);
  L.svals = o;  o = align_up(o + static_cast<size_t>(L.sel_ws) * 8);
  L.scl = o;    o = align_up(o + static_cast<size_t>(L.ntile_ws) * kTile * 4);
  L.scn = o;    o = align_up(o + static_cast<size_t>(L.ntile_ws) * 4);
  L.tie_p = o;  o = align_up(o + static_cast<size_t>(kGroups) * L.tie_seg * 8);
  L.tie_o = o;  o = align_up(o + static_cast<size_t>(kGroups) * L.tie_seg * 8);
  L.tcnt = o;   o = align_up(o + static_cast<size_t>(L.nscan_ws) * 4);
  const size_t slots = pmode == 2 ? static_cast<size_t>(L.sel_ws) : 0;
  L.pto = o;    o = align_up(o + (pmode ? N * 12 : 0));
  L.msum = o;   o = align_up(o + slots * 24);
  L.mcnt = o;   o = align_up(o + slots * 4);
  L.total = o;
  return L;
}

__host__ __device__ inline uint64_t magic_of(const Layout& L) {
  return kMagic ^ (static_cast<uint64_t>(L.n_ws) << 8) ^ (static_cast<uint64_t>(L.ncmax) << 56) ^
         (static_cast<uint64_t>(L.pmode) << 48) ^ (static_cast<uint64_t>(L.tscale) << 44);
}

// Device view of the workspace for a stage of n points (n <= the workspace's size).
__host__ __device__ inline Ws make_ws(char* base, const Layout& L, int64_t n) {
  Ws w;
  w.h = reinterpret_cast<Header*>(base + L.hdr);
  w.pts = reinterpret_cast<float4*>(base + L.pts);
  w.invp = reinterpret_cast<int32_t*>(base + L.invp);
  w.tag_s = reinterpret_cast<uint8_t*>(base + L.tag_s);
  w.tag_o = reinterpret_cast<uint8_t*>(base + L.tag_o);
  w.part = reinterpret_cast<uint32_t*>(base + L.part);
  w.bh = reinterpret_cast<uint32_t*>(base + L.bh);
  w.binpre = reinterpret_cast<uint32_t*>(base + L.binpre);
  w.bsum = reinterpret_cast<uint32_t*>(base + L.bsum);
  w.ckeys = reinterpret_cast<unsigned long long*>(base + L.ckeys);
  w.cmasks = reinterpret_cast<unsigned long long*>(base + L.cmasks);
  w.ccl = reinterpret_cast<int32_t*>(base + L.ccl);
  w.hrep = reinterpret_cast<unsigned long long*>(base + L.hrep);
  w.ccn = reinterpret_cast<int32_t*>(base + L.ccn);
  w.skeys = reinterpret_cast<unsigned long long*>(base + L.skeys);
  w.svals = reinterpret_cast<unsigned long long*>(base + L.svals);
  w.scl = reinterpret_cast<int32_t*>(base + L.scl);
  w.scn = reinterpret_cast<int32_t*>(base + L.scn);
  w.tie_p = reinterpret_cast<uint64_t*>(base + L.tie_p);
  w.tie_o = reinterpret_cast<int64_t*>(base + L.tie_o);
  w.tcnt = reinterpret_cast<uint32_t*>(base + L.tcnt);
  w.pmode = L.pmode;
  w.pt_out = L.pmode ? reinterpret_cast<float*>(base + L.pto) : nullptr;
  w.msum = L.pmode == 2 ? reinterpret_cast<unsigned long long*>(base + L.msum) : nullptr;
  w.mcnt = L.pmode == 2 ? reinterpret_cast<uint32_t*>(base + L.mcnt) : nullptr;
  w.xyz_out = nullptr;
  w.n = n;
  w.ntile = static_cast<int32_t>((n + kTile - 1) / kTile);
  w.npad = static_cast<int64_t>(w.ntile) * kTile;
  w.nscan = static_cast<int32_t>((n + kScanTile - 1) / kScanTile);
  w.nbb = static_cast<int32_t>(blocks_of(kKBin, n, bin_shift(L.tscale)));
  w.nbbox = static_cast<int32_t>(blocks_of(kKBBox, n));
  w.cap = table_cap(n, tab_scale(L.tscale));
  w.cmask = w.cap - 1;
  w.cap_ws = L.cap_ws;
  w.ntile_ws = L.ntile_ws;
  w.ncmax = L.ncmax;
  w.tie_seg = L.tie_seg;
  w.xyz = nullptr;
  w.idx = nullptr;
  w.info_dev = nullptr;
  w.M = 0;
  return w;
}

// Parameters of any entry point; the selections whose representatives are not cloud
// points (centre, mean) only through hav_sample_points.
bool params_any_ok(const hav_params_t* p);
bool params_ok(const hav_params_t* p) {
  return params_any_ok(p) && (p->select == HAV_SELECT_CENTRE_CLOSEST || p->select == HAV_SELECT_RANDOM);
}
int points_mode(const hav_params_t* p) {
  return p->select == HAV_SELECT_CENTRE ? 1 : (p->select == HAV_SELECT_MEAN ? 2 : 0);
}
bool params_any_ok(const hav_params_t* p) {
  if (!p || p->abi_version != HAV_ABI_VERSION) return false;
  if (p->layers < 1 || p->layers > HAV_MAX_LAYERS) return false;
  if (p->layer_ratio < 2 || p->layer_ratio > 16) return false;
  if (p->t_max < 1 || p->t_max > 20) return false;
  if (!std::isfinite(p->sigma) || p->sigma < 0.0 || p->sigma > 16.0) return false;
  if (p->flags & ~HAV_FIXED_VOXEL) return false;
  if (p->spec_depth < 0 || p->spec_depth > kMaxDepth) return false;
  if (p->spec_budget < 0 || p->spec_budget > 1024) return false;
  if (p->search_blocks < 0 || p->search_blocks > 65536) return false;
  if (p->table_scale < 0 || p->table_scale > 3) return false;
  if (p->bin_points != 0 && p->bin_points != 2048 && p->bin_points != 4096 && p->bin_points != 8192)
    return false;
  if (!std::isfinite(p->trim_window) || p->trim_window > 64.0f) return false;
  if (p->select < HAV_SELECT_CENTRE_CLOSEST || p->select > HAV_SELECT_MEAN) return false;
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
__host__ __device__ inline void layer_sizes(int64_t M, int k, int r, int64_t* m) {
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

// Radix rounds over the top priority bits before one block settles the bucket:
// enough that the expected bucket (n / 256^R) stays small.
// Radix rounds of a trim over about v voxels: enough that the expected bucket left
// for k_ties (v / 256^R) is small enough to rank directly.
__host__ __device__ inline int trim_rounds(int64_t v) {
  int R = 1;
  while (R < 7 && (v >> (kTrimBits * R)) > kTieRank / 2) ++R;
  return R;
}

// The sampling parameters a plan needs (plain values, so a kernel can take them).
struct ParamLite {
  int32_t layers, ratio, t_max, depth, tscale, fixed, spec_budget;
  double sigma;
  float trim_window;
  float aspect[3], fixed_v[3];
  int32_t select;
  uint32_t seed;
};

ParamLite lite_of(const hav_params_t* p) {
  ParamLite q;
  q.layers = p->layers;
  q.ratio = p->layer_ratio;
  q.t_max = p->t_max;
  q.depth = depth_of(p);
  q.tscale = tscale_of(p);
  q.fixed = (p->flags & HAV_FIXED_VOXEL) ? 1 : 0;
  q.spec_budget = p->spec_budget;
  q.sigma = p->sigma;
  q.trim_window = p->trim_window;
  q.select = p->select;
  q.seed = p->select_seed;
  for (int a = 0; a < 3; ++a) {
    q.aspect[a] = p->aspect[a];
    q.fixed_v[a] = p->fixed_voxel[a];
  }
  return q;
}

// One cloud of a call: input, output, report and its workspace segment (laid out for
// n_cap >= n points).
struct CloudSpec {
  const float* xyz;
  int32_t* idx;
  hav_info_t* info;
  char* seg;
  int64_t n, m, n_cap;
  float* xyz_out;  // points modes only (else null)
};

__host__ __device__ inline Cloud make_cloud(const CloudSpec& c, const ParamLite& q) {
  Cloud cd;
  const int pmode = q.select == HAV_SELECT_CENTRE ? 1 : (q.select == HAV_SELECT_MEAN ? 2 : 0);
  const Layout L = make_layout(c.n_cap, q.depth, q.tscale, pmode);
  cd.w = make_ws(c.seg, L, c.n);
  cd.w.xyz = c.xyz;
  cd.w.xyz_out = c.xyz_out;
  cd.w.idx = c.idx;
  cd.w.info_dev = c.info;
  cd.w.M = c.m;
  Plan& P = cd.P;
  P.t_max = q.t_max;
  P.depth = q.depth;
  P.fixed = q.fixed;
  P.magic = magic_of(L);
  P.cap = cd.w.cap;
  P.sel_cap = sel_cap_of(cd.w.n, tab_scale(q.tscale));
  P.spec_mult = q.spec_budget ? static_cast<float>(q.spec_budget) : kSpecMult;
  P.win_sigma = q.trim_window == 0.0f ? kWinSigma : q.trim_window;
  P.select = q.select;
  P.seed = q.seed;
  P.identity = c.m == c.n ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    P.aspect[a] = q.aspect[a];
    P.fixed_v[a] = q.fixed_v[a];
  }
  int64_t m[HAV_MAX_LAYERS];
  layer_sizes(c.m, q.layers, q.ratio, m);
  int nl = 0;
  for (int l = 0; l < HAV_MAX_LAYERS; ++l) {
    P.m[l] = 0;
    P.upper[l] = 0;
    P.rounds[l] = 0;
  }
  for (int l = 0; l < q.layers; ++l) {
    if (m[l] == 0) continue;
    const double up = floor(static_cast<double>(m[l]) * (1.0 + q.sigma));
    P.m[nl] = static_cast<uint32_t>(m[l]);
    P.upper[nl] = up >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(up);
    P.rounds[nl] = P.fixed ? trim_rounds(static_cast<int64_t>(P.upper[nl])) : 0;
    ++nl;
  }
  P.nlayers = nl;
  return cd;
}

// ----------------------------------------------------------------------------- batched calls

// Kernel arguments of k_setup: up to kSetupChunk clouds of a call.
constexpr int kSetupChunk = 32;
struct SetupArgs {
  BatchDev* bd;
  Cloud* clouds;
  BlockRef* bmap;
  int32_t* act;
  ParamLite q;
  int32_t B, first, count;
  int32_t kind_off[kKinds], kind_total[kKinds];
  CloudSpec cl[kSetupChunk];
};

// Every cloud's device view, and (first chunk) the batch header.
__global__ void __launch_bounds__(64) k_setup(SetupArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) a.clouds[a.first + i] = make_cloud(a.cl[i], a.q);
  if (a.first == 0 && i == 0) {
    BatchDev* bd = a.bd;
    bd->B = a.B;
    bd->depth = a.q.depth;
    bd->bshift = bin_shift(a.q.tscale);
    for (int k = 0; k < kKinds; ++k) {
      bd->kind_off[k] = a.kind_off[k];
      bd->kind_total[k] = a.kind_total[k];
    }
    bd->nact = 0;
    bd->clouds = a.clouds;
    bd->bmap = a.bmap;
    bd->act = a.act;
    bd->nfin[0] = 0;
    bd->err[0] = 0;
  }
}

// Block map of every grid kind (block k of this kernel builds kind k): for each cloud
// in order, its blocks (cloud, block within the cloud, the cloud's block count).
__global__ void __launch_bounds__(kThreads) k_map(BatchDev* bd) {
  __shared__ uint32_t s_tmp[kThreads / 64];
  const int kind = blockIdx.x;
  const int B = bd->B;
  BlockRef* out = bd->bmap + bd->kind_off[kind];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < B; c0 += kThreads) {
    const int c = c0 + threadIdx.x;
    const uint32_t nb = c < B ? static_cast<uint32_t>(blocks_of(kind, bd->clouds[c].w.n, bd->bshift)) : 0u;
    uint32_t ex;
    const uint32_t tot = block_exclusive_scan<kThreads>(nb, &ex, s_tmp);
    for (uint32_t b = 0; b < nb; ++b) {
      BlockRef r;
      r.c = c;
      r.b = static_cast<int32_t>(b);
      r.nb = static_cast<int32_t>(nb);
      r.pad = 0;
      out[carry + ex + b] = r;
    }
    carry += tot;
    __syncthreads();
  }
}

// The clouds that search in layer L (in cloud order), and the batch's search counters.
__global__ void __launch_bounds__(kThreads) k_search_prep(Many src, int L) {
  __shared__ uint32_t s_tmp[kThreads / 64];
  BatchDev* bd = src.bd;
  const int B = bd->B;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < B; c0 += kThreads) {
    const int c = c0 + threadIdx.x;
    uint32_t on = 0;
    if (c < B) {
      const Cloud& cd = bd->clouds[c];
      on = layer_due(cd, L) && !cd.P.fixed ? 1u : 0u;
    }
    uint32_t ex;
    const uint32_t tot = block_exclusive_scan<kThreads>(on, &ex, s_tmp);
    if (on) bd->act[carry + ex] = c;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bd->nact = static_cast<int32_t>(carry);
    bd->nfin[0] = 0;
    bd->err[0] = 0;
  }
}

// The voxel searches of every cloud of a batch in one launch. Each cloud keeps its
// own ticket queue and controller (as in k_search). A block picks, among the searching
// clouds (starting from a rotating position), one whose current pass still has tiles
// to hand out, takes a ticket there and runs it. Waits are only for tiles that running
// blocks hold, so any grid size makes progress.
__global__ void __launch_bounds__(kThreads) k_search_many(Many src, int L) {
  BatchDev* bd = src.bd;
  const int nact = bd->nact;
  if (nact == 0) return;
  extern __shared__ uint64_t lds[];
  __shared__ SearchShared S;
  uint64_t *lvals, *lkeys;
  search_lds_init(lds, bd->depth, lvals, lkeys);
  int cur_c = -1, cur_p = -1;  // cloud and pass whose state S.st holds
  int start = static_cast<int>(blockIdx.x) % nact;
  float4 pt[kPerThread];
  while (true) {
    __syncthreads();  // every thread has read the previous ticket's shared fields
    if (threadIdx.x < 64) {
      // wave 0: lane k looks at searching cloud start + k (+ 64 j)
      const int lane = threadIdx.x;
      uint32_t spins = 0;
      const uint32_t limit = g_search_spin_limit;
      while (true) {
        int pick = -1;
        for (int base = 0; base < nact && pick < 0; base += 64) {
          const int k = base + lane;
          int c = -1;
          bool avail = false;
          if (k < nact) {
            c = bd->act[(start + k) % nact];
            Header* hc = bd->clouds[c].w.h;
            const uint32_t nt = static_cast<uint32_t>(bd->clouds[c].w.ntile);
            const uint32_t gen = ld_agent(&hc->sq_gen[0]);
            const uint32_t tk = ld_agent(&hc->sq_ticket[0]);
            const uint32_t fin = ld_agent(&hc->sq_fin[0]);
            avail = !fin && tk < (gen + 1) * nt;
          }
          const uint64_t bal = __ballot(avail);
          if (bal) pick = __shfl(c, static_cast<int>(__ffsll(static_cast<long long>(bal)) - 1), 64);
        }
        if (pick >= 0) {
          if (lane == 0) {
            Header* hc = bd->clouds[pick].w.h;
            const uint32_t nt = static_cast<uint32_t>(bd->clouds[pick].w.ntile);
            const uint32_t t = atomicAdd(&hc->sq_ticket[0], 1u);
            S.cloud = pick;
            S.pass = static_cast<int>(t / nt);
            S.tile = static_cast<int>(t % nt);
            S.go = 1;
          }
          break;
        }
        if (ld_agent(&bd->nfin[0]) >= static_cast<uint32_t>(nact) || ld_agent(&bd->err[0])) {
          if (lane == 0) S.go = 0;
          break;
        }
        if (++spins > limit) {
          if (lane == 0) {
            atomicOr(&bd->err[0], 1u);
            S.go = 0;
          }
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
    if (!S.go) break;
    const int c = S.cloud, p = S.pass, tile = S.tile;
    start = (start + 1) % nact;
    const Cloud& cd = bd->clouds[c];
    const Ws& w = cd.w;
    const Plan& P = cd.P;
    Header* h = w.h;
    if (p >= P.t_max) continue;  // a ticket past the last possible pass
    uint32_t tg[kPerThread];
    issue_tile(w, tile, pt, tg);
    if (c != cur_c || p != cur_p) {
      if (threadIdx.x == 0) S.go = wait_pass(h, p, &bd->err[0]);
      __syncthreads();
      if (S.go < 0) break;
      if (S.go == 0) continue;  // that cloud's search has ended: drop the ticket
      if (threadIdx.x < kPubWords)
        reinterpret_cast<uint32_t*>(&S.st)[threadIdx.x] =
            ld_agent(p == 0 ? &h->pub_first[L][threadIdx.x] : &h->pub[threadIdx.x]);
      __syncthreads();
      cur_c = c;
      cur_p = p;
    }
    const int r = run_ticket(w, P, S, lvals, lkeys, pt, tg, p, tile, tile, w.ntile, -1);
    if (r == kTicketPublished) cur_p = p + 1;
    if (r == kTicketFinished) {
      if (threadIdx.x == 0) atomicAdd(&bd->nfin[0], 1u);
      cur_c = -1;
    }
  }
  if (threadIdx.x == 0 && ld_agent(&bd->err[0]))
    for (int k = 0; k < nact; ++k) mark_search_failed(bd->clouds[bd->act[k]].w.h);
}

int grid_for(int64_t work) {
  const int64_t g = (work + kThreads - 1) / kThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, 4096)));
}


// Blocks of a search launch: one per tile, at most as many as the device holds at
// once (more would only wait for tickets). The limit is cached per device, kernel
// (single or batched) and depth.
int search_grid(int ntile, int depth, bool many, int requested) {
  if (requested > 0) return std::min(requested, std::max(1, ntile));
  static std::atomic<int> cache[kMaxDevices][2][kMaxDepth + 1];
  int dev = 0;
  int cap = 1024;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
    int c = cache[dev][many][depth].load(std::memory_order_relaxed);
    if (c == 0) {
      const size_t lds = 2 * static_cast<size_t>(depth) * kBrickCap * sizeof(uint64_t);
      int per_cu = 0, cus = 0;
      const void* fn = many ? reinterpret_cast<const void*>(&k_search_many)
                            : reinterpret_cast<const void*>(&k_search);
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          per_cu > 0 && cus > 0)
        c = per_cu * cus;
      else
        c = cap;
      cache[dev][many][depth].store(c, std::memory_order_relaxed);
    }
    cap = c;
  }
  return std::max(1, std::min(ntile, cap));
}

// Kernel timing for measurement (hav_timing_enable): a pair of HIP events on the
// launch stream around every launch, kept until hav_timing_collect reads them.
struct TimedLaunch {
  const char* name;
  hipEvent_t e0, e1;
};
std::mutex g_timing_mu;
std::atomic<int> g_timing_on{0};
std::vector<TimedLaunch> g_timed;

hipEvent_t timing_mark(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return nullptr;  // nothing is timed while a stream records a graph
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, st) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void timing_keep(const char* name, hipEvent_t e0, hipEvent_t e1) {
  if (!e0 || !e1) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return;
  }
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timed.push_back({name, e0, e1});
}

#define HAV_LAUNCH(kern, grid, block, lds, st, ...)                              \
  do {                                                                           \
    const bool tm_ = g_timing_on.load(std::memory_order_relaxed) != 0;           \
    hipEvent_t e0_ = tm_ ? timing_mark(st) : nullptr;                            \
    hipLaunchKernelGGL(kern, grid, block, lds, st, __VA_ARGS__);                 \
    if (hipGetLastError() != hipSuccess) {                                       \
      if (e0_) (void)hipEventDestroy(e0_);                                       \
      return HAV_ERR_HIP;                                                        \
    }                                                                            \
    if (tm_) timing_keep(#kern, e0_, timing_mark(st));                           \
  } while (0)

hav_status_t run_stage(const float* xyz, int64_t N, int64_t M, const hav_params_t* p, int32_t* idx,
                       char* ws, const Layout& L, hav_info_t* info_dev, hipStream_t st,
                       float* xyz_out = nullptr) {
  const CloudSpec spec{xyz, idx, info_dev, ws, N, M, L.n_ws, xyz_out};
  const One one{make_cloud(spec, lite_of(p))};
  const Ws& w = one.c.w;
  const Plan& P = one.c.P;
  HAV_LAUNCH(k_bbox<One>, dim3(w.nbbox), dim3(kThreads), 0, st, one);
  if (P.identity) {
    HAV_LAUNCH(k_identity<One>, dim3(w.nscan), dim3(kThreads), 0, st, one);
    return HAV_OK;
  }
  HAV_LAUNCH(k_bin_count<One>, dim3(w.nbb), dim3(CountThreads<One>::value), 0, st, one);
  HAV_LAUNCH(k_bin_scan<One>, dim3(kBinChunks / scan_group(w.nbb)), dim3(kThreads), 0, st, one);
  if (w.nbb <= 256)
    HAV_LAUNCH((k_bin_scatter<One, 2 * kThreads>), dim3(w.nbb + 1), dim3(2 * kThreads), 0, st, one);
  else
    HAV_LAUNCH((k_bin_scatter<One, kThreads>), dim3(w.nbb + 1), dim3(kThreads), 0, st, one);
  // a cloud of few tiles splits each tile's candidates over tickets of their own, so that
  // more blocks share a pass (each holds one candidate's LDS tables)
  const int split = w.ntile * P.depth <= kSplitTickets ? P.depth : 1;
  const int sdepth = split > 1 ? 1 : P.depth;
  const int sgrid = search_grid(w.ntile * split, sdepth, false, p->search_blocks);
  const size_t eval_lds = 2 * static_cast<size_t>(sdepth) * kBrickCap * sizeof(uint64_t);
  const size_t sel_lds = 2 * static_cast<size_t>(kLdsCap) * sizeof(uint64_t);
  for (int l = 0; l < P.nlayers; ++l) {
    if (!P.fixed) HAV_LAUNCH(k_search, dim3(sgrid), dim3(kThreads), eval_lds, st, one, l, split);
    HAV_LAUNCH(k_select<One>, dim3(w.ntile), dim3(kThreads), sel_lds, st, one, l);
    if (w.pmode == 2) HAV_LAUNCH(k_mean, dim3(w.ntile), dim3(kThreads), 0, st, one, l);
    for (int r = 0; r < P.rounds[l]; ++r)
      HAV_LAUNCH(k_trim_hist<One>, dim3(w.ntile), dim3(kThreads), 0, st, one, l, r);
    HAV_LAUNCH(k_mark<One>, dim3(w.ntile), dim3(kThreads), 0, st, one, l);
  }
  HAV_LAUNCH(k_out<One>, dim3(w.nscan), dim3(kThreads), 0, st, one);
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
  Layout stage;
  size_t buf0 = 0, buf1 = 0, local = 0, total = 0;
};

ChainLayout make_chain_layout(int64_t N, const int64_t* M, int depth, int tscale) {
  ChainLayout C;
  C.stage = make_layout(N, depth, tscale);
  size_t o = align_up(C.stage.total);
  C.buf0 = o;  o = align_up(o + static_cast<size_t>(M[0]) * 12);
  C.buf1 = o;  o = align_up(o + static_cast<size_t>(M[0]) * 12);
  C.local = o; o = align_up(o + static_cast<size_t>(M[0]) * 4);
  C.total = o;
  return C;
}

// Initialise a workspace for layout L; with `only_if_needed`, a workspace already
// initialised for L (its magic matches) is left alone (one cheap launch reads the magic).
hav_status_t init_ws(char* base, const Layout& L, hipStream_t st, bool only_if_needed = false) {
  Ws w = make_ws(base, L, L.n_ws);
  const size_t nct = 2 * static_cast<size_t>(L.ncmax) * L.cap_ws;
  const size_t ncn = 2 * static_cast<size_t>(L.ncmax) * L.ntile_ws;
  HAV_LAUNCH(k_ws_init, dim3(only_if_needed ? 512 : 2048), dim3(kThreads), 0, st, w, nct, ncn,
             static_cast<size_t>(L.cap_ws), static_cast<size_t>(L.sel_ws),
             static_cast<size_t>(L.ntile_ws),
             2 * static_cast<size_t>(L.ncmax) * kReps * kHotCap, static_cast<size_t>(L.nscan_ws),
             L.pmode == 2 ? static_cast<size_t>(L.sel_ws) : size_t(0),
             only_if_needed ? magic_of(L) : uint64_t(0));
  HAV_LAUNCH(k_ws_seal, dim3(1), dim3(64), 0, st, w.h, magic_of(L));
  return HAV_OK;
}

// ----------------------------------------------------------------------------- static workspace

// The workspace of hav_sample_static: one per device, in the library's own device memory,
// laid out for kStaticPoints points at any N up to that (so calls of different sizes
// share one initialisation). Host code never passes `scratch` itself to a kernel: its
// name is a host-side stand-in; the device address comes from hipGetSymbolAddress, once
// per device (static_ptr).
constexpr int64_t kStaticPoints = HAV_STATIC_MAX_POINTS;
constexpr size_t kStaticBytes = HAV_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

char* static_ptr(int dev) {
  static std::once_flag once[kMaxDevices];
  static char* ptr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(once[dev], [dev]() {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) ptr[dev] = static_cast<char*>(p);
  });
  return ptr[dev];
}

// ----------------------------------------------------------------------------- batched host side

constexpr int32_t kMaxBatch = 4096;
static_assert(sizeof(SetupArgs) <= 3072, "k_setup arguments");

// A batched call's region: header, cloud views, block maps, searching-cloud list.
struct BatchLayout {
  size_t bd = 0, clouds = 0, bmap = 0, act = 0, total = 0;
  int32_t kind_off[kKinds] = {}, kind_total[kKinds] = {};
};

BatchLayout make_batch_layout(int32_t B, const int64_t* n, int bshift) {
  BatchLayout BL;
  int64_t off = 0;
  for (int k = 0; k < kKinds; ++k) {
    int64_t t = 0;
    for (int32_t i = 0; i < B; ++i) t += blocks_of(k, n[i], bshift);
    BL.kind_off[k] = static_cast<int32_t>(off);
    BL.kind_total[k] = static_cast<int32_t>(t);
    off += t;
  }
  size_t o = 0;
  BL.bd = o;     o = align_up(o + sizeof(BatchDev));
  BL.clouds = o; o = align_up(o + static_cast<size_t>(B) * sizeof(Cloud));
  BL.bmap = o;   o = align_up(o + static_cast<size_t>(off) * sizeof(BlockRef));
  BL.act = o;    o = align_up(o + static_cast<size_t>(B) * 4);
  BL.total = o;
  return BL;
}

// All kernels of one stage for B clouds at once. `region` holds the BatchLayout;
// every spec has its own initialised segment.
hav_status_t run_batch(const CloudSpec* specs, int32_t B, const hav_params_t* p, char* region,
                       const BatchLayout& BL, hipStream_t st) {
  const ParamLite q = lite_of(p);
  BatchDev* bd = reinterpret_cast<BatchDev*>(region + BL.bd);
  Cloud* clouds = reinterpret_cast<Cloud*>(region + BL.clouds);
  BlockRef* bmap = reinterpret_cast<BlockRef*>(region + BL.bmap);
  int32_t* act = reinterpret_cast<int32_t*>(region + BL.act);
  int max_layers = 0, max_rounds = 0;
  bool any_identity = false, any_work = false, any_search = false;
  for (int32_t i = 0; i < B; ++i) {
    const Cloud cd = make_cloud(specs[i], q);
    if (cd.P.identity) {
      any_identity = true;
      continue;
    }
    any_work = true;
    any_search |= !cd.P.fixed;
    max_layers = std::max(max_layers, cd.P.nlayers);
    for (int l = 0; l < cd.P.nlayers; ++l) max_rounds = std::max(max_rounds, cd.P.rounds[l]);
  }
  for (int32_t first = 0; first < B; first += kSetupChunk) {
    SetupArgs a;
    std::memset(&a, 0, sizeof(a));
    a.bd = bd;
    a.clouds = clouds;
    a.bmap = bmap;
    a.act = act;
    a.q = q;
    a.B = B;
    a.first = first;
    a.count = std::min<int32_t>(kSetupChunk, B - first);
    for (int k = 0; k < kKinds; ++k) {
      a.kind_off[k] = BL.kind_off[k];
      a.kind_total[k] = BL.kind_total[k];
    }
    for (int32_t i = 0; i < a.count; ++i) a.cl[i] = specs[first + i];
    HAV_LAUNCH(k_setup, dim3(1), dim3(64), 0, st, a);
  }
  HAV_LAUNCH(k_map, dim3(kKinds), dim3(kThreads), 0, st, bd);
  const Many many{bd};
  const int* T = BL.kind_total;
  HAV_LAUNCH(k_bbox<Many>, dim3(T[kKBBox]), dim3(kThreads), 0, st, many);
  if (any_identity) HAV_LAUNCH(k_identity<Many>, dim3(T[kKScan]), dim3(kThreads), 0, st, many);
  if (!any_work) return HAV_OK;
  HAV_LAUNCH(k_bin_count<Many>, dim3(T[kKBin]), dim3(CountThreads<Many>::value), 0, st, many);
  HAV_LAUNCH(k_bin_scan<Many>, dim3(T[kKBScan]), dim3(kThreads), 0, st, many);
  HAV_LAUNCH((k_bin_scatter<Many, kThreads>), dim3(T[kKScat]), dim3(kThreads), 0, st, many);
  const int sgrid = search_grid(T[kKTile], q.depth, true, p->search_blocks);
  const size_t eval_lds = 2 * static_cast<size_t>(q.depth) * kBrickCap * sizeof(uint64_t);
  const size_t sel_lds = 2 * static_cast<size_t>(kLdsCap) * sizeof(uint64_t);
  for (int l = 0; l < max_layers; ++l) {
    if (any_search) {
      HAV_LAUNCH(k_search_prep, dim3(1), dim3(kThreads), 0, st, many, l);
      HAV_LAUNCH(k_search_many, dim3(sgrid), dim3(kThreads), eval_lds, st, many, l);
    }
    HAV_LAUNCH(k_select<Many>, dim3(T[kKTile]), dim3(kThreads), sel_lds, st, many, l);
    for (int r = 0; r < max_rounds; ++r)
      HAV_LAUNCH(k_trim_hist<Many>, dim3(T[kKTile]), dim3(kThreads), 0, st, many, l, r);
    HAV_LAUNCH(k_mark<Many>, dim3(T[kKTile]), dim3(kThreads), 0, st, many, l);
  }
  HAV_LAUNCH(k_out<Many>, dim3(T[kKScan]), dim3(kThreads), 0, st, many);
  return HAV_OK;
}

// Workspace of hav_sample_batch: the batch region, then one segment per cloud.
struct BatchWsLayout {
  BatchLayout BL;
  std::vector<size_t> seg;
  size_t total = 0;
};

bool batch_args_ok(int32_t B, const int64_t* N, const int64_t* M) {
  if (B < 1 || B > kMaxBatch || !N) return false;
  for (int32_t i = 0; i < B; ++i) {
    if (N[i] < 1 || N[i] > kMaxPoints) return false;
    if (M && (M[i] < 1 || M[i] > N[i])) return false;
  }
  return true;
}

BatchWsLayout make_batch_ws_layout(int32_t B, const int64_t* N, int depth, int tscale) {
  BatchWsLayout W;
  W.BL = make_batch_layout(B, N, bin_shift(tscale));
  size_t o = align_up(W.BL.total);
  W.seg.resize(static_cast<size_t>(B));
  for (int32_t i = 0; i < B; ++i) {
    W.seg[i] = o;
    o = align_up(o + make_layout(N[i], depth, tscale).total);
  }
  W.total = o;
  return W;
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
  p.spec_depth = 0;
  p.spec_budget = 0;
  p.search_blocks = 0;
  p.trim_window = 0.0f;
  p.select = HAV_SELECT_CENTRE_CLOSEST;
  p.select_seed = 0;
  p.table_scale = 0;
  p.bin_points = 0;
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
    case HAV_ERR_WORKSPACE_NOT_INIT: return "workspace not initialised for this size";
    case HAV_NOT_READY: return "not ready";
  }
  return "unknown status";
}

size_t hav_workspace_size(int64_t N, int64_t M, const hav_params_t* params) {
  if (N < 1 || M < 1 || M > N || N > kMaxPoints || !params_any_ok(params)) return 0;
  return make_layout(N, depth_of(params), tscale_of(params), points_mode(params)).total;
}

hav_status_t hav_workspace_init(int64_t N, const hav_params_t* params, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!ws || N < 1 || N > kMaxPoints || !params_any_ok(params)) return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const Layout L = make_layout(N, depth_of(params), tscale_of(params), points_mode(params));
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  return init_ws(static_cast<char*>(ws), L, static_cast<hipStream_t>(stream));
}

hav_status_t hav_sample(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                        int32_t* idx, void* ws, size_t ws_bytes, hav_info_t* info_dev,
                        void* stream) {
  if (!xyz || !idx || !ws || N < 1 || M < 1 || M > N || N > kMaxPoints ||
      !params_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const Layout L = make_layout(N, depth_of(params), tscale_of(params));
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  return run_stage(xyz, N, M, params, idx, static_cast<char*>(ws), L, info_dev,
                   static_cast<hipStream_t>(stream));
}

hav_status_t hav_sample_static(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                               int32_t* idx, hav_info_t* info_dev, void* stream) {
  if (!xyz || !idx || N < 1 || M < 1 || M > N || N > kMaxPoints || !params_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (N > kStaticPoints) return HAV_ERR_WORKSPACE_TOO_SMALL;
  const Layout L = make_layout(kStaticPoints, depth_of(params), tscale_of(params));
  if (L.total > kStaticBytes) return HAV_ERR_WORKSPACE_TOO_SMALL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HAV_ERR_HIP;
  char* ws = static_ptr(dev);
  if (!ws) return HAV_ERR_HIP;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  // (re)initialised on the device when it holds another layout, or none yet, or a call
  // that gave up left it dirty; else left as the last call left it
  const hav_status_t s = init_ws(ws, L, st, true);
  if (s != HAV_OK) return s;
  return run_stage(xyz, N, M, params, idx, ws, L, info_dev, st);
}

hav_status_t hav_sample_points(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                               int32_t* idx, float* xyz_out, void* ws, size_t ws_bytes,
                               hav_info_t* info_dev, void* stream) {
  if (!xyz || !idx || !xyz_out || !ws || N < 1 || M < 1 || M > N || N > kMaxPoints ||
      !params_any_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const Layout L = make_layout(N, depth_of(params), tscale_of(params), points_mode(params));
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  return run_stage(xyz, N, M, params, idx, static_cast<char*>(ws), L, info_dev,
                   static_cast<hipStream_t>(stream), xyz_out);
}

}  // extern "C"

namespace {
// A kept launch name ("k_select<One>", or "(k_bin_scatter<One, 2 * kThreads>)" where the
// template arguments hold a comma) matches the plain kernel name.
bool same_kernel(const char* kept, const char* name) {
  if (kept[0] == '(') ++kept;
  size_t i = 0;
  for (; name[i] && kept[i] == name[i]; ++i) {
  }
  return name[i] == 0 && (kept[i] == 0 || kept[i] == '<');
}
}  // namespace

extern "C" {

size_t hav_batch_workspace_size(int32_t B, const int64_t* N_host, const int64_t* M_host,
                                const hav_params_t* params) {
  if (!batch_args_ok(B, N_host, M_host) || !params_ok(params)) return 0;
  return make_batch_ws_layout(B, N_host, depth_of(params), tscale_of(params)).total;
}

hav_status_t hav_batch_workspace_init(int32_t B, const int64_t* N_host, const hav_params_t* params,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!ws || !batch_args_ok(B, N_host, nullptr) || !params_ok(params)) return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const int depth = depth_of(params);
  const BatchWsLayout W = make_batch_ws_layout(B, N_host, depth, tscale_of(params));
  if (ws_bytes < W.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  char* base = static_cast<char*>(ws);
  for (int32_t i = 0; i < B; ++i) {
    const hav_status_t s = init_ws(base + W.seg[i], make_layout(N_host[i], depth, tscale_of(params)),
                                   static_cast<hipStream_t>(stream));
    if (s != HAV_OK) return s;
  }
  return HAV_OK;
}

hav_status_t hav_sample_batch(const float* xyz_concat, const int64_t* offsets_host,
                              const int64_t* M_host, int32_t B, const hav_params_t* params,
                              int32_t* idx_concat, void* ws, size_t ws_bytes, hav_info_t* info_dev,
                              void* stream) {
  if (!xyz_concat || !offsets_host || !M_host || !idx_concat || !ws || B < 1 || B > kMaxBatch ||
      !params_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  if (offsets_host[0] != 0) return HAV_ERR_INVALID_ARG;
  std::vector<int64_t> N(static_cast<size_t>(B));
  for (int32_t i = 0; i < B; ++i) N[i] = offsets_host[i + 1] - offsets_host[i];
  if (!batch_args_ok(B, N.data(), M_host)) return HAV_ERR_INVALID_ARG;
  const int depth = depth_of(params);
  const BatchWsLayout W = make_batch_ws_layout(B, N.data(), depth, tscale_of(params));
  if (ws_bytes < W.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  char* base = static_cast<char*>(ws);
  std::vector<CloudSpec> specs(static_cast<size_t>(B));
  int64_t mo = 0;
  for (int32_t i = 0; i < B; ++i) {
    specs[i] = CloudSpec{xyz_concat + 3 * offsets_host[i], idx_concat + mo,
                         info_dev ? info_dev + i : nullptr, base + W.seg[i], N[i], M_host[i], N[i],
                         nullptr};
    mo += M_host[i];
  }
  return run_batch(specs.data(), B, params, base, W.BL, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// Resident blocks of the grouping kernel on the current device: its grid (the blocks
// take work items until none is left).
int ball_blocks() {
  static std::atomic<int> cache[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_ball_group),
                                                     kBallThreads, 0) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        per_cu > 0 && cus > 0)
      c = per_cu * cus;
    else
      c = 256;
    cache[dev].store(c, std::memory_order_relaxed);
  }
  return c;
}

struct hav_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

hav_status_t hav_graph_capture_begin(void* stream) {
  if (!stream) return HAV_ERR_INVALID_ARG;
  return hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal) ==
                 hipSuccess
             ? HAV_OK
             : HAV_ERR_HIP;
}

hav_status_t hav_graph_capture_end(void* stream, hav_graph_t** out) {
  if (!stream || !out) return HAV_ERR_INVALID_ARG;
  *out = nullptr;
  auto g = new hav_graph();
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g->graph) != hipSuccess || !g->graph) {
    delete g;
    return HAV_ERR_HIP;
  }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return HAV_ERR_HIP;
  }
  *out = g;
  return HAV_OK;
}

hav_status_t hav_graph_launch(hav_graph_t* g, void* stream) {
  if (!g) return HAV_ERR_INVALID_ARG;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? HAV_OK
                                                                                : HAV_ERR_HIP;
}

void hav_graph_destroy(hav_graph_t* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

hav_status_t hav_debug_scan_spin_limit(uint32_t limit) {
  const uint32_t v = limit ? limit : hav::kScanSpinDefault;
  return hipMemcpyToSymbol(HIP_SYMBOL(hav::g_scan_spin_limit), &v, sizeof(v)) == hipSuccess ? HAV_OK
                                                                                         : HAV_ERR_HIP;
}

hav_status_t hav_debug_search_spin_limit(uint32_t limit) {
  const uint32_t v = limit ? limit : hav::kSearchSpinDefault;
  return hipMemcpyToSymbol(HIP_SYMBOL(hav::g_search_spin_limit), &v, sizeof(v)) == hipSuccess
             ? HAV_OK
             : HAV_ERR_HIP;
}

hav_status_t hav_timing_enable(int32_t on) {
  g_timing_on.store(on ? 1 : 0, std::memory_order_relaxed);
  return HAV_OK;
}

hav_status_t hav_timing_collect(const char* kernel, int32_t* launches, double* total_ms) {
  if (!kernel || !launches || !total_ms) return HAV_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  int32_t n = 0;
  double ms = 0.0;
  hav_status_t status = HAV_OK;
  std::vector<TimedLaunch> rest;
  for (const TimedLaunch& t : g_timed) {
    if (!same_kernel(t.name, kernel)) {
      rest.push_back(t);
      continue;
    }
    float e = 0.0f;
    if (hipEventSynchronize(t.e1) != hipSuccess || hipEventElapsedTime(&e, t.e0, t.e1) != hipSuccess)
      status = HAV_ERR_HIP;
    ms += e;
    ++n;
    (void)hipEventDestroy(t.e0);
    (void)hipEventDestroy(t.e1);
  }
  g_timed.swap(rest);
  *launches = n;
  *total_ms = ms;
  return status;
}

hav_status_t hav_ball_query_sampled(const float* xyz, int64_t N, const int32_t* idx, int64_t M,
                                    float radius, int32_t K, int32_t* out, int32_t* count,
                                    void* ws, size_t ws_bytes, const hav_params_t* params, void* stream) {
  if (!xyz || !idx || !out || !ws || N < 1 || N > kMaxPoints || M < 1 || M > N || K < 1 ||
      K > kBallMaxK || !(radius > 0.0f) || !std::isfinite(radius) || !params_any_ok(params))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const Layout L = make_layout(N, depth_of(params), tscale_of(params), points_mode(params));
  if (ws_bytes < L.total) return HAV_ERR_WORKSPACE_TOO_SMALL;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const Ws w = make_ws(static_cast<char*>(ws), L, N);
  const float r2 = radius * radius;
  HAV_LAUNCH(k_ball_bucket, dim3(grid_for(M)), dim3(kThreads), 0, st, w, idx, M, K, out, count);
  const int G = std::min(kBallGroup, kBallRowWords / K);
  HAV_LAUNCH(k_ball_plan, dim3(1), dim3(kBallThreads), 0, st, w, G);
  HAV_LAUNCH(k_ball_group, dim3(ball_blocks()), dim3(kBallThreads), 0, st, w, xyz, idx, radius, r2, K, out,
             count);
  return HAV_OK;
}

size_t hav_chain_workspace_size(int64_t N, const int64_t* M_host, int32_t n_stages,
                                const hav_params_t* params) {
  if (N < 1 || N > kMaxPoints || !params_ok(params) ||
      !chain_sizes_ok(N, M_host, n_stages))
    return 0;
  return make_chain_layout(N, M_host, depth_of(params), tscale_of(params)).total;
}

hav_status_t hav_sample_chain(const float* xyz, int64_t N, const int64_t* M_host,
                              int32_t n_stages, const hav_params_t* params, int32_t* idx_concat,
                              void* ws, size_t ws_bytes, hav_info_t* info_dev, void* stream) {
  if (!xyz || !idx_concat || !ws || N < 1 || N > kMaxPoints || !params_ok(params) ||
      !chain_sizes_ok(N, M_host, n_stages))
    return HAV_ERR_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return HAV_ERR_INVALID_ARG;
  const ChainLayout C = make_chain_layout(N, M_host, depth_of(params), tscale_of(params));
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
    const hav_status_t s =
        run_stage(cur, n, m, params, dst, base, C.stage, info_dev ? info_dev + j : nullptr, st);
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

#include "hav_server.inc"
