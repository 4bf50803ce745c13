/* hav.h — C ABI of the HAVSampler library (libhav.so, HIP for gfx950).
 *
 * HAVSampler is the hierarchical adaptive voxel-guided point sampler of arXiv
 * 2305.14306. A sampler S maps a cloud of n points to a subset of exactly m of them
 * (Sec. 3.1, problem formulation); this library returns the subset as indices, so
 * the sampled points are xyz[idx].
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller, unless the name
 *     says _host. The library never allocates, frees or keeps them.
 *   - `stream` is a hipStream_t (NULL = the null stream). Calls only enqueue work on
 *     it and return without synchronising; results (idx, info) are valid once the
 *     stream reaches that point.
 *   - Host-checkable argument errors return a status at once and enqueue nothing.
 *     Data-dependent errors (non-finite coordinates, a frame the 21-bit voxel
 *     coordinate cannot hold) are found on the device and reported in info->status;
 *     idx is then unspecified.
 *   - Results depend only on (xyz, M, params): never on the stream, the workspace
 *     address, the tuning fields of hav_params_t or the launch shape.
 *   - Workspace contract: a workspace is initialised once with hav_workspace_init for
 *     a size N and a speculation depth, and then belongs to the library: every call
 *     leaves it in the initialised state, so calls never clear whole tables. Do not
 *     write into it between calls (re-initialise it if you do). Two calls in flight
 *     at once need two workspaces. A call on a workspace initialised for another size
 *     reports HAV_ERR_WORKSPACE_NOT_INIT in info->status and computes nothing.
 */
#ifndef HAV_H_
#define HAV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HAV_ABI_VERSION 1
#define HAV_MAX_LAYERS 8

typedef enum {
  HAV_OK = 0,
  HAV_ERR_INVALID_ARG = 1,         /* a host-checkable argument is out of range */
  HAV_ERR_WORKSPACE_TOO_SMALL = 2, /* ws_bytes < the matching *_workspace_size() */
  HAV_ERR_OUT_OF_MEMORY = 3,       /* reserved for entry points that allocate */
  HAV_ERR_UNSUPPORTED = 4,         /* device: extent > 2^100, or a fixed voxel too small
                                      for 21-bit voxel coordinates */
  HAV_ERR_NONFINITE = 5,           /* device: a coordinate is NaN or infinite */
  HAV_ERR_HIP = 6,                 /* a HIP launch failed */
  HAV_ERR_WORKSPACE_NOT_INIT = 7,  /* device: workspace not initialised for this call's
                                      size and depth (see hav_workspace_init) */
  HAV_NOT_READY = 8                /* serving: the request has not finished yet */
} hav_status_t;

/* flags */
#define HAV_FIXED_VOXEL 1u /* use fixed_voxel[] instead of the adaptive search
                              (the "Fix" setting of the ablation, Sec. 4.5 Table 6) */

/* representative of an occupied voxel (hav_params_t.select) */
#define HAV_SELECT_CENTRE_CLOSEST 0 /* the point closest to the voxel centre, ties to the
                                       lowest index (Sec. 3.2; "CC" of Table 6) */
#define HAV_SELECT_RANDOM 1         /* a random member: the point with the smallest top 32
                                       bits of SplitMix64 output i+1 for select_seed (point
                                       i), ties to the lowest index ("RA" of Table 6) */
#define HAV_SELECT_CENTRE 2         /* the voxel's centre ("CE"), hav_sample_points only */
#define HAV_SELECT_MEAN 3           /* the mean of the voxel's points ("ME"), hav_sample_points
                                       only */

/* Sampling parameters. Start from hav_params_default(). */
typedef struct {
  int32_t abi_version; /* must be HAV_ABI_VERSION */
  int32_t layers;      /* k, hierarchical layers, 1..8; default 2 (Sec. 4.1) */
  int32_t layer_ratio; /* m_l = ratio * m_{l-1} (Sec. 3.4, Eq. 3), 2..16; default 4 */
  int32_t t_max;       /* max voxel-counter evaluations per layer (Sec. 3.3), 1..20;
                          default 20 (Sec. 4.1) */
  double sigma;        /* tolerance: accept counts in [m, floor(m (1+sigma))] (Sec. 3.3),
                          0..16; default 0.05 (Sec. 4.1) */
  float aspect[3];     /* voxel shape v = s * aspect (Sec. 3.2, v = (vx, vy, vz)),
                          each in [2^-16, 2^16]; default {1,1,1} */
  uint32_t flags;      /* HAV_FIXED_VOXEL or 0 */
  float fixed_voxel[3];/* used iff HAV_FIXED_VOXEL; each in [2^-100, 2^100] */
  int32_t spec_depth;  /* tuning only: voxel sizes one pass of the search evaluates, along
                          the bisection path a count model predicts, 1..7; 0 = library
                          default (4). Results do not depend on it; workspace size does. */
  int32_t spec_budget; /* tuning only: a pass stops its chain before a size whose predicted
                          voxel count exceeds this many times the window top; 0 = default
                          (16), else 1..1024 */
  int32_t search_blocks; /* tuning only: blocks of the voxel-search launch; 0 = as many as
                            the device holds at once (at most one per tile), else 1..65536 */
  float trim_window;   /* tuning only: half-width, in standard deviations of its expected
                          position, of the priority window the trim first tries as the bucket
                          holding its threshold; 0 = default (6), negative = no window (the
                          bucket is every voxel), else at most 64. Results do not depend on it. */
  int32_t select;      /* HAV_SELECT_CENTRE_CLOSEST (default) or HAV_SELECT_RANDOM; CENTRE and
                          MEAN with hav_sample_points and its workspace only (the workspace size
                          depends on it) */
  uint32_t select_seed;/* generator seed of HAV_SELECT_RANDOM */
  int32_t table_scale; /* tuning only: the brick and voxel tables get 2^table_scale times their
                          default slots (a power of two >= max(N, min(8N, 2^20))), so that their
                          load factor halves per step; 0..3, default 0. Changes the workspace
                          size, never a result. */
  int32_t bin_points;  /* tuning only: points each binning workgroup sorts (the spatial binning
                          that precedes the search), 2048, 4096 or 8192; 0 = default (4096).
                          Fewer points per workgroup mean more workgroups and larger binning
                          histograms. Changes the workspace size, never a result. */
} hav_params_t;

/* Per-call report, written by the device into caller memory (info_dev). */
typedef struct {
  int32_t status;   /* hav_status_t of the device-side checks */
  int32_t layers;   /* layers that ran (those with m_l > 0) */
  float hi0;        /* search bracket: smallest power of two >= the largest
                       extent/aspect of the cloud (floored at 2^-64) */
  float mn[3];      /* grid origin = per-axis minimum of the cloud */
  float mx[3];      /* per-axis maximum */
  int32_t m[HAV_MAX_LAYERS];        /* points sampled by each layer */
  float s[HAV_MAX_LAYERS];          /* chosen voxel scale (0 with HAV_FIXED_VOXEL) */
  int32_t evals[HAV_MAX_LAYERS];    /* voxel-counter evaluations made */
  int32_t count[HAV_MAX_LAYERS];    /* non-empty voxels at the chosen size */
  int32_t accepted[HAV_MAX_LAYERS]; /* 1 if the count landed in the tolerance window */
  int32_t trimmed[HAV_MAX_LAYERS];  /* voxels dropped to reach m exactly */
  int32_t padded[HAV_MAX_LAYERS];   /* extra points added to reach m exactly */
} hav_info_t;

/* Defaults of Sec. 4.1 (2 layers, sigma 0.05, t_max 20) and Sec. 3.4 (ratio 4). */
hav_params_t hav_params_default(void);

/* Static string for a status code. */
const char* hav_status_string(hav_status_t status);

/* Bytes of device workspace hav_sample needs for N points (host-only, no GPU call).
 * Depends on N and params->spec_depth. Returns 0 if the arguments are invalid. */
size_t hav_workspace_size(int64_t N, int64_t M, const hav_params_t* params);

/* Enqueue the one-time initialisation of a workspace for calls with N points (and for
 * hav_sample_chain with first-stage size N) and params->spec_depth. ws is device
 * memory of ws_bytes >= hav_workspace_size (or hav_chain_workspace_size), 256-byte
 * aligned, arbitrary contents. Needed again only after the caller writes into the
 * workspace or to switch N / depth. */
hav_status_t hav_workspace_init(int64_t N, const hav_params_t* params, void* ws, size_t ws_bytes,
                                void* stream);

/* Sample exactly M of the N points (Sec. 3, Eq. 3 with AVS of Sec. 3.3 and the
 * centre-closest selection of Sec. 3.2).
 *   xyz    [N][3] float32, row-major (x, y, z per point), device.
 *   N, M   1 <= M <= N <= 2^30 - 1.
 *   idx    [M] int32, device: the picked indices in ascending order.
 *   ws     device workspace of ws_bytes >= hav_workspace_size(N, M, params),
 *          256-byte aligned, initialised by hav_workspace_init(N, params, ...).
 *   info_dev  device hav_info_t or NULL.
 * M == N gives 0..N-1. Returns HAV_OK once the work is enqueued. */
hav_status_t hav_sample(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                        int32_t* idx, void* ws, size_t ws_bytes, hav_info_t* info_dev,
                        void* stream);

/* ---- Sampling without a caller workspace, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as hav_sample, minus the workspace: the call uses a
 * workspace the library holds in its own device memory, one per device (a static array
 * of HAV_STATIC_WORKSPACE_BYTES, held by each GPU the library runs on until the process
 * ends). The call allocates nothing: it (re)initialises that workspace on the device
 * when it holds another layout or was left dirty by a call that gave up, then samples.
 *   N  1 <= M <= N <= HAV_STATIC_MAX_POINTS; a larger N, or tuning fields whose workspace
 *      does not fit the array (spec_depth above 5 or table_scale above 0), return
 *      HAV_ERR_WORKSPACE_TOO_SMALL at once and enqueue nothing.
 * Every call on a device shares that device's workspace: calls that overlap on one
 * device (two streams, two threads) race and give undefined results; serialise them. */
#define HAV_STATIC_MAX_POINTS 32768
#define HAV_STATIC_WORKSPACE_BYTES (64u << 20)
hav_status_t hav_sample_static(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                               int32_t* idx, hav_info_t* info_dev, void* stream);

/* Workspace for hav_sample_chain with stage sizes M_host[0..n_stages-1]; initialise it
 * with hav_workspace_init(N, params, ...). */
size_t hav_chain_workspace_size(int64_t N, const int64_t* M_host, int32_t n_stages,
                                const hav_params_t* params);

/* Chained down-sampling (the stage-wise "progressively downsamples" use of Sec. 3.1;
 * Fig. 7 times three chained steps): stage j samples M_host[j] points of the cloud
 * stage j-1 produced, i.e. of xyz[idx_{j-1}] taken in ascending index order.
 *   M_host  host array, N >= M_host[0] >= M_host[1] >= ... >= 1.
 *   idx_concat  [sum M_host] int32, device: stage j's picks as ORIGINAL indices
 *               (ascending), stage after stage.
 *   info_dev  device hav_info_t[n_stages] or NULL. */
hav_status_t hav_sample_chain(const float* xyz, int64_t N, const int64_t* M_host,
                              int32_t n_stages, const hav_params_t* params, int32_t* idx_concat,
                              void* ws, size_t ws_bytes, hav_info_t* info_dev, void* stream);

/* ---- Batched calls: many clouds of uneven size in one launch sequence.
 * Every kernel of the stage runs once for the whole batch: one grid covers the tiles
 * of all clouds, each cloud keeps its own workspace segment, voxel search controller
 * and output, and the result of each cloud is the one hav_sample gives it alone. */

/* Bytes of workspace for a batch of B clouds of N_host[i] points (M_host may be NULL
 * when only the size is wanted; else each 1 <= M_host[i] <= N_host[i]). 0 if the
 * arguments are invalid. 1 <= B <= 4096, 1 <= N_host[i] <= 2^30 - 1. */
size_t hav_batch_workspace_size(int32_t B, const int64_t* N_host, const int64_t* M_host,
                                const hav_params_t* params);

/* One-time initialisation of a batch workspace for clouds of N_host[i] points (same
 * contract as hav_workspace_init, per cloud segment). */
hav_status_t hav_batch_workspace_init(int32_t B, const int64_t* N_host, const hav_params_t* params,
                                      void* ws, size_t ws_bytes, void* stream);

/* Sample M_host[i] of the points of each cloud i of a batch.
 *   xyz_concat    [sum N][3] float32, device: cloud i is rows offsets_host[i] ..
 *                 offsets_host[i+1]-1.
 *   offsets_host  host, B+1 entries, offsets_host[0] = 0, non-decreasing.
 *   M_host        host, B entries.
 *   idx_concat    [sum M] int32, device: cloud i's picks as indices into cloud i
 *                 (0-based, ascending), at offset M_host[0] + ... + M_host[i-1].
 *   ws            initialised with hav_batch_workspace_init for the same N.
 *   info_dev      device hav_info_t[B] or NULL. */
hav_status_t hav_sample_batch(const float* xyz_concat, const int64_t* offsets_host,
                              const int64_t* M_host, int32_t B, const hav_params_t* params,
                              int32_t* idx_concat, void* ws, size_t ws_bytes, hav_info_t* info_dev,
                              void* stream);

/* ---- Serving loop (continuous batching).
 * A server owns device memory within an HBM budget: per-request slots in capacity
 * classes of 2^k points (4,096 .. 16,777,216), each keeping its workspace initialised on
 * the device for its life, and one batch region per stream. A worker thread admits
 * submitted requests in arrival order as slots become free (a request that does not fit
 * yet lets smaller ones behind it pass; idle slots of other classes are released when
 * the budget needs the room), and launches every admitted request in the next batch on
 * a free stream, so up to `streams` batches overlap on the device. Each result equals
 * what hav_sample gives the same cloud alone. Latency is measured from submit to the
 * worker seeing the batch complete (host steady clock). */
typedef struct hav_server hav_server_t;

typedef struct {
  int64_t submitted, completed, batches, max_batch_seen;
  int64_t slots, slots_created, evictions, points_done;
  uint64_t hbm_used; /* bytes of device memory the server holds */
} hav_server_stats_t;

/* Create a server on the current device. max_batch 1..1024 requests per launch,
 * streams 1..8 batches in flight. NULL on invalid arguments or if the batch regions
 * cannot be allocated (this entry point allocates device and pinned host memory). */
hav_server_t* hav_server_create(size_t hbm_budget_bytes, int32_t max_batch, int32_t streams,
                                const hav_params_t* params);

/* Queue a request: N points at xyz_host_pinned ([N][3] float32 in pinned host memory that
 * stays valid and unchanged until the request completes), sample M. Writes a ticket.
 * HAV_ERR_OUT_OF_MEMORY if one slot of its class cannot fit the budget. */
hav_status_t hav_server_submit(hav_server_t* server, const float* xyz_host_pinned, int64_t N,
                               int64_t M, uint64_t* ticket);

/* HAV_NOT_READY while the request runs. Once it has finished: copies the M ascending
 * indices to idx_host (if not NULL and the request succeeded), its report to info_host
 * and its latency in milliseconds, forgets the ticket and returns the request's status. */
hav_status_t hav_server_poll(hav_server_t* server, uint64_t ticket, int32_t* idx_host,
                             hav_info_t* info_host, double* latency_ms);

hav_status_t hav_server_stats(hav_server_t* server, hav_server_stats_t* out);

/* Finish the batches in flight, drop requests not yet admitted, free everything. */
void hav_server_destroy(hav_server_t* server);

/* ---- HIP graphs of library calls.
 * Library calls only enqueue kernels (no host synchronisation, allocation or memset on
 * the stream), so a sequence of calls can be recorded once and replayed: begin capture
 * on a stream that is not the null stream, make the calls on it (they are recorded,
 * not run), end the capture to get an instantiated graph, and launch it any number of
 * times. A replay reads and writes exactly the buffers the recorded calls named, and
 * gives the same results as the calls. The workspaces involved must be initialised
 * before the capture. */
typedef struct hav_graph hav_graph_t;
hav_status_t hav_graph_capture_begin(void* stream);
hav_status_t hav_graph_capture_end(void* stream, hav_graph_t** graph);
hav_status_t hav_graph_launch(hav_graph_t* graph, void* stream);
void hav_graph_destroy(hav_graph_t* graph);

/* Test hook for the failure path of the tag scans (for tests, not for callers). Sets,
 * for the current device, how many polls a scan block makes for the counts of the blocks
 * before it before it gives up (default 1 << 22; `limit` = 0 restores it). A call whose
 * scan gives up reports HAV_ERR_HIP in info->status; every block still finishes and the
 * workspace stays usable. Synchronous; affects calls issued after it returns.
 * Returns HAV_ERR_HIP if the device copy fails. */
hav_status_t hav_debug_scan_spin_limit(uint32_t limit);

/* Test hook for the failure path of the voxel search (for tests, not for callers). Sets,
 * for the current device, how many polls a search block makes while it waits for the
 * pass it holds a ticket of to be published, before it gives up (default 1 << 22;
 * `limit` = 0 restores it). A search that gives up reports HAV_ERR_HIP in info->status
 * and leaves its workspace needing hav_workspace_init again (a batch marks every cloud
 * that was searching); every block still finishes. Synchronous; affects calls issued
 * after it returns. Returns HAV_ERR_HIP if the device copy fails. */
hav_status_t hav_debug_search_spin_limit(uint32_t limit);

/* Measurement support. While enabled (on != 0), every kernel launch the library makes
 * is bracketed by a pair of HIP events recorded on the call's stream; the events are
 * kept by the library. Off by default; timing adds the event records to the stream. */
hav_status_t hav_timing_enable(int32_t on);

/* Wait for and release the kept event pairs of the kernel named `kernel` (the device
 * function's name, e.g. "k_search"; other kernels' pairs are kept). Writes the number
 * of launches and their summed duration in milliseconds. HAV_ERR_HIP if an event could
 * not be read (its duration then counts as 0). */
hav_status_t hav_timing_collect(const char* kernel, int32_t* launches, double* total_ms);

/* Voxel representatives as points: the "CE" (centre) and "ME" (mean) selections of the
 * ablation (Sec. 4.5, Table 6), whose representative of a voxel is not a cloud point.
 * The call samples exactly like hav_sample with centre-closest selection (same search,
 * trim, pad, layers and idx: the kept voxels' centre-closest points, ascending), and
 * xyz_out[j] is the point that stands for idx[j]:
 *   params->select == HAV_SELECT_CENTRE: the voxel centre mn + v * (g + 0.5), in float32
 *     as ((g + 0.5) * v) + mn, mn the cloud's min corner (the grid origin);
 *   params->select == HAV_SELECT_MEAN: the mean of the voxel's points (those not taken by
 *     an earlier layer), summed exactly in fixed point: along axis a,
 *     q = floor(r * 2^32 / H_a) with r = x - mn_a and H_a the smallest power of two >=
 *     the extent, and mean = (float)(mn_a + (sum q / n) * H_a * 2^-32) in double;
 *   CENTRE_CLOSEST / RANDOM: the point itself;
 *   a padded point (a layer with fewer voxels than m_l) stands for itself.
 *   xyz_out [M][3] float32 device. ws: hav_workspace_size(N, M, params) bytes initialised
 *   with hav_workspace_init(N, params, ...) (the points modes need more workspace). Errors
 *   as hav_sample. */
hav_status_t hav_sample_points(const float* xyz, int64_t N, int64_t M, const hav_params_t* params,
                               int32_t* idx, float* xyz_out, void* ws, size_t ws_bytes,
                               hav_info_t* info_dev, void* stream);

/* ---------------------------------------------------------------------------------
 * The samplers of the latency comparison (Sec. 4.2, Fig. 7). Same conventions as
 * above: device pointers, asynchronous on `stream`, nothing allocated.
 * --------------------------------------------------------------------------------- */

#define HAV_FPS_MAX_POINTS 1048576     /* 256 blocks x 1024 threads x 4 points */
#define HAV_RPS_MAX_POINTS 1073741823  /* 2^30 - 1 */

/* Farthest point sampling (Sec. 3.1, Eq. 1): idx[0] = start, then idx[j] is the
 * point whose squared distance to the nearest of idx[0..j-1] is largest, ties to
 * the lowest index. Squared distances are computed in double as
 * ((dx*dx + dy*dy) + dz*dz) with dx = (double)x_i - (double)x_c and no fused
 * multiply-add, so results are reproducible bit for bit. idx holds M indices in
 * selection order (not sorted). Coordinates must be finite.
 *   xyz [N][3] float32 device; 1 <= M <= N <= HAV_FPS_MAX_POINTS; 0 <= start < N.
 *   blocks: 0 = automatic; else 1..256 blocks share the cloud (N must fit 4 points per
 *   thread of 1024-thread blocks, and the device must hold all the blocks at once, else
 *   HAV_ERR_HIP).
 *   ws: hav_fps_workspace_size(N) bytes of device memory, no initialisation needed;
 *   one call at a time per workspace.
 * Returns HAV_ERR_INVALID_ARG / HAV_ERR_WORKSPACE_TOO_SMALL / HAV_ERR_HIP at once. A
 * multi-block call whose blocks could not all run at once gives up after a bounded
 * wait and raises the flag hav_fps_error reads (idx is then incomplete). */
size_t hav_fps_workspace_size(int64_t N);
hav_status_t hav_fps(const float* xyz, int64_t N, int64_t M, int64_t start, int32_t* idx, void* ws,
                     size_t ws_bytes, int32_t blocks, void* stream);
/* Synchronous read of the flag above (0 = the last call on ws completed). */
hav_status_t hav_fps_error(const void* ws, uint32_t* flag_host);

/* Random point sampling: point i gets the key mix(seed + (i + 1) * 0x9E3779B97F4A7C15)
 * (output i + 1 of the SplitMix64 generator seeded with `seed`; mix as in the trim
 * priority), and the M points of smallest key are returned in ascending index order.
 *   1 <= M <= N <= HAV_RPS_MAX_POINTS; idx [M] int32 device.
 *   window: tuning only, the half-width in standard deviations of the key window a
 *   first pass tries around the expected threshold; 0 = default (6), negative = none
 *   (select over all keys), at most 64. Results do not depend on it.
 *   ws: hav_rps_workspace_size(N) bytes, initialised once with hav_rps_workspace_init
 *   for that N (or any larger N); every call leaves it initialised. One call at a time
 *   per workspace. */
size_t hav_rps_workspace_size(int64_t N);
hav_status_t hav_rps_workspace_init(void* ws, size_t ws_bytes, int64_t N, void* stream);
hav_status_t hav_rps(int64_t N, int64_t M, uint64_t seed, float window, int32_t* idx, void* ws,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Coverage and spacing of a sample (Sec. 3.1, Fig. 3): nearest-sample distances.
 * --------------------------------------------------------------------------------- */

#define HAV_NN_MAX_SAMPLES 1073741823  /* 2^30 - 1, also the query limit */

/* For every query q_j the squared distance to its nearest sample, in double as
 * ((ex*ex + ey*ey) + ez*ez) with ex = (double)sample_x - (double)query_x (no fused
 * multiply-add): exact, so results are reproducible bit for bit. With exclude_self the
 * queries must be the samples themselves (Q == M >= 2) and query j skips sample j: the
 * values are then each sample's spacing to its nearest other sample (the distribution
 * Fig. 3 plots). *max_d2 gets the largest value (with the cloud as queries: the squared
 * covering radius of the sample), or -1 if an internal bounded wait gave up.
 *   samples [M][3], queries [Q][3] float32 device; d2_out [Q] double device or NULL;
 *   max_d2 one double, device. 1 <= M, Q <= HAV_NN_MAX_SAMPLES; finite coordinates.
 *   ws: hav_nn_workspace_size(M) bytes initialised once with hav_nn_workspace_init (for
 *   that M or a larger one); every call leaves it initialised; one call at a time. */
size_t hav_nn_workspace_size(int64_t M);
hav_status_t hav_nn_workspace_init(void* ws, size_t ws_bytes, int64_t M, void* stream);
hav_status_t hav_nn(const float* samples, int64_t M, const float* queries, int64_t Q, int32_t exclude_self,
                    double* d2_out, double* max_d2, void* ws, size_t ws_bytes, void* stream);

/* Ball query: the grouping step that follows sampling in a set-abstraction block (the
 * sampled points become centres; Sec. 3.1 places the sampler in front of grouping).
 * For centre j, idx[j][0..n-1] are the n = min(K, count[j]) lowest indices i with
 * d2 < radius^2 (strict), ascending, d2 in float32 as ((dx*dx + dy*dy) + dz*dz),
 * dx = x_i - c_j, no fused multiply-add, radius^2 = fl(radius * radius); the rest of the
 * row repeats idx[j][0], or is -1 when the ball is empty. count[j] (optional) is the
 * number of points inside the ball.
 *   xyz [N][3], centres [Q][3] float32 device; idx [Q][K] int32 device; count [Q] int32
 *   device or NULL. 1 <= N, Q <= HAV_NN_MAX_SAMPLES; 1 <= K <= 64; radius > 0 finite.
 *   ws: hav_ball_workspace_size(N) bytes initialised once with hav_ball_workspace_init
 *   (for that N or a larger one); one call at a time. */
size_t hav_ball_workspace_size(int64_t N);
hav_status_t hav_ball_workspace_init(void* ws, size_t ws_bytes, int64_t N, void* stream);
hav_status_t hav_ball_query(const float* xyz, int64_t N, const float* centres, int64_t Q, float radius,
                            int32_t K, int32_t* idx, int32_t* count, void* ws, size_t ws_bytes,
                            void* stream);

/* Ball query on the sampler's own spatial structure: the grouping step after sampling
 * in a set-abstraction block (Sec. 3.1 places the sampler in front of grouping), with
 * the sampled points as centres and no second sort of the cloud. A hav_sample call
 * leaves its workspace holding the cloud counting-sorted by spatial cell (with each
 * point's place in that order and the cells' extents); this call finds each centre's
 * neighbours in the few cells its ball overlaps. Results are those of hav_ball_query
 * with centres[j] = xyz[idx[j]]: the n = min(K, count[j]) lowest indices i with
 * d2 < radius^2 (strict), d2 in float32 as ((dx*dx + dy*dy) + dz*dz), dx = x_i - c_j, no
 * fused multiply-add, radius^2 = fl(radius * radius), ascending, the rest of the row
 * repeating out[j][0]; count[j] the number of points inside.
 *   xyz [N][3] float32 device: the cloud of the preceding hav_sample call on `ws`.
 *   idx [M] int32 device: the centres, distinct points of the cloud (e.g. that call's
 *       picks); 1 <= M <= N. out [M][K] int32 device; count [M] int32 device or NULL.
 *   1 <= K <= 64; radius > 0 finite.
 *   ws, ws_bytes, params: the workspace and parameters of that hav_sample call (same N),
 *       enqueued before this call on the same stream; no call may use ws in between.
 * The call reads the workspace's sorted cloud and borrows its per-tile selection lists
 * (returned to their initialised state). If the workspace does not hold this cloud's
 * sorted points (another N, M == N, a chained call, or a call that reported an error),
 * or a centre is not a point of the cloud (or appears twice), that row is all -1 and its
 * count -1. Host-checkable errors return at once. */
hav_status_t hav_ball_query_sampled(const float* xyz, int64_t N, const int32_t* idx, int64_t M,
                                    float radius, int32_t K, int32_t* out, int32_t* count,
                                    void* ws, size_t ws_bytes, const hav_params_t* params, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HAV_H_ */
