/*
 * nbt_ig.h -- C ABI of the MI355X (gfx950) information-gain raycasting library.
 *
 * The library evaluates the information gain (IG) that camera perspectives
 * around a point of interest would collect from a voxel occupancy map, as
 * defined in Sec. III of Renz et al., "Next-Best-Trajectory Planning of Robot
 * Manipulators for Effective Observation and Exploration" (2025):
 *
 *   - every perspective casts N_E = width*height rays from its centre to a
 *     grid of endpoints on the far frustum plane at depth d_Cam, bounded by
 *     the border rays at d_h = d_Cam tan(FoV_h/2), d_v = d_Cam tan(FoV_v/2)
 *     (Sec. III, endpoint calculation);
 *   - a ray's gain is the sum of the voxel gains g(v) (Eq. 2: 1-P occupied,
 *     P free, 1 unknown) over the voxels it meets, up to and including the
 *     first occupied voxel or up to its endpoint (Sec. III, IG calculation);
 *   - a perspective's IG is the mean ray gain over its N_E rays.
 *
 * Conventions the paper leaves open (all arithmetic in IEEE binary32 without
 * fused multiply-add, gains accumulated in binary64):
 *   - ray k = j*width + i; endpoint (u, v, d_Cam) in camera coordinates with
 *     u = d_h*((2i-(width-1))/(width-1)) (0 when width == 1), likewise v;
 *   - pose = 12 floats: row-major 3x3 camera->world rotation R (columns:
 *     camera x = image right, y = image down, z = viewing direction), then
 *     the centre t; world endpoint e = t + ((R_a0*u + R_a1*v) + R_a2*d_Cam);
 *   - the segment t -> e is walked voxel by voxel (Amanatides-Woo 3D-DDA) in
 *     voxel units (x - origin) * (1/voxel_size), clipped to the map and to
 *     the segment; ties between axes advance x before y before z; a face
 *     crossing exactly at the endpoint is still taken; voxels outside the
 *     map do not exist (pad the map with P = 0.5 to treat them as unknown);
 *   - a ray whose voxel-unit coordinates are not finite is INVALID and makes
 *     its perspective's IG NaN.
 *   - voxel (ix,iy,iz) spans origin + voxel_size*[i, i+1); its linear index
 *     is (iz*ny + iy)*nx + ix whatever the internal layout.
 *
 * Memory: unless stated otherwise every pointer argument is a caller-owned
 * DEVICE pointer (e.g. a torch tensor's data_ptr()).  Calls are enqueued on
 * `stream` (a hipStream_t; NULL = the default stream) and return before the
 * work completes.  Calls that use the same context must be ordered on one
 * stream: they share the context's reduction workspace.
 *
 * Errors: every entry point returns an nbt_ig_status; nothing throws or
 * aborts across the ABI.  Argument errors are reported before anything is
 * launched (NBT_IG_EINVAL) and nbt_ig_last_error() returns a thread-local
 * message for the last failure.  Faults inside kernels surface as
 * NBT_IG_EDEVICE from a later call that synchronises.
 */
#ifndef NBT_IG_H
#define NBT_IG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBT_IG_ABI_VERSION 1

typedef enum {
    NBT_IG_OK = 0,
    NBT_IG_EINVAL = -1,         /* invalid argument; nothing was launched */
    NBT_IG_ENOMEM = -2,         /* device or host allocation failed */
    NBT_IG_EDEVICE = -3,        /* a HIP runtime call or a kernel failed */
    NBT_IG_EUNSUPPORTED = -4    /* size or device outside what this build supports */
} nbt_ig_status;

/* Why a ray stopped (nbt_ig_ray_digest.reason). */
enum {
    NBT_IG_RAY_MISS = 0,        /* the segment never enters the map */
    NBT_IG_RAY_HIT = 1,         /* stopped at (and including) its first occupied voxel */
    NBT_IG_RAY_END = 2,         /* reached its endpoint inside the map */
    NBT_IG_RAY_EXIT = 3,        /* left the map before its endpoint */
    NBT_IG_RAY_INVALID = 4      /* non-finite coordinates */
};

/* Voxel states (Eq. 2). */
enum { NBT_IG_OCCUPIED = 1, NBT_IG_FREE = 2, NBT_IG_UNKNOWN = 3 };

/* Device storage order of an encoded map (nbt_ig_ctx_set_map_layout). */
enum {
    NBT_IG_LAYOUT_LINEAR = 0,   /* x fastest over the bordered grid */
    NBT_IG_LAYOUT_COLUMN4 = 1,  /* 4x4 columns: the x-y plane in 4x4 tiles (64 B, x fastest), a tile's
                                   layers stored z after z, tiles x fastest */
    NBT_IG_LAYOUT_COLUMN2 = 2,  /* the same with 2x2 tiles (16 B per layer) */
    NBT_IG_LAYOUT_COLUMN8 = 3   /* the same with 8x8 tiles (256 B per layer) */
};

typedef struct nbt_ig_ctx nbt_ig_ctx;
typedef struct nbt_ig_map nbt_ig_map;
typedef struct nbt_ig_batch nbt_ig_batch;
typedef struct nbt_ig_surrogate nbt_ig_surrogate;

/* The far-plane endpoint grid of one perspective (Sec. III, endpoint calculation). */
typedef struct {
    uint32_t width, height;     /* endpoints per row / column, each >= 1; N_E = width*height */
    float tan_half_fov_h;       /* tan(FoV_h/2), > 0, rounded once from double on the host */
    float tan_half_fov_v;       /* tan(FoV_v/2), > 0 */
    float range;                /* d_Cam: far-plane depth along the camera z axis, metres, > 0 */
} nbt_ig_camera;

/* Voxel classification from occupancy probability (Eq. 2 states). */
typedef struct {
    float occ_threshold;        /* Occupied if P > occ_threshold (default 0.5) */
    float free_threshold;       /* Free if P < free_threshold (default 0.5); Unknown otherwise */
} nbt_ig_classify;

/* Per-ray record of the parity mode (32 bytes). */
typedef struct {
    uint64_t hash;              /* FNV-1a-64 over the visited linear indices, 4 little-endian bytes each */
    double gain;                /* g_R: summed Eq. 2 gains of the visited voxels */
    uint32_t steps;             /* voxels visited (N_O) */
    int32_t stop_lin;           /* linear index of the last visited voxel, -1 if none */
    uint32_t reason;            /* NBT_IG_RAY_* */
    uint32_t reserved;
} nbt_ig_ray_digest;

/* ---- context ---------------------------------------------------------------
 * A context binds one device (HIP ordinal) and owns the reduction workspace.
 * Fails with NBT_IG_EUNSUPPORTED when the device is not gfx950.
 */
int nbt_ig_ctx_create(int device, nbt_ig_ctx** out);
void nbt_ig_ctx_destroy(nbt_ig_ctx* ctx);       /* NULL is a no-op; caller syncs its streams and destroys
                                                   the context's batches, surrogates and maps first */

/* Storage order of the maps this context creates from now on
 * (NBT_IG_LAYOUT_*, default NBT_IG_LAYOUT_COLUMN4; NBT_IG_EINVAL otherwise).  Every call gives the same
 * results on either; the order only changes how many cache lines one
 * 64-ray gather touches.  The getter reports the current setting;
 * nbt_ig_map_layout the order of an existing map. */
int nbt_ig_ctx_set_map_layout(nbt_ig_ctx* ctx, int layout);
int nbt_ig_ctx_get_map_layout(const nbt_ig_ctx* ctx, int* layout);

/* ---- maps -------------------------------------------------------------------
 * Copies the occupancy grid `prob` (float32 [nz][ny][nx], x fastest, values
 * in [0,1]; HOST or DEVICE pointer) into a device-resident encoded map: each
 * voxel stores its Eq. 2 gain with the sign bit marking Occupied, inside a
 * one-voxel border that stops every ray leaving the map, stored in the
 * context's map layout.  1 <= n <= 4096 per axis and (nx+2)(ny+2)(nz+2) <
 * 2^30 (for the column orders: the count with x and y padded to whole tiles < 2^30).  `origin` (HOST, 3 floats) is the world
 * position of the min corner of voxel (0,0,0); `voxel_size` > 0 is s_Vox.
 * `cls` may be NULL (0.5/0.5); 0 <= free_threshold <= occ_threshold <= 1.
 * Probabilities outside [0,1] or NaN give NBT_IG_EINVAL (checked on the
 * device; the call synchronises `stream` once).  The map is immutable and
 * may be read by concurrent evaluations; destroy it only after they finish.
 */
int nbt_ig_create_map(nbt_ig_ctx* ctx, const float* prob, int nx, int ny, int nz, float voxel_size,
                      const float origin[3], const nbt_ig_classify* cls, void* stream,
                      nbt_ig_map** out);
void nbt_ig_destroy_map(nbt_ig_map* map);        /* NULL is a no-op */

/* Re-encodes an existing map in place from new probabilities of the same
 * dimensions (the map is rebuilt whenever a new point cloud has been fused,
 * Sec. III).  `prob` is a DEVICE pointer; the call is asynchronous on
 * `stream` and does not synchronise.  Values outside [0,1] or NaN are
 * encoded as Unknown and recorded; nbt_ig_map_check() synchronises `stream`
 * and returns NBT_IG_EINVAL if any update since the last check saw one.
 * Evaluations already enqueued on other streams must finish first. */
int nbt_ig_update_map(nbt_ig_map* map, const float* prob, void* stream);

/* ---- map update by depth-image insertion ----------------------------------------
 * The occupancy update that precedes IG evaluation: the map is built from the
 * camera's point clouds (Sec. II-III; the paper leaves it to its mapping
 * library, so the usual clamped log-odds update is used).  A scan is a pose
 * and a width x height z-depth image taken with the camera of the endpoint
 * grid: the return of pixel (i, j) lies on that pixel's endpoint ray at
 * parameter s = depth / range.  Depth NaN or <= 0: no measurement; s >= 1:
 * no return within range (the whole segment is carved free).  The walk is the
 * IG walk (same voxels, same tie rule) ending at the return and not stopping
 * at occupied voxels; its last voxel is hit if the return lies inside the
 * map, the others are free.  Per scan each marked voxel's log-odds value L
 * moves once, by l_hit if any ray hit it, else by l_miss, and is clamped to
 * [l_min, l_max] (binary32: add, then max, then min).  Scans apply in order.
 */
typedef struct {
    float l_hit, l_miss;        /* log-odds increments of a hit and of a pass-through */
    float l_min, l_max;         /* clamping bounds, l_min <= l_max, all finite */
} nbt_ig_insert_params;

/* log(p/(1-p)) of hit 0.7, miss 0.4 and the bounds 0.1192 / 0.971, in binary32. */
nbt_ig_insert_params nbt_ig_insert_default_params(void);

/* 32-bit words of the device workspace nbt_ig_insert_scans needs for `map`
 * (two mark bytes per voxel); 0 for NULL. */
uint64_t nbt_ig_insert_workspace_words(const nbt_ig_map* map);

/* Inserts n_scans scans into the log-odds grid of `map`'s geometry.
 *   poses     DEVICE float [n_scans][12] (row-major R camera->world, then t)
 *   depth     DEVICE float [n_scans][height][width], z-depth in metres
 *   params    HOST, NULL = nbt_ig_insert_default_params()
 *   logodds   DEVICE float [nz][ny][nx] (x fastest), updated in place
 *   prob_out  DEVICE float [nz][ny][nx] or NULL: 1/(1+exp(-L)) of the result,
 *             for nbt_ig_update_map (within a few binary32 ulp of the exact logistic)
 *   workspace DEVICE uint32 [workspace_words] >= nbt_ig_insert_workspace_words(map),
 *             all zero before the first call; every call leaves it zero.  Owned
 *             by the caller; calls that share it must not overlap.
 * Asynchronous on `stream` (two launches per scan).  The map's encoded words
 * are not touched.  NBT_IG_EINVAL for NULL pointers, a short workspace or bad
 * parameters. */
int nbt_ig_insert_scans(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                        const float* depth, uint32_t n_scans, const nbt_ig_insert_params* params,
                        float* logodds, float* prob_out, uint32_t* workspace,
                        uint64_t workspace_words, void* stream);
int nbt_ig_map_check(nbt_ig_map* map, void* stream);

/* Dimensions of a map (HOST outputs, any may be NULL). */
int nbt_ig_map_info(const nbt_ig_map* map, int* nx, int* ny, int* nz, float* voxel_size,
                    float origin[3], size_t* device_bytes);
int nbt_ig_map_layout(const nbt_ig_map* map, int* layout);

/* Rewrites an existing map in another storage order (NBT_IG_LAYOUT_*): a new
 * device buffer is filled from the old one on `stream`, the call synchronises
 * `stream` and then frees the old buffer.  No evaluation of the map may run
 * meanwhile (on any stream).  NBT_IG_EINVAL while a batch holds the map (its
 * descriptor would go stale); a no-op when the map already has the order. */
int nbt_ig_map_set_layout(nbt_ig_map* map, int layout, void* stream);

/* ---- per-perspective IG (Sec. III, IG calculation) ----------------------------
 * ig_out[p] = g_P of pose p: the mean over its N_E rays of the ray gain g_R
 * (Eq. 2 summed to the first occupied voxel or the endpoint), rounded once
 * to float32; NaN if any of its rays is INVALID.  steps_out[p] (may be NULL)
 * = total voxels visited by its rays (exact).  poses: float32 [n][12].
 * n == 0 is a no-op.  Results are bit-identical from run to run.
 */
int nbt_ig_eval_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                           uint32_t n, float* ig_out, uint64_t* steps_out, void* stream);

/* ---- per-perspective IG without allocation ---------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same results as
 * nbt_ig_eval_viewpoints, bit for bit, from the same kernels, but the
 * cross-workgroup reduction slots live in a fixed array of
 * NBT_IG_NOALLOC_MAX_VIEWPOINTS slots (24 B each, 1.5 MiB) that the library
 * holds on every device it runs on until the process ends; the call allocates
 * nothing and never grows a workspace.  n > NBT_IG_NOALLOC_MAX_VIEWPOINTS
 * returns NBT_IG_EUNSUPPORTED before anything is launched.  The slots needed
 * are cleared on `stream` by a fill kernel at the start of each call.  All
 * calls on one device share that array: two such calls that overlap (on
 * different streams, or from different threads without ordering) race and
 * give wrong results.  Arguments, layouts and errors as nbt_ig_eval_viewpoints.
 */
#define NBT_IG_NOALLOC_MAX_VIEWPOINTS 65536u
int nbt_ig_eval_viewpoints_noalloc(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                   uint32_t n, float* ig_out, uint64_t* steps_out, void* stream);

/* ---- per-trajectory IG ----------------------------------------------------------
 * A trajectory is poses_per_traj consecutive poses: poses is float32
 * [n_traj][poses_per_traj][12].  U_t = the set of voxels visited by any ray
 * of any pose of trajectory t (the walk of Sec. III, each voxel counted
 * once however often it is seen along the path).  Outputs (DEVICE):
 *   ig_union[t]    sum over U_t of the Eq. 2 gains (binary64, rounded once to
 *                  float32); NaN if any ray of the trajectory is INVALID;
 *   counts[4t+0..3] |U_t|, occupied, free and unknown voxels of U_t (exact);
 *   visits[t]      total voxel visits of all its rays (exact; may be NULL: the
 *                  walk then keeps no per-ray visit count, which is faster).
 * Each trajectory's visited set is a bitset over the voxel box holding its
 * frusta, kept in LDS; a box with more bits than the context's LDS budget
 * holds is covered in several passes over the trajectory's rays, each marking
 * one slice of the box (same results, bit for bit).  Nothing is read back to
 * the host: the call only enqueues work on `stream` (so it can be captured in
 * a graph once a call with as many trajectories has sized the workspace).
 * n_traj == 0 is a no-op.
 */
int nbt_ig_eval_trajectories(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                             uint32_t n_traj, uint32_t poses_per_traj, float* ig_union,
                             uint32_t* counts, uint64_t* visits, void* stream);

/* LDS per workgroup that a trajectory bitset may use, its two bookkeeping
 * words included (0 = the default: as much as does not lower how many union
 * workgroups fit on a compute unit; capped at the device maximum); larger
 * boxes take several passes.  Context properties (HOST outputs, may be NULL;
 * lds_budget reports the bytes in effect for the current workgroup size). */
int nbt_ig_ctx_set_lds_budget(nbt_ig_ctx* ctx, size_t bytes);
int nbt_ig_ctx_info(const nbt_ig_ctx* ctx, int* cu_count, size_t* lds_per_group, size_t* lds_budget);

/* Wavefronts per workgroup of the trajectory kernel (one workgroup per
 * trajectory): 4, 8 or 16 (default 8); NBT_IG_EINVAL otherwise.  Results do
 * not depend on it. */
int nbt_ig_ctx_set_traj_waves(nbt_ig_ctx* ctx, int waves_per_group);
int nbt_ig_ctx_get_traj_waves(const nbt_ig_ctx* ctx, int* waves_per_group);

/* ---- parity mode ---------------------------------------------------------------
 * One nbt_ig_ray_digest per ray: out[p*N_E + k] for pose p, ray k.
 */
int nbt_ig_trace_rays(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                      uint32_t n, nbt_ig_ray_digest* out, void* stream);

/* Parity mode of the throughput walks: the same kernels as
 * nbt_ig_eval_viewpoints (in the context's launch shape, pipelined gathers,
 * incremental offsets in the map's storage order) and nbt_ig_eval_trajectories
 * (the union walk with its bitset marks), instantiated to also write one
 * record per ray.  Each record is built from the byte offsets that the walk
 * gathered, decoded back into voxel coordinates, in visiting order: hash,
 * steps, stop_lin and reason must equal nbt_ig_trace_rays's; gain is the
 * gathered words' gains summed in binary64 in visiting order.  The IG, step,
 * count and visit outputs are those of the untraced calls, bit for bit.
 *   nbt_ig_trace_viewpoints:   out[p*N_E + k] for pose p, ray k; reserved = 0.
 *   nbt_ig_trace_trajectories: out[(t*poses_per_traj + l)*N_E + k] for pose l of
 *                              trajectory t; reserved = the number of visits
 *                              whose bitset position names another voxel than
 *                              the one gathered (0 for a correct walk).
 * Other arguments as for the untraced calls. */
int nbt_ig_trace_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                            uint32_t n, float* ig_out, uint64_t* steps_out, nbt_ig_ray_digest* out,
                            void* stream);
int nbt_ig_trace_trajectories(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                              uint32_t n_traj, uint32_t poses_per_traj, float* ig_union, uint32_t* counts,
                              uint64_t* visits, nbt_ig_ray_digest* out, void* stream);

/* Full voxel sequences of selected rays.  rays: uint32 [count][2] = (pose
 * index, ray index k); lin_out: int32 [count][max_len] receives the visited
 * linear indices in order (entries past the ray's length are left as is);
 * len_out: uint32 [count] receives the full number of visited voxels (which
 * may exceed max_len; then only the first max_len are written).  Rays whose
 * pose index >= n or ray index >= N_E get length 0.
 */
int nbt_ig_trace_paths(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                       uint32_t n, const uint32_t* rays, uint32_t count, uint32_t max_len,
                       int32_t* lin_out, uint32_t* len_out, void* stream);

/* ---- launch shape (set by the autotuner) -----------------------------------------
 * How nbt_ig_eval_viewpoints maps rays to the GPU: waves_per_group in
 * {1,2,4,8} wavefronts per workgroup; each wave walks pixel tiles of
 * (1<<tile_w_log2) x (64>>tile_w_log2) rays (tile_w_log2 in 0..6);
 * tiles_per_wave >= 1 tiles per wave per workgroup, or 0 to deal the
 * camera's tiles evenly over as few workgroups as 16 tiles per wave allow
 * (the default); xcd_remap = C > 0
 * deals runs of C consecutive workgroups (the workgroups of neighbouring
 * perspectives) to one XCD and its L2, 0 keeps the hardware's round-robin
 * order (C <= 65536); pipeline_depth in
 * {1,2,4,8} map gathers in flight per ray (0 = default, 8).  A new context
 * starts at 4 waves, 8x8 tiles, balanced tiles per wave, no remap, 8 gathers
 * in flight.  Any shape gives the same step counts; IG agrees to the
 * last-place rounding of its sum.
 */
typedef struct {
    int32_t waves_per_group;
    int32_t tile_w_log2;
    int32_t tiles_per_wave;
    int32_t xcd_remap;
    int32_t pipeline_depth;
} nbt_ig_launch;

int nbt_ig_ctx_set_launch(nbt_ig_ctx* ctx, const nbt_ig_launch* launch);
int nbt_ig_ctx_get_launch(const nbt_ig_ctx* ctx, nbt_ig_launch* launch);

/* ---- batched evaluation over many maps -------------------------------------------
 * The per-perspective IG of nbt_ig_eval_viewpoints for many maps of uneven
 * size and uneven perspective counts in ONE persistent launch: workgroups
 * (as many as fit on the device at once) pull (perspective, ray-slice) items
 * in map-major order from a device work queue until it is empty.
 *
 * nbt_ig_batch_create: `maps` (HOST array of n_maps handles of this context,
 * each outliving the batch; their storage order is pinned while it exists)
 * and the camera are fixed for the batch; max_total_viewpoints bounds the
 * perspectives of one run.  The launch shape starts as the context's.
 *
 * nbt_ig_batch_run: vp_offsets is a DEVICE CSR uint32 [n_maps+1] (perspectives
 * of map k are vp_offsets[k] .. vp_offsets[k+1]-1, non-decreasing,
 * vp_offsets[0] = 0); poses float32 [total][12], ig_out float32 [total],
 * steps_out uint64 [total] or NULL, where total = vp_offsets[n_maps] (runs
 * clamp it to max_total_viewpoints).  The offsets are read on the device, so
 * the same batch can run different counts without host synchronisation.  The
 * first run (and any run with different buffer pointers) builds a hipGraph of
 * the queue reset and the persistent kernel; later runs replay it.  Results
 * equal nbt_ig_eval_viewpoints on each map (step counts exactly).  Runs of one
 * batch must be ordered on one stream.
 */
int nbt_ig_batch_create(nbt_ig_ctx* ctx, const nbt_ig_map* const* maps, uint32_t n_maps,
                        const nbt_ig_camera* cam, uint32_t max_total_viewpoints, nbt_ig_batch** out);
void nbt_ig_batch_destroy(nbt_ig_batch* batch);  /* NULL is a no-op; caller syncs first */
int nbt_ig_batch_run(nbt_ig_batch* batch, const uint32_t* vp_offsets, const float* poses, float* ig_out,
                     uint64_t* steps_out, void* stream);
/* xcd_remap is ignored by the persistent launch.  persistent_groups (HOST, may be
 * NULL) receives the number of workgroups launched. */
int nbt_ig_batch_set_launch(nbt_ig_batch* batch, const nbt_ig_launch* launch);
int nbt_ig_batch_get_launch(const nbt_ig_batch* batch, nbt_ig_launch* launch, uint32_t* persistent_groups);

/* ---- autotuning ----------------------------------------------------------------------
 * Time candidate launch shapes (every combination of waves_per_group 1/2/4/8,
 * tile_w_log2 2/3/4, tiles_per_wave 0/2/4/16 and pipeline_depth 2/4/8: 144
 * shapes, each run once untimed and then timed) on the given inputs, keep
 * the fastest in the context (or batch) and report it with its
 * mean time per launch in milliseconds (HOST outputs).  Outputs are written
 * as by the evaluation calls.  Synchronises `stream`.
 */
int nbt_ig_autotune_viewpoints(const nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                               uint32_t n, float* ig_out, uint64_t* steps_out, void* stream,
                               nbt_ig_launch* best, float* best_ms);
int nbt_ig_batch_autotune(nbt_ig_batch* batch, const uint32_t* vp_offsets, const float* poses,
                          float* ig_out, uint64_t* steps_out, void* stream, nbt_ig_launch* best,
                          float* best_ms);

/* Chooses the storage order of the batch's maps (all alike): times the batch
 * in every storage order (linear and the three column tile sizes) at its
 * current launch shape, leaves the maps in the fastest one (*best_layout, HOST; mean ms per run in *best_ms) and updates the
 * batch.  Synchronises `stream`; no other work may use the maps meanwhile.
 * NBT_IG_EINVAL when another batch holds one of the maps too. */
int nbt_ig_batch_autotune_layout(nbt_ig_batch* batch, const uint32_t* vp_offsets, const float* poses,
                                 float* ig_out, uint64_t* steps_out, void* stream, int* best_layout,
                                 float* best_ms);

/* For trajectory IG: times nbt_ig_eval_trajectories on every storage order of
 * the map and each trajectory workgroup size (4, 8, 16 waves), keeps the
 * fastest (the map rewritten in *best_layout, the context set to *best_waves;
 * HOST outputs, mean ms per call in *best_ms).  Outputs are written as by the
 * evaluation.  Synchronises `stream`; the map must not be held by a batch. */
int nbt_ig_autotune_trajectories(nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses,
                                 uint32_t n_traj, uint32_t poses_per_traj, float* ig_union, uint32_t* counts,
                                 uint64_t* visits, void* stream, int* best_layout, int* best_waves,
                                 float* best_ms);

/* As nbt_ig_autotune_viewpoints, and first the map's storage order: times
 * nbt_ig_eval_viewpoints in every order at the context's launch shape, keeps
 * the map in the fastest one (*best_layout, HOST; see nbt_ig_map_set_layout),
 * then searches the launch shape.  The map must not be held by a batch. */
int nbt_ig_autotune_map(nbt_ig_map* map, const nbt_ig_camera* cam, const float* poses, uint32_t n,
                        float* ig_out, uint64_t* steps_out, void* stream, nbt_ig_launch* best,
                        int* best_layout, float* best_ms);

/* ---- learned IG surrogate ----------------------------------------------------------
 * A small network trained on this library's own exact IG predicts g_P of a
 * candidate perspective from (a) a 32^3 x 2 patch around the PoI holding the
 * fraction of occupied and of unknown voxels per cell and (b) the candidate's
 * unit direction and distance from the PoI; it prunes candidates so that only
 * the best few are raycast exactly (Sec. III's g_P decides).
 * Network: 4 conv3d layers (3^3, stride 2, ReLU; 2-16-32-64-64 channels,
 * 32^3 -> 2^3) -> 512 features; MLP 516 -> 256 -> 256 -> 1 (ReLU).  Inference
 * runs in BF16 on MFMA with FP32 accumulation; the pose-independent part of
 * the first MLP layer is computed once per map.
 *
 * weights (HOST, nbytes): "NBTS", uint32 version 1, float extent (patch cube
 * side, metres), dist_mean, dist_scale, out_scale, 2 reserved uint32, then
 * little-endian float32: conv1..4 weights [cout][cin][3][3][3] and biases,
 * fc1 [256][516] + bias, fc2 [256][256] + bias, fc3 [256] + bias.  Patch cells
 * are f^3 voxels, f = max(1, round(extent / (32 voxel_size))), centred on the
 * voxel nearest the PoI; voxels outside the map count as neither state.
 */
int nbt_ig_surrogate_create(nbt_ig_ctx* ctx, const void* weights, size_t nbytes, nbt_ig_surrogate** out);
void nbt_ig_surrogate_destroy(nbt_ig_surrogate* s);   /* NULL is a no-op; caller syncs first */

/* pred[i] (DEVICE float32 [n]) = predicted IG of pose i (DEVICE float32 [n][12])
 * for the PoI `poi` (HOST, 3 floats, world metres).  Calls on one surrogate
 * must be ordered on one stream (they share its buffers). */
int nbt_ig_surrogate_predict(nbt_ig_surrogate* s, const nbt_ig_map* map, const float poi[3],
                             const float* poses, uint32_t n, float* pred, void* stream);

/* Predict all n candidates, keep the k_rescore best predictions (ties to the
 * lower index), evaluate those exactly (nbt_ig_eval_viewpoints with `cam`),
 * and return the k best by exact IG: idx_out (DEVICE uint32 [k]) candidate
 * indices, ig_out (DEVICE float32 [k]) their exact IG, best first (ties to the
 * lower index).  1 <= k <= k_rescore <= 1024, k_rescore <= n <= 2^22. */
int nbt_ig_surrogate_select(nbt_ig_surrogate* s, const nbt_ig_map* map, const nbt_ig_camera* cam,
                            const float poi[3], const float* poses, uint32_t n, uint32_t k_rescore,
                            uint32_t k, uint32_t* idx_out, float* ig_out, void* stream);

/* Intermediate values for verification (DEVICE outputs, either may be NULL):
 * the patch as float32 [2][32][32][32] (channel, z, y, x) and the 512 trunk
 * features as float32 (their BF16 values). */
int nbt_ig_surrogate_features(nbt_ig_surrogate* s, const nbt_ig_map* map, const float poi[3],
                              float* patch_out, float* features_out, void* stream);

/* The surrogate's input patch for any cube side `extent` (training data):
 * out DEVICE float32 [2][32][32][32]. */
int nbt_ig_extract_patch(const nbt_ig_map* map, const float poi[3], float extent, float* out, void* stream);

/* ---- next-best-view selection -------------------------------------------------------
 * The k largest of n values (DEVICE float32, e.g. the per-perspective IG of
 * nbt_ig_eval_viewpoints: k = 1 is the NBV of an ID), best first, ties to
 * the lower index; idx_out DEVICE uint32 [k], val_out DEVICE float32 [k] (may
 * be NULL).  NaN ranks last; -0 and +0 are equal values.  1 <= k <= 1024,
 * k <= n <= 2^22. */
int nbt_ig_top_k(nbt_ig_ctx* ctx, const float* values, uint32_t n, uint32_t k, uint32_t* idx_out,
                 float* val_out, void* stream);

/* ---- planner-side IG terms (Sec. IV, cost function extension) ---------------------
 * For n_horizons candidate horizons of `steps` camera poses each (DEVICE
 * float32 [n_horizons][steps][12]) and a buffer of n_ids information
 * distributions (DEVICE: id_pos float32 [n_ids][n_persp][3] perspective start
 * points, id_ig float32 [n_ids][n_persp] their g_P; index 0 = oldest):
 *   g_out[h][k]  G(x) of Eq. 3: sum over IDs u of 1/(n_ids - u) times the
 *                inverse-distance-weighted IG (distance power p) at the
 *                camera centre; a centre that coincides exactly with
 *                perspectives of an ID takes their mean IG for that ID;
 *   o_out[h][k]  orientation factor: cos of the angle between the viewing
 *                axis and the direction to `poi` (HOST, 3 floats), 0 when the
 *                PoI is outside the field of view tan_half_fov_h/v;
 *   cost_out[h]  c_I = sum_k w_i / (O G + eps) (may be NULL).
 * FP32 distances and weights with FP64 sums; results agree with a float64
 * evaluation to ~1e-6 relative (FoV decisions can differ within ~1e-6 of
 * the field-of-view border). */
int nbt_ig_eval_cost(nbt_ig_ctx* ctx, const float* id_pos, const float* id_ig, uint32_t n_ids,
                     uint32_t n_persp, float p, const float* poses, uint32_t n_horizons, uint32_t steps,
                     const float poi[3], float tan_half_fov_h, float tan_half_fov_v, float w_i, float eps,
                     float* g_out, float* o_out, float* cost_out, void* stream);

/* ---- helpers ------------------------------------------------------------------- */

/* Endpoint grid from the paper's grid scaling (Sec. III: endpoint spacing
 * s_G * s_Vox on the far plane, including both border rays):
 * width = floor(2 d_h / (s_G s_Vox)) + 1, height likewise with d_v.
 * Angles in radians; all outputs HOST. */
int nbt_ig_camera_from_grid(double fov_h, double fov_v, double d_cam, double s_vox, double s_g,
                            nbt_ig_camera* out);

/* ---- memory probes (measurement of the ray kernels' ceilings) ----------------------
 * Not part of the method: reads a caller's DEVICE buffer (16-byte aligned) with the
 * access patterns of a voxel walk, so that a ray kernel's rate can be set against what
 * the memory level holding a map of the same size delivers.  `sink` (DEVICE uint32
 * [nbt_ig_probe_sink_words(ctx)]) receives one xor of the words read per workgroup.
 *   NBT_IG_PROBE_STREAM       reads every 16-byte piece of buf, `count` passes;
 *                             bytes/16 a power of two, count * bytes/16 < 2^32;
 *                             useful bytes = count * bytes;
 *   NBT_IG_PROBE_GATHER       8 * cu_count workgroups of 256 lanes, each lane reads
 *                             `count` 4-byte words at pseudo-random positions;
 *   NBT_IG_PROBE_QUAD_GATHER  the same, but the four lanes of a quad read the four
 *                             words of one pseudo-random 16-byte piece;
 *                             for both gathers bytes/4 is a power of two and useful
 *                             bytes = 4 * count * 256 * 8 * cu_count. */
#define NBT_IG_PROBE_STREAM 0
#define NBT_IG_PROBE_GATHER 1
#define NBT_IG_PROBE_QUAD_GATHER 2
int nbt_ig_probe_sink_words(const nbt_ig_ctx* ctx);
int nbt_ig_probe_memory(nbt_ig_ctx* ctx, int kind, const void* buf, size_t bytes, uint32_t count,
                        uint32_t* sink, void* stream);

/* ---- MFMA probe (measurement of the surrogate MLP's ceiling) ----------------------
 * Launches cu_count * waves_per_simd workgroups of 4 waves (one per SIMD), each
 * wave running `iters` rounds of independent BF16 MFMA accumulation chains on
 * register operands (16 chains of v_mfma_f32_16x16x32_bf16, or 8 of
 * v_mfma_f32_32x32x16_bf16), with no memory traffic in the loop.  sink (DEVICE,
 * at least nbt_ig_probe_sink_words(ctx) words) receives one xor of the
 * accumulators per workgroup; *flops (HOST, may be NULL) the launch's floating
 * point operations (2 M N K per instruction), to be divided by the caller's own
 * timing of the launch on `stream`.  waves_per_simd in [1, 8], iters >= 1. */
#define NBT_IG_PROBE_MFMA_16X16X32_BF16 0
#define NBT_IG_PROBE_MFMA_32X32X16_BF16 1
int nbt_ig_probe_mfma(nbt_ig_ctx* ctx, int kind, int waves_per_simd, uint32_t iters, uint32_t* sink,
                      double* flops, void* stream);

const char* nbt_ig_status_string(int status);
const char* nbt_ig_last_error(void);             /* thread-local; never NULL */
int nbt_ig_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBT_IG_H */
