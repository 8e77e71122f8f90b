/*
 * mvf.h -- C ABI of the MI355X multi-volume TSDF mapping library (libmvf).
 *
 * Implements the data-parallel core of Salvato, Finman, Leonard,
 * "Multi-Volume High Resolution RGB-D Mapping with Dynamic Volume
 * Placement" (arXiv 1511.07106): projective TSDF integration of a depth +
 * RGB frame into every active subvolume, raycasting of all subvolumes into
 * one shared depth/vertex/normal map, host<->device volume passing under a
 * device-memory budget, and the ray-endpoint placement rule.  Beside the
 * plain per-volume form it offers a batched form (all volumes of many
 * independent scenes in one launch) and a differentiable raycast.
 *
 * Conventions (all calls):
 *  - Units are metres.  Poses T_wc are row-major 3x4 camera-to-world
 *    [R | t] (x_w = R x_c + t), OpenCV camera axes (x right, y down,
 *    z forward).  Intrinsics are (fx, fy, cx, cy); pixel (u, v) has its
 *    centre at integer coordinates.
 *  - A grid is a world voxel lattice: voxel g (int3) has its centre at
 *    origin + voxel_size * (g + 1/2).  A volume covers global voxels
 *    [offset, offset + dims) of one grid ("t_s = t_l + h_t", Volumetric
 *    Integration section; translations in voxel units, Dynamic Mapping for
 *    SLAM section).
 *  - "device" pointers are HIP device memory (e.g. a torch tensor's
 *    data_ptr()); "host" pointers are ordinary process memory.  `stream` is
 *    a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on `stream` and the call returns before it completes unless
 *    the call says it synchronises; device buffers passed in must stay
 *    valid until the stream reaches the work.
 *  - Every call returns an mvf_status; on failure mvf_last_error() gives a
 *    message for the calling thread.  No call throws.  A context is used by
 *    one host thread at a time.  Asynchronous device faults surface at the
 *    next synchronising call as MVF_ERR_HIP.
 *
 * Numeric contract (shared with the CPU oracle used by the tests): every
 * decision (voxel -> pixel, update or not, colour band, ray sample in
 * domain/valid, zero crossing, nearest volume, placement cell) is made in
 * IEEE binary32 with one rounding per operation in a fixed order and no
 * fused multiply-add, so integer weights and colours are bit-exact.
 */
#ifndef MVF_H
#define MVF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mvf_status;
#define MVF_OK 0
#define MVF_ERR_INVALID_ARG 1 /* bad pointer, size, id or parameter */
#define MVF_ERR_NOT_FOUND 2   /* unknown grid or volume id */
#define MVF_ERR_OOM 3         /* device or pinned host allocation failed */
#define MVF_ERR_BUDGET 4      /* one volume is larger than the device budget */
#define MVF_ERR_HIP 5         /* a HIP runtime call failed (message has details) */
#define MVF_ERR_STATE 6       /* call not valid in the object's current state */
#define MVF_ERR_UNSUPPORTED 7 /* feature not available */

typedef struct mvf_ctx mvf_ctx;

/* Context flags. */
#define MVF_FLAG_TIMING 1u /* time integrate/raycast kernels with HIP events */

typedef struct {
    uint64_t hbm_budget_bytes; /* device bytes volumes may occupy; 0 = no limit */
    float ray_step;            /* raycast sample spacing in voxels, (0, 1); 0 = 0.5 */
    float t_far;               /* raycast range in metres; 0 = 10 */
    int32_t device;            /* HIP device ordinal */
    uint32_t flags;            /* MVF_FLAG_* */
} mvf_config;

typedef struct {
    float origin[3];    /* world position of the corner of voxel (0,0,0) */
    float voxel_size;   /* s, metres */
    float trunc_voxels; /* truncation mu = trunc_voxels * s */
    uint16_t w_max;     /* running-weight cap, >= 1 */
    uint16_t reserved;
} mvf_grid_desc;

typedef struct {
    int32_t grid_id;
    int32_t offset[3];  /* h_t: global voxel index of local voxel (0,0,0) */
    int32_t dims[3];    /* h_r per axis, each in [2, 2048]; at most 2^30 voxels
                           after padding each axis to a multiple of 8 */
    int32_t stream_id;  /* scene this volume belongs to, >= 0 */
} mvf_volume_desc;

typedef struct {
    float fx, fy, cx, cy;
} mvf_intrinsics;

typedef struct {
    const float* depth;  /* device, height rows of depth_pitch floats; z-depth, <=0/NaN/inf = none */
    const uint8_t* rgb;  /* device, height rows of rgb_pitch bytes, RGB8; may be NULL */
    int32_t width, height;
    int32_t depth_pitch; /* floats per row; 0 = width */
    int32_t rgb_pitch;   /* bytes per row; 0 = 3 * width */
} mvf_frame;

typedef struct {
    float* depth;    /* device H*W: camera z of the surface, 0 = no surface */
    float* vertex;   /* device H*W*3 world position, NaN = none; may be NULL */
    float* normal;   /* device H*W*3 world unit normal, NaN = none; may be NULL */
    int32_t* hit;    /* device H*W id of the volume hit, -1 = none; may be NULL */
    int32_t width, height;
} mvf_raycast_out;

typedef struct {
    uint64_t voxels_updated;     /* voxels that passed the truncation test */
    uint64_t voxels_band;        /* of those, voxels inside the colour band */
    uint64_t pixels_raycast;     /* output pixels written by raycasts */
    uint64_t bytes_h2d;          /* volume bytes swapped in */
    uint64_t bytes_d2h;          /* volume bytes swapped out */
    uint64_t swaps_in, swaps_out;
    uint64_t integrate_launches, raycast_launches, step_launches;
    double integrate_ms;         /* HIP-event time of integrate kernels (MVF_FLAG_TIMING) */
    double raycast_ms;           /* HIP-event time of raycast kernels (MVF_FLAG_TIMING) */
    double step_ms;              /* HIP-event time of batched step graphs (MVF_FLAG_TIMING) */
    uint64_t resident_bytes;     /* device bytes held by volumes now */
    int32_t resident_volumes;
    int32_t reserved;
    uint64_t bricks_projected;   /* bricks integrated voxel by voxel (projection, range gather) */
    uint64_t bricks_deep;        /* bricks updated wholesale with phi = 1 (in front of the
                                    measured surface by more than mu everywhere) */
} mvf_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context on cfg->device.  cfg may be NULL (defaults).  Output
 * *out owns every volume slab and pinned mirror it creates. */
/* Test hook: when the environment variable MVF_FAULT_SLAB_ALLOCS = n is set
 * at creation, the context's next n volume-slab allocations fail as if the
 * device were out of memory (exercising the drop-the-pool-and-retry path
 * and the MVF_ERR_OOM return). */
mvf_status mvf_create(mvf_ctx** out, const mvf_config* cfg);
/* Synchronise and free everything the context owns.  NULL is a no-op. */
mvf_status mvf_destroy(mvf_ctx* ctx);
/* Block until all work the context enqueued (any stream) has finished. */
mvf_status mvf_synchronize(mvf_ctx* ctx);
/* Change the device budget; volumes above it are swapped out lazily. */
mvf_status mvf_set_budget(mvf_ctx* ctx, uint64_t bytes);
/* Synchronising.  Counters since creation or the last reset. */
mvf_status mvf_get_stats(mvf_ctx* ctx, mvf_stats* out);
mvf_status mvf_reset_stats(mvf_ctx* ctx);
const char* mvf_status_string(mvf_status s);
/* Message of the calling thread's last failure ("" if none). */
const char* mvf_last_error(void);
/* Library version string. */
const char* mvf_version(void);

/* ---- grids and volumes (Initialization; Dynamic Volume Allocation) ---- */

/* Register a voxel lattice shared by volumes (origin, s, mu, W cap). */
mvf_status mvf_grid_create(mvf_ctx* ctx, const mvf_grid_desc* desc, int32_t* grid_id);

/* Describe a subvolume h = (h_l, h_r, h_t) on a grid.  Its state starts
 * empty (TSDF 0, weight 0, colour 0); no memory is touched until it is
 * first used.  It is not active until placed. */
mvf_status mvf_volume_create(mvf_ctx* ctx, const mvf_volume_desc* desc, int32_t* vol_id);
/* Forget a volume and release its device slab and host mirror
 * (synchronises with work using it). */
mvf_status mvf_volume_destroy(mvf_ctx* ctx, int32_t vol_id);
/* Add a volume to the active set H: every later integrate/raycast of its
 * stream processes it (Dynamic Volume Allocation, Input and Output). */
mvf_status mvf_volume_place(mvf_ctx* ctx, int32_t vol_id);
/* Remove a volume from H (the removal function g).  Its state is kept.
 * flags & MVF_EVICT_SWAP_OUT also moves it to host memory now. */
#define MVF_EVICT_SWAP_OUT 1u
mvf_status mvf_volume_evict(mvf_ctx* ctx, int32_t vol_id, uint32_t flags);
/* Explicit memory passing (Memory Passing section; "upload to GPU" and
 * the download after raycasting): make the volume device-resident, or copy
 * it to its pinned host mirror and release the device slab.  Copies run on
 * the context's copy stream, ordered after the work already enqueued on
 * `stream` and before later work on it. */
mvf_status mvf_volume_swap_in(mvf_ctx* ctx, int32_t vol_id, void* stream);
mvf_status mvf_volume_swap_out(mvf_ctx* ctx, int32_t vol_id, void* stream);
/* Synchronising.  Copy the volume's state to host buffers in canonical
 * x-fastest layout (index (z*ny + y)*nx + x): F float32 in truncation
 * units (0 where W == 0), W uint16, rgba 4 bytes per voxel (A = colour
 * weight).  Any pointer may be NULL to skip that plane. */
mvf_status mvf_volume_read(mvf_ctx* ctx, int32_t vol_id, float* F, uint16_t* W, uint8_t* rgba);
/* Synchronising.  Overwrite the volume's state from host buffers in the
 * same layout (F of voxels with W == 0 is ignored).  NULL planes are set
 * to their empty value. */
mvf_status mvf_volume_write(mvf_ctx* ctx, int32_t vol_id, const float* F, const uint16_t* W,
                            const uint8_t* rgba);
/* Synchronising.  Copy the volume's brick summaries to host buffers of
 * nb = bx * by * bz bytes each, where (bx, by, bz) = ceil(dims / 8), in
 * brick order (index (x * by + y) * bz + z, z fastest).  flag: 1 if some
 * voxel of the 8^3 brick may hold F <= 2^-100 (set when an update writes
 * such a value, never cleared except by mvf_volume_write), else 0.  dist:
 * the Chebyshev distance in bricks to the nearest flagged brick, capped at
 * 12, as of the last integration or write.  These are the exact-skip
 * structures of the raycast (the zero crossing can only lie in a cell with
 * a corner F <= 0, Raycasting section); a diagnostic for tests.  Either
 * pointer may be NULL. */
mvf_status mvf_volume_brick_summary(mvf_ctx* ctx, int32_t vol_id, uint8_t* flag, uint8_t* dist);
/* Surface points of a volume (Input and Output: the output vertex set V
 * with normals N, at most one vertex per voxel; Metrics: a voxel that the
 * surface crosses gets a vertex; Insertion and Removal: the point cloud of a
 * removed volume is downloaded).  Voxel g gives a vertex when its cell
 * [g, g+1]^3 lies in the volume with all 8 corners observed (W > 0) and F
 * changes sign inside the band (|F| < 1; one end > 0, the other <= 0)
 * along one of the edges +x, +y, +z leaving g: the first such edge in that
 * order holds the vertex, at the linear zero crossing, with the normalised
 * gradient of the cell's trilinear TSDF there as its normal (pointing into
 * observed free space).
 * V, N: device float32 buffers of cap x 3 (world metres; unit normals).
 * G: device int32 cap x 3 global voxel indices of the emitting voxels, or
 * NULL.  Points are written in brick order (8^3 bricks, z-fastest brick
 * numbering; inside a brick z-slice by z-slice, x fastest), a fixed order.
 * *n_total (host) receives the number of points; min(n_total, cap) are
 * written (cap = 0 only counts, and V, N may then be NULL).  The volume is
 * made device-resident first (under the budget, like integration).  Runs
 * on `stream` and synchronises it.  A never-observed volume gives 0. */
mvf_status mvf_volume_extract(mvf_ctx* ctx, int32_t vol_id, float* V, float* N, int32_t* G,
                              int64_t cap, int64_t* n_total, void* stream);
/* The descriptor a volume was created with (also for volumes the
 * placement step created). */
mvf_status mvf_volume_describe(mvf_ctx* ctx, int32_t vol_id, mvf_volume_desc* out);
/* Resident (1) or not (0), device bytes of its slab, active flag. */
mvf_status mvf_volume_query(mvf_ctx* ctx, int32_t vol_id, int32_t* resident, uint64_t* bytes,
                            int32_t* active);

/* Checkpoint: write the context's grids, volumes (ids, descriptors, active
 * flags and full state, brick summaries included) and the placement
 * bookkeeping to the file `path`.  Synchronising.  The library's internal
 * volumes are not saved.  The file is in this build's memory layout and
 * host byte order. */
mvf_status mvf_checkpoint_save(mvf_ctx* ctx, const char* path);
/* Resume: restore a checkpoint into a context that has no grids or volumes
 * yet (MVF_ERR_STATE otherwise).  Ids are those of the saved context;
 * volumes with state come back in host memory (swapped out) and are
 * uploaded when first needed.  MVF_ERR_INVALID_ARG for a file that is not
 * such a checkpoint, is truncated, or holds another layout; the context is
 * then left empty. */
mvf_status mvf_checkpoint_load(mvf_ctx* ctx, const char* path);

/* ---- per-frame hot path ----------------------------------------------- */

/* Volumetric integration (Volumetric Integration section; Algorithm 1's
 * voxel loop) of one frame into every active volume of `stream_id` whose
 * box meets the view frustum.  Volumes not resident are swapped in first;
 * if they do not all fit in the budget they are processed in waves, the
 * paper's one-volume-at-a-time memory passing being the smallest case. */
mvf_status mvf_integrate(mvf_ctx* ctx, int32_t stream_id, const mvf_frame* frame,
                         const float T_wc[12], const mvf_intrinsics* K, void* stream);
/* Raycast (Raycasting section; Algorithm 1's pixel loop) every active
 * volume of `stream_id` into one shared map: per pixel the first
 * plus-to-minus zero crossing of the trilinear TSDF along the ray, the
 * nearest over all volumes winning (ties: lower volume id); normal = the
 * gradient of the trilinear interpolant.  out->width/height give the image
 * size. */
mvf_status mvf_raycast(mvf_ctx* ctx, int32_t stream_id, const float T_wc[12],
                       const mvf_intrinsics* K, const mvf_raycast_out* out, void* stream);

/* ---- batched form ------------------------------------------------------ */

typedef struct {
    int32_t stream_id;
    mvf_frame frame;
    float T_wc[12];
    mvf_intrinsics K;
} mvf_stream_frame;

/* Integrate frames[i] into the active volumes of frames[i].stream_id, then
 * raycast every stream at its frame's pose into outs[i], for all n streams
 * at once: one persistent integration launch and one persistent raycast
 * launch over a device volume table, captured once into a HIP graph and
 * replayed.  Results equal the plain calls bit for bit.  When the active
 * in-view volumes of the streams do not fit the budget together they are
 * processed in waves that do (swapping volumes in and out, Memory Passing
 * section), one graph replay per wave, the raycast of each wave merged
 * with the earlier ones per pixel; MVF_ERR_BUDGET only when one volume
 * alone exceeds the budget.  Steps split into waves are not autotuned. */
mvf_status mvf_step(mvf_ctx* ctx, int32_t n, const mvf_stream_frame* frames,
                    const mvf_raycast_out* outs, void* stream);

/* Launch schedule of mvf_step (no part of the paper's method: the batched
 * form's own tuning).  Every schedule gives the same results bit for bit.
 *   zchunk            bricks per integration work item along z: 1, 2, 4 or 8
 *   persistent        0: one integration wavefront per work item;
 *                     1: 8 wavefronts per SIMD walking the items
 *   ray_lanes         lanes that march one ray together: 2, 4 or 8 (pixel
 *                     tiles 8x4, 4x4, 4x2)
 * Default {4, 0, 4}. */
typedef struct {
    int32_t zchunk;
    int32_t persistent;
    int32_t ray_lanes;
    int32_t reserved;   /* 0 */
} mvf_schedule;

/* Fix the schedule of later mvf_step calls (and switch autotuning off).
 * MVF_ERR_INVALID_ARG for a value outside the lists above. */
mvf_status mvf_set_schedule(mvf_ctx* ctx, const mvf_schedule* sched);
/* The schedule the last mvf_step call ran with (the default before any). */
mvf_status mvf_get_schedule(mvf_ctx* ctx, mvf_schedule* out);

#define MVF_AUTOTUNE_OFF 0      /* fixed schedule (mvf_set_schedule or the default) */
#define MVF_AUTOTUNE_TUNE 1     /* tune shapes the cache does not hold */
#define MVF_AUTOTUNE_CACHED 2   /* use the cache; the default schedule for other shapes */
/* Autotuning of mvf_step.  A step shape is the stream count, the output
 * sizes, the number of volumes and their brick dimensions.  In TUNE mode
 * the first 120 steps of a new shape run blocks of eight steps, the default
 * schedule between each two of the 7 other candidates (timed with HIP events
 * on the call's stream; the step's results are unaffected); each block
 * counts by the mean of its last seven runs without their highest and lowest
 * (the first pays the graph capture), and the shape keeps the candidate
 * fastest relative to the mean of the default blocks around it.  Tune on
 * representative frames: the fastest schedule depends on how much of the
 * volumes the frames see.  cache_path (may be NULL: memory
 * only) is a JSON-lines file read now (missing file: empty cache) and
 * appended to whenever a shape is tuned; one line per shape:
 * {"key": "...", "zchunk": z, "persistent": p, "ray_lanes": l, "ms": t}.
 * The string is copied.  MVF_ERR_INVALID_ARG for an unknown mode, a line
 * that does not parse or a schedule outside the lists. */
mvf_status mvf_autotune(mvf_ctx* ctx, int32_t mode, const char* cache_path);

/* ---- placement (Dynamic Mapping for SLAM; Insertion and Removal) -------- */

typedef struct {
    int32_t grid_id;
    int32_t d_v;        /* voxels per side of placed volumes (>= 3) */
    int32_t n_max;      /* most volumes alive at once */
    float beta;         /* a newcomer must exceed beta x the lowest count; >= 1 */
} mvf_placement_params;

typedef struct {
    int32_t n_added, n_removed;
    int32_t added[64];     /* volume ids created and placed */
    int32_t removed[64];   /* volume ids evicted (state kept on the host) */
    int32_t n_cells;       /* distinct endpoint cells this frame */
    int32_t reserved;
} mvf_placement_result;

/* Count, per cell k of the placement lattice (side d_v - 2 voxels), the
 * valid depth rays of `frame` whose endpoint R (D K^-1 [u v 1]) + t falls in
 * it, then run the insertion f and removal g steps on the stream's volumes
 * created by this call: keep the n_max highest-count cells with hysteresis
 * beta; new volumes get offset k (d_v - 2) and dims d_v; removed volumes
 * are evicted and swapped out.  Synchronises on `stream`. */
mvf_status mvf_placement_update(mvf_ctx* ctx, int32_t stream_id, const mvf_frame* frame,
                                const float T_wc[12], const mvf_intrinsics* K,
                                const mvf_placement_params* p, mvf_placement_result* r,
                                void* stream);
/* Volumes of several sizes on one grid: the insertion/removal rule with
 * the size chosen by count rank (Dynamic Mapping for SLAM: f may set the
 * volume parameters).  Classes are taken in the given order, the first
 * taking the highest-count regions.  Class i counts, on its own lattice
 * (side classes[i].d_v - 2 voxels), only the endpoints that no live volume
 * of classes 0..i-1 (as updated this frame) contains, then keeps at most
 * classes[i].quota volumes by the same rule as mvf_placement_update (count
 * order, hysteresis beta, translations unique within a class).  A volume
 * whose endpoints a larger volume has taken over counts 0 and yields to the
 * next candidate that beats it.  With one class this is
 * mvf_placement_update.  Volumes are keyed per stream by (d_v, cell): a
 * cell seen before reuses its volume (state kept on the host).
 * MVF_ERR_INVALID_ARG for n_classes outside [1, MVF_MAX_PLACEMENT_CLASSES],
 * a d_v outside [3, 2048] or given twice, a negative quota or quotas summing
 * above 64.  n_cells in the result counts distinct (class, cell) pairs.
 * Synchronises on `stream` (one count and readback per class). */
#define MVF_MAX_PLACEMENT_CLASSES 8
typedef struct {
    int32_t d_v;    /* voxels per side of this class's volumes (>= 3) */
    int32_t quota;  /* most live volumes of this class (>= 0) */
} mvf_placement_class;

typedef struct {
    int32_t grid_id;
    int32_t n_classes;
    mvf_placement_class classes[MVF_MAX_PLACEMENT_CLASSES];
    float beta;         /* a newcomer must exceed beta x the lowest count; >= 1 */
    int32_t reserved;
} mvf_placement_class_params;

mvf_status mvf_placement_update_classes(mvf_ctx* ctx, int32_t stream_id, const mvf_frame* frame,
                                        const float T_wc[12], const mvf_intrinsics* K,
                                        const mvf_placement_class_params* p, mvf_placement_result* r,
                                        void* stream);
/* User-defined insertion f (Dynamic Volume Allocation, Input and Output: f
 * and g may be any functions of the frames and the live volumes; Dynamic
 * Mapping for SLAM, e.g. a higher resolution where an application wants
 * it).  For each class in order the library counts the endpoints on the
 * device exactly as mvf_placement_update_classes does (excluding those held
 * by live volumes of the earlier classes), then calls fn on the host with:
 * the class index and d_v; the class's live cells (n_live x 3 ints); this
 * frame's (cell, count) pairs (n_cells); the class quota.  fn writes the
 * class's live cells after the update (at most quota, no cell twice) to
 * keep (3 ints each, room for quota cells) and their number to *n_keep, and
 * returns 0 (non-zero aborts with MVF_ERR_STATE; cells already placed or
 * removed for earlier classes stay so).  The removal g follows: live cells
 * not kept are evicted and swapped out; kept cells not live are placed
 * (reusing the volume a cell had before).  beta is not used.  Other errors
 * as mvf_placement_update_classes; MVF_ERR_INVALID_ARG when fn keeps too
 * many cells, one twice, or one whose offset k (d_v - 2) lies beyond 2^22.
 * The arrays passed to fn are valid during the call only. */
typedef int32_t (*mvf_placement_fn)(void* user, int32_t class_index, int32_t d_v, const int32_t* live,
                                    int32_t n_live, const int32_t* cells, const int32_t* counts,
                                    int32_t n_cells, int32_t quota, int32_t* keep, int32_t* n_keep);
mvf_status mvf_placement_update_custom(mvf_ctx* ctx, int32_t stream_id, const mvf_frame* frame,
                                       const float T_wc[12], const mvf_intrinsics* K,
                                       const mvf_placement_class_params* p, mvf_placement_fn fn,
                                       void* user, mvf_placement_result* r, void* stream);
/* The endpoint counts alone: up to max_cells (cell xyz, count) tuples written
 * to host `cells` (3 ints) and `counts`; *n_cells = number of distinct cells.
 * Synchronises on `stream`. */
mvf_status mvf_placement_count(mvf_ctx* ctx, const mvf_frame* frame, const float T_wc[12],
                               const mvf_intrinsics* K, int32_t grid_id, int32_t d_v,
                               int32_t* cells, int32_t* counts, int32_t max_cells,
                               int32_t* n_cells, void* stream);
/* Host-only insertion/removal step on cell keys (no device work).  active:
 * n_active cells (3 ints each) in H; counts: n_cells (cell, count) pairs.
 * Writes the new active set (out_active, up to n_max cells), the added and
 * removed cells (each up to n_active + n_cells) and their numbers. */
mvf_status mvf_placement_policy(const int32_t* active, int32_t n_active, const int32_t* cells,
                                const int32_t* counts, int32_t n_cells, int32_t n_max,
                                float beta, int32_t* out_active, int32_t* n_out,
                                int32_t* added, int32_t* n_added, int32_t* removed,
                                int32_t* n_removed);

/* ---- camera tracking (Depth Map Conversion; Camera Tracking) ------------ */

/* The model the frame is tracked against: the vertex and normal maps of
 * the last raycast (as written by mvf_raycast / mvf_step: world frame,
 * NaN where no surface), device float32 height x width x 3 each, and the
 * camera-to-world pose they were rendered from. */
typedef struct {
    const float* vertex;
    const float* normal;
    int32_t width, height;
    float T_wc[12];
} mvf_track_model;

typedef struct {
    int32_t levels;     /* pyramid levels, 1..3 */
    int32_t iters[3];   /* Gauss-Newton steps at levels 0 (full), 1, 2; run coarse to fine; <= 64 in all */
    float eps_d;        /* association distance, metres (> 0) */
    float cos_theta;    /* association normal test |n . n_model| >= cos_theta, in [0, 1] */
    float tau;          /* pyramid: depths within tau metres of the 2x2 block's first valid one */
    float smooth;       /* smoothing window: neighbours within this many metres of the centre depth; 0 = none */
} mvf_track_params;

typedef struct {
    int32_t steps;          /* Gauss-Newton steps run */
    int32_t pairs[64];      /* per step: associated pairs */
    double sq_err[64];      /* per step: sum of squared point-to-plane residuals (m^2) */
} mvf_track_stats;

/* Depth Map Conversion alone: the vertex map v = K^-1 [x y 1]^T D and the
 * normal map (v(x+1, y) - v(x, y)) x (v(x, y+1) - v(x, y)), normalised, of
 * pyramid level `level` (0..2; smoothing and pyramid as in mvf_track, with
 * smooth and tau), in camera coordinates, NaN where undefined: device
 * float32 V and N of (height >> level) x (width >> level) x 3 each.  Runs
 * on `stream` and synchronises it (to free its temporaries). */
mvf_status mvf_depth_maps(mvf_ctx* ctx, const mvf_frame* frame, const mvf_intrinsics* K, int32_t level,
                          float tau, float smooth, float* V, float* N, void* stream);
/* Pose of a depth frame by projective point-to-plane ICP (Camera Tracking:
 * the KinectFusion tracker the paper cites), from the estimate T_init
 * (host, row-major 3x4 camera-to-world, binary64) to T_out.
 * The depth is first smoothed (smooth > 0): a valid pixel takes the mean of
 * the valid depths of its 7x7 window within `smooth` metres of its own,
 * weighted by the binomial C(6, dx + 3) C(6, dy + 3) (an edge-preserving
 * filter, as the KinectFusion tracker smooths its input).
 * Depth map conversion: vertex v = K^-1 [x y 1]^T D, normal n = (v(x+1, y)
 * - v(x, y)) x (v(x, y+1) - v(x, y)) normalised; a pyramid of `levels`
 * depth maps, level l+1 the mean of each 2x2 block's valid depths within
 * tau of its first valid one, with intrinsics f / 2^l, (c + 1/2) / 2^l -
 * 1/2; the model maps of level l+1 take the sample (2x, 2y) of level l.
 * Each step associates every pixel with a valid vertex and normal: v_g =
 * T v is projected into the model's camera to the nearest pixel; the pair
 * counts when that pixel holds a model vertex v_m, |v_g - v_m| <= eps_d and
 * |R n . n_m| >= cos_theta.  With r = n_m . (v_g - v_m) and J = [n_m,
 * v_g x n_m] the step solves (sum J J^T) xi = -sum J r (binary64, Cholesky)
 * and sets T <- Exp(xi) T, xi = (rho, omega); a step with fewer than 6
 * pairs or a matrix that is not positive definite leaves T unchanged.
 * Decisions are binary32 (the estimate rounded to binary32), sums binary64.
 * The model maps must have the frame's size.  Runs on `stream`, all steps
 * without a host round trip, then synchronises it.  stats may be NULL. */
mvf_status mvf_track(mvf_ctx* ctx, const mvf_frame* frame, const mvf_intrinsics* K,
                     const mvf_track_model* model, const double T_init[12], const mvf_track_params* p,
                     double T_out[12], mvf_track_stats* stats, void* stream);

/* ---- differentiable raycast ------------------------------------------- */

typedef struct {
    const float* F;      /* device, dims[2] x dims[1] x dims[0] x-fastest, truncation units */
    const uint16_t* W;   /* device, same layout; W == 0 marks unobserved voxels */
    int32_t dims[3];
    int32_t offset[3];
    float origin[3];
    float voxel_size;
    /* 0: F and W may have changed since the last call.  Otherwise the
     * caller's promise that they are unchanged since the last forward call
     * with the same pointers, description and generation; bump it after
     * changing either plane. */
    uint64_t generation;
} mvf_dense_tsdf;

/* Raycast depth of one dense volume (same rules as mvf_raycast) and a
 * per-pixel record of the crossing (k of the second sample, -1 = none),
 * device int32 H*W.  The context keeps a brick-layout copy of the volume
 * (an internal volume with its skip summaries, counted against the device
 * budget), rebuilt from F and W unless the generation rule above lets the
 * last one stand; the march is that of mvf_raycast.  dims <= 2048 per axis
 * and at most 2^30 voxels once padded to 8^3 bricks. */
mvf_status mvf_diffray_forward(mvf_ctx* ctx, const mvf_dense_tsdf* v, const float T_wc[12],
                               const mvf_intrinsics* K, int32_t width, int32_t height,
                               float* depth, int32_t* record, void* stream);
/* Backward of L given dL/d(depth) (device H*W): with the crossings of the
 * forward record held fixed, accumulate dL/dF into grad_F (device, same
 * layout as F; may be NULL) and write dL/dxi for the right pose
 * perturbation T_wc Exp(xi), xi = (rho, omega), to grad_xi (device, 6
 * doubles).  The two bracketing ray samples are recomputed, not stored. */
mvf_status mvf_diffray_backward(mvf_ctx* ctx, const mvf_dense_tsdf* v, const float T_wc[12],
                                const mvf_intrinsics* K, int32_t width, int32_t height,
                                const float* grad_depth, const int32_t* record,
                                float* grad_F, double* grad_xi, void* stream);
/* mvf_diffray_backward without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results;
 * the per-block pose partials go to a static device array of the library
 * (768 KiB per GPU, held until the process ends) instead of a buffer the
 * context allocates.  Limit: ceil(width / 16) * ceil(height / 16) <= 16384
 * (e.g. 2048 x 2048); larger images return MVF_ERR_INVALID_ARG.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (other
 * streams, other contexts or threads) race and must be serialised by the
 * caller. */
mvf_status mvf_diffray_backward_noalloc(mvf_ctx* ctx, const mvf_dense_tsdf* v, const float T_wc[12],
                                        const mvf_intrinsics* K, int32_t width, int32_t height,
                                        const float* grad_depth, const int32_t* record,
                                        float* grad_F, double* grad_xi, void* stream);
/* Host-only: T_out = T Exp(xi) for xi = (rho, omega) (binary64 3x4). */
mvf_status mvf_pose_retract(const double T[12], const double xi[6], double T_out[12]);
/* Host-only: the right Jacobian J (6x6 row-major, binary64) of Exp at xi:
 * T Exp(xi + d) = T Exp(xi) Exp(J d) to first order in d.  A gradient g
 * with respect to the right perturbation at T Exp(xi) (what
 * mvf_diffray_backward returns) is a gradient with respect to xi itself
 * after g <- J^T g. */
mvf_status mvf_pose_right_jacobian(const double xi[6], double J[36]);

#ifdef __cplusplus
}
#endif

#endif /* MVF_H */
