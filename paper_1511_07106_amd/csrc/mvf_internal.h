// Internal types shared by the host runtime (mvf_runtime.cpp) and the HIP
// kernels (mvf_kernels.hip).  Not part of the public ABI.
//
// Device volume layout ("brick-linear"): a volume of dims (nx, ny, nz) is
// padded to bricks of 8x8x8 voxels, bd = ceil(dims / 8) bricks per axis.
// Bricks are numbered z-fastest, brick(bx, by, bz) = (bx * bd.y + by) * bd.z
// + bz, so a column of bricks (fixed bx, by) is one contiguous run.  Inside a
// brick voxels are x-fastest: (z & 7) * 64 + (y & 7) * 8 + (x & 7); one
// z-slice of a brick is 64 consecutive elements, exactly one wavefront.
//
// Planes, each padded to a 256-byte multiple, in one slab per volume:
//   F     float32  TSDF in truncation units; NaN while the voxel is
//                  unobserved (W == 0), so one trilinear read both
//                  interpolates and tests that all 8 corners were observed
//   W     uint16   running weight
//   C     uint32   RGBA8 colour, A = colour weight
//   flag  uint8    per brick: 1 if some voxel of the brick may hold
//                  F <= 2^-100 (set by integration, never cleared except by
//                  a full recompute); 0 guarantees F > 0 or NaN everywhere
//                  in the brick, which lets the raycast skip it exactly.
//   dist  uint8    per brick: Chebyshev distance, in bricks, to the nearest
//                  flagged brick, capped at kDistCap (0 = flagged); every
//                  brick within dist - 1 of this one is unflagged.  Derived
//                  from the flags after each integration.
//   colm  uint64   per brick column (bx, by) and 64 bricks of it along z:
//                  word (bx * bd[1] + by) * col_words(bd[2]) + (bz >> 6),
//                  bit bz & 63 equal to the brick's flag (maintained with
//                  the flags; the distance transform reads only these),
//                  then one word that is always zero.
//   fmask uint64   per brick: bit z2 * 16 + y2 * 4 + x2 set if some voxel of
//                  the 2x2x2 sub-block (x2, y2, z2) of the brick may hold
//                  F <= 2^-100 (same monotone rule as flag, which equals
//                  fmask != 0).
//   cmask uint64   per brick: the same bits for cells: bit (x2, y2, z2) set
//                  if a voxel of [2 x2, 2 x2 + 2] x [2 y2, 2 y2 + 2] x
//                  [2 z2, 2 z2 + 2] (brick-local, reaching into the +x, +y,
//                  +z neighbour bricks) may hold F <= 2^-100, i.e. some cell
//                  whose base voxel lies in that sub-block may have a corner
//                  F <= 2^-100.  fmask dilated by one sub-block; derived
//                  after each integration with the distance transform.
#pragma once
#include <stdint.h>

#ifndef MVF_HD
#if defined(__HIPCC__)
#define MVF_HD __host__ __device__ __forceinline__
#else
#define MVF_HD inline
#endif
#endif

namespace mvf {

constexpr int kBrick = 8;
constexpr int kBrickVox = 512;
constexpr float kFlagThreshold = 0x1p-100f;
constexpr int kDistCap = 12;

// 64-bit words per brick column of the colm flag bits
MVF_HD int col_words(int bd2) { return (bd2 + 63) >> 6; }

struct DevVolume {
    float* F;
    uint16_t* W;
    uint32_t* C;
    uint8_t* flag;
    uint8_t* dist;
    uint64_t* colm;          // per brick column: flags as bits along z
    uint64_t* fmask;         // per brick: sub-block flags
    uint64_t* cmask;         // per brick: cell sub-block flags
    int32_t dims[3];
    int32_t off[3];
    int32_t bd[3];
    int32_t id;          // public volume id (hit output, tie-break)
    float o[3];          // grid origin
    float s;             // voxel size
    float inv_s;         // 1 / s (binary32, correctly rounded)
    float mu;            // trunc_voxels * s (binary32)
    float inv_mu;        // 1 / mu
    int32_t w_max;
    int32_t frame;       // index of the stream's frame in the frame table
    int32_t zt_base;     // first entry of this volume in the launch's z table
};

struct DevFrame {
    const float* range;      // H*W: depth * ray-length factor, 0 = invalid
    const uint32_t* color;   // H*W packed RGB (may be null)
    float* rmax;             // [0]: max range of the frame (for clipping); [1 + b]: per prep block
    int32_t rmax_parts;      // prep blocks of this frame (ceil(width / 32) * ceil(height / 8))
    const float* tmax;       // maximum range of each 8x8 pixel tile (row-major), then the minimum of each
                             // (tiles_x * tiles_y further on; 0 where a pixel has no range), or null
    int32_t tiles_x, tiles_y;
    int32_t width, height;
    float fx, fy, cx, cy;
    float T[12];
    // raycast outputs
    float* depth;
    float* vertex;
    float* normal;
    int32_t* hit;
    float* best_t;           // per-pixel running best (multi-wave raycast)
    int32_t* best_id;
    int32_t* record;         // per pixel: k of the nearest crossing's second sample, -1 = none; or null
    int32_t out_w, out_h;
    // raycast range bounds per 8x8 output-pixel cell (cells_x * cells_y,
    // row-major), or null: the nearest and farthest camera distance of any
    // sample the march may have to evaluate; a cell no brick reaches holds
    // (inf, 0).  Written by launch_ray_bounds_merge.
    float* rb_lo;
    float* rb_hi;
    int32_t cells_x, cells_y;
};

struct RayParams {
    float delta;             // step * s (binary32); all volumes of a call share one grid
    int32_t kmax;            // floor(t_far / delta)
};

// 64-bit counters written by kernels.  kCntSlots copies, each on its own
// 128-byte line (slot k at counters + k * kCntNum), spread the atomics of
// many blocks over several addresses; a reader sums the slots.
enum Counter { kCntUpdated = 0, kCntBand = 1, kCntBricks = 2, kCntDeep = 3, kCntNum = 16 };
constexpr int kCntSlots = 64;

// Launch parameters that live in device memory, so that a captured graph
// replays with new tables (volume set, frame pointers, poses) without
// re-capture.
struct LaunchHeader {
    int32_t nvol;          // entries of the volume table used by integration
    int32_t total_items;   // integration work items
    int32_t zchunk;        // bricks per integration item along z
    int32_t nstreams;      // frames in the frame table
    int32_t total_tiles;   // raycast pixel tiles over all streams
    int32_t total_bricks;  // bricks over all volumes of the table (distance transform)
    int32_t first_wave;    // raycast: 1 = start from no hit, 0 = merge with best_t/best_id
    RayParams rp;
    int32_t total_z;       // entries of the integration z table (sum of 8 * bd[2])
    int32_t rb_parity;     // raycast range bounds: which half of RayBounds::counts this launch fills
    int32_t list_parity;   // integration: which of the two visited-item counts this launch uses
};

// Footprint of one brick in the raycast range bounds: cells [x0, x1] x
// [y0, y1] of its volume's frame and the camera distances [dn, df] of its box.
struct RayBoundEntry {
    uint16_t x0, x1, y0, y1;
    float dn, df;
};

// Range-bound footprints of a launch.  Volume v of the table appends to
// entries + brick_base[v] (room for all its bricks) and counts its entries
// in counts[rb_parity * cap + v]; the merge reads them and clears the other
// half for the next launch.
struct RayBounds {
    RayBoundEntry* entries;
    uint32_t* counts;          // 2 * cap, zero before first use
    int32_t cap;               // volume slots per half (>= nvol)
};

// Frame preparation input for one stream.
struct PrepItem {
    const float* depth;
    const uint8_t* rgb;
    int32_t depth_pitch, rgb_pitch;
    int32_t width, height;
    float fx, fy, cx, cy;
    float* range;
    uint32_t* color;
    float* rmax;             // [0] frame's maximum range, [1 + b] maximum of prep block b
    float* tmax;             // maximum range of each 8x8 pixel tile, ceil(width / 8) per row; the
                             // minima follow (ceil(width / 8) * ceil(height / 8) further on)
};

// Integration work item: a brick column (8x8 voxel columns) of one volume
// over a chunk of zchunk bricks along z.  Items of table entry v are
// [item_base[v], item_base[v+1]).
//
// z table: for volume v and local z in [0, 8 * bd[2]), entry
// vols[v].zt_base + z holds 3 floats: T[8], T[9], T[10] times
// (x_w(z) - T[11]), the camera-frame offset of the voxel plane z (binary32,
// the same operations as the voxel test).  Written by launch_ztable before
// the integration kernel runs; ztab holds >= hdr->total_z entries.
struct IntegrateLaunch {
    const LaunchHeader* hdr;
    const DevVolume* vols;
    const DevFrame* frames;
    const int32_t* item_base;  // nvol + 1 prefix sums
    unsigned long long* counters;
    float* ztab;
    // per item, kVisitPerItem bytes: byte j is 1 if brick bz0 + j of the
    // item may hold a voxel the frame updates (written by the z-table
    // launch), or null (visit all); needs zchunk <= kVisitPerItem
    uint8_t* visit;
    // optional: block 0 computes a raycast tile order (see launch_tile_order)
    // from these costs instead of integrating; the grid has one more block
    const uint32_t* tile_cost;
    int32_t* tile_order;
    int32_t order_tiles;
    // visited work, compacted (needs visit): the z-table launch appends
    // every brick to visit voxel by voxel to list and every deep brick (each
    // voxel updated with phi = 1, proved by the visit test) to deep_list,
    // both as item * 8 + j (brick j of the item; room for total_items *
    // zchunk each); list_count[hdr->list_parity] counts both (visited bricks
    // in the low 32 bits, deep bricks in the high 32).  Integration gives
    // each entry a wavefront, the visited bricks first.  The z-table launch
    // also zeroes list_count[list_parity ^ 1] for the next launch, so the
    // two words must be zero before first use.
    int32_t* list;
    unsigned long long* list_count;
    int32_t* deep_list;
};
constexpr int kVisitPerItem = 8;

// Lanes that march one ray together in the raycast kernel (P consecutive
// samples per round of gathers: 2, 4 or 8), and the pixel tile of a
// 64-lane block for each (8x4, 4x4, 4x2).  kRayLanes is the default.
constexpr int kRayLanes = 4;
MVF_HD int ray_tile_w(int lanes) { return lanes == 2 ? 8 : 4; }
MVF_HD int ray_tile_h(int lanes) { return 64 / lanes / ray_tile_w(lanes); }
constexpr int kBoundCell = 8;   // output pixels per side of a raycast range-bound cell (a ray tile lies in one)
// Raycast launch order: groups of kRayGroup consecutive tiles are ordered by
// their summed last duration, slowest first.  Blocks are dealt round-robin
// over the 8 XCDs, so a window of 8 * kRayGroup blocks takes 8 groups, each
// group's tiles on one XCD (they gather the same bricks).
constexpr int kRayGroup = 4;
constexpr int kXcds = 8;
MVF_HD int ray_groups(int tiles) { return (tiles + kRayGroup - 1) / kRayGroup; }
MVF_HD int ray_blocks(int tiles) { return (ray_groups(tiles) + kXcds - 1) / kXcds * kXcds * kRayGroup; }

struct RaycastLaunch {
    const LaunchHeader* hdr;
    const DevVolume* vols;      // table
    const DevFrame* frames;     // one per stream
    const int32_t* lists;       // concatenated per-stream lists of table indices, nearest first
    const int32_t* list_base;   // per stream: [list_base[s], list_base[s+1])
    const int32_t* tile_base;   // per stream: first pixel tile; nstreams + 1 entries
    int32_t tile_w, tile_h;     // pixel tile: ray_tile_w(lanes) x ray_tile_h(lanes)
    int32_t lanes;              // lanes per ray (2, 4 or 8)
    uint32_t* tile_cost;        // per tile: its duration in the last launch (10 ns ticks), or null
    const int32_t* tile_order;  // tile groups in launch order, or null (index order)
};

// Host-side launchers (defined in mvf_kernels.hip).  All return hipError_t
// as int (0 = success).
// Frame preparation of n frames.  With tsrc set (a captured step) the items
// are read from pinned host memory and the launch also copies tbytes (a
// multiple of 16, 16-byte aligned) from tsrc to tdst; set_frame_prep_node
// points such a node of an instantiated graph at another host slot.
int launch_frame_prep(const PrepItem* items, int n, int max_w, int max_h, void* stream, const void* tsrc = nullptr,
                      void* tdst = nullptr, size_t tbytes = 0);
int set_frame_prep_node(void* exec, void* node, const PrepItem* items, int n, int max_w, int max_h, const void* tsrc,
                        void* tdst, size_t tbytes);
int launch_volume_init(DevVolume v, void* stream);
// The z table of a launch and, when L.visit is set, the visit pass over
// the launch's `bricks` bricks (total_items * zchunk; one thread per brick,
// up to 2048 blocks of 512 threads, which then walk the rest); must precede
// launch_integrate on the stream.
int launch_ztable(const IntegrateLaunch& L, int bricks, void* stream);
// Integration kernel: blocks of 256 threads, 4 items in flight per block; a
// grid smaller than total_items / 4 walks the items (plus block 0 when
// L.tile_order is set).
// With ev_start/ev_stop (hipEvent_t) the kernel's own dispatch records them.
int launch_integrate(const IntegrateLaunch& L, int blocks, void* stream, void* ev_start = nullptr,
                     void* ev_stop = nullptr);
// Raycast kernel over ray_blocks(total tiles) blocks (or fewer: a grid-stride loop).
int launch_raycast(const RaycastLaunch& L, int blocks, void* stream, void* ev_start = nullptr,
                   void* ev_stop = nullptr);
// Launch order of the ray_groups(n) groups of n raycast tiles from their
// last durations, longest first (a slow tile started late bounds the launch).
int launch_tile_order(const uint32_t* cost, int32_t* order, int n, void* stream);
int launch_brick_summary(DevVolume v, void* stream);
// Brick distance transform of every volume in the table (3 passes).
// brick_base: nvol + 1 prefix sums of the volumes' brick counts (each a
// multiple of 64).  With frames and rb.entries set, the last pass also
// collects the range-bound footprints (as launch_ray_bounds_collect).
int launch_brick_distance(const LaunchHeader* hdr, const DevVolume* vols, const int32_t* brick_base,
                          int blocks, void* stream, const DevFrame* frames = nullptr, RayBounds rb = RayBounds{});
// Range-bound footprints of the bricks of every volume of the table whose
// cell mask is not empty, for the volume's frame.
int launch_ray_bounds_collect(const LaunchHeader* hdr, const DevVolume* vols, const int32_t* brick_base,
                              const DevFrame* frames, RayBounds rb, int blocks, void* stream);
// Range bounds of every cell of each stream's frame from the footprints of
// the stream's volumes (lists / list_base as in RaycastLaunch); clears the
// other half of rb.counts.  max_cells_x/y: largest cell grid of the frames.
int launch_ray_bounds_merge(const LaunchHeader* hdr, const DevFrame* frames, const int32_t* lists,
                            const int32_t* list_base, const int32_t* brick_base, RayBounds rb, int nstreams,
                            int max_cells_x, int max_cells_y, void* stream);
int launch_to_canonical(DevVolume v, float* F, uint16_t* W, uint32_t* C, void* stream);
int launch_from_canonical(DevVolume v, const float* F, const uint16_t* W, const uint32_t* C,
                          void* stream);
// Surface points of one volume: per-brick counts, their exclusive prefix sum
// (offsets, nbricks entries; total[0] = the sum) and, when cap > 0, the
// emission of the first cap points (V, N: 3 floats each; G: 3 ints, or null)
// in brick order.  counts: nbricks entries.
int launch_extract(DevVolume v, uint32_t* counts, unsigned long long* offsets, long long* total, float* V,
                   float* N, int32_t* G, long long cap, void* stream);
int launch_fill_u64(unsigned long long* p, int n, unsigned long long value, void* stream);
int launch_placement_clear(unsigned long long* table, int table_size, void* stream);
int launch_placement_count(const float* depth, int depth_pitch, int width, int height,
                           float fx, float fy, float cx, float cy, const float* T,
                           float o0, float o1, float o2, float cell,
                           unsigned long long* table, int table_size, int* overflow,
                           const int32_t* boxes, int n_boxes, float voxel, void* stream);

// Camera tracking (mvf_track.hip).  The pose estimate and the statistics of
// every Gauss-Newton step live in device memory.
constexpr int kTrackSums = 29;          // A (21, upper triangle), b (6), pairs, sum r^2
constexpr int kTrackThreads = 256;
constexpr int kTrackPixPerThread = 4;
constexpr int kTrackMaxSteps = 64;

struct TrackState {
    double T[12];        // estimate, camera-to-world, row-major 3x4
    float T32[12];       // its binary32 rounding (the association reads it)
    int32_t steps;
    int32_t pairs[kTrackMaxSteps];
    double sq_err[kTrackMaxSteps];
};

struct TrackLaunch {
    const float* V;      // current level: vertex and normal maps, w x h x 3, camera frame
    const float* N;
    int32_t w, h;
    const float* Vm;     // model level: world maps of the same size
    const float* Nm;
    float fx, fy, cx, cy;
    float Tm[12];        // the model's camera-to-world pose
    float eps_d, cos_theta;
    TrackState* state;
    double* partials;    // track_blocks(w, h) x kTrackSums
    uint8_t* inlier;     // per current pixel, or null
};

// Edge-preserving smoothing of a depth map (out: w x h, pitch w).
int launch_track_smooth(const float* D, int pitch, int w, int h, float delta, float* out, void* stream);
int launch_track_down(const float* D, int pitch, int w, int h, float tau, float* D2, void* stream);
int launch_track_vn(const float* D, int pitch, int w, int h, const float K[4], float* V, float* N, void* stream);
int launch_track_model_down(const float* V, const float* N, int w, int h, float* V2, float* N2, void* stream);
int track_blocks(int w, int h);
// Association + reduction, then the solve and update of step `step`.
int launch_icp_step(const TrackLaunch& L, TrackState* state, int step, void* stream);
int launch_track_init(TrackState* state, void* stream);

struct DiffVolume {
    const float* F;
    const uint16_t* W;
    int32_t dims[3];
    int32_t off[3];
    float o[3];
    float s, inv_s;
};
int launch_diffray_backward(DiffVolume v, const float* T, float fx, float fy, float cx, float cy,
                            int width, int height, RayParams rp, const float* grad_depth,
                            const int32_t* record, float* grad_F, double* partials,
                            int n_partials, double* grad_xi, void* stream);
int diffray_partials_needed(int width, int height);
// Allocation-free backward: a static device array holds the pose partials of
// at most kDiffScratchBlocks 16x16-pixel blocks (768 KiB per GPU).
constexpr int kDiffScratchBlocks = 16384;
constexpr int kMaxDevices = 64;
// Take the current device's address of the static array (once per device;
// the device must be current).  0 on success, else a hipError_t.
int diffray_scratch_init(int device);
// That address, or null before diffray_scratch_init(device) succeeded.
double* diffray_scratch(int device);

}  // namespace mvf
