// Host runtime of libmvf: context, grid/volume registry, residency manager
// (device budget, slab pool, pinned host mirrors, swaps on a side copy
// stream ordered by events), launch-table arena, the plain per-volume
// integrate/raycast, the batched graph-captured step, placement, the
// differentiable raycast, read/write and statistics.  Implements include/mvf.h.
// Paper: Salvato, Finman, Leonard, arXiv 1511.07106.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_internal.h"

using namespace mvf;

namespace {

thread_local std::string g_last_error;

mvf_status set_error(mvf_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define CHECK_HIP(call)                                                                        \
    do {                                                                                       \
        hipError_t e__ = (call);                                                               \
        if (e__ != hipSuccess)                                                                 \
            return set_error(MVF_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e__));    \
    } while (0)

#define CHECK_LAUNCH(call)                                                                     \
    do {                                                                                       \
        int e__ = (call);                                                                      \
        if (e__ != 0)                                                                          \
            return set_error(MVF_ERR_HIP, "%s failed: %s", #call,                              \
                             hipGetErrorString((hipError_t)e__));                              \
    } while (0)

#define CHECK_ST(call)                   \
    do {                                 \
        mvf_status s__ = (call);         \
        if (s__ != MVF_OK) return s__;   \
    } while (0)

constexpr size_t kAlign = 256;
// scratch slot of the differentiable raycast (public stream ids are >= 0)
constexpr int kDiffStream = -1;
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Grid {
    mvf_grid_desc d;
    float mu, inv_s, inv_mu;
};

enum class State { Empty, Device, Host };

struct Volume {
    bool alive = false;
    mvf_volume_desc d{};
    int bd[3] = {0, 0, 0};
    size_t nvox_pad = 0, off_W = 0, off_C = 0, off_flag = 0, off_dist = 0, off_colm = 0, off_fmask = 0, off_cmask = 0, bytes = 0;
    size_t nbricks = 0;
    uint8_t* dev = nullptr;    // device slab while resident
    uint8_t* host = nullptr;   // pinned mirror (allocated on first swap-out)
    State state = State::Empty;
    bool active = false;
    uint64_t last_use = 0;
    hipEvent_t host_ready = nullptr;  // mirror written (swap-out finished)
    bool host_pending = false;
    bool internal = false;  // the library's own (the differentiable raycast's mirror): no public id
};

// Swaps move a slab in chunks of kSwapChunk bytes, each with its own event,
// so that a swap-in into a slab still being swapped out copies chunk k as
// soon as the download of chunk k is done: the two directions of the host
// link then run at once.
constexpr size_t kSwapChunk = (size_t)64 << 20;

struct Slab {
    uint8_t* ptr;
    size_t bytes;
    std::vector<hipEvent_t> chunk_done;  // download of chunk k finished (on d2h_stream); the last: all
};

struct Scratch {
    int w = 0, h = 0;
    float* range = nullptr;
    uint32_t* color = nullptr;
    float* rmax = nullptr;   // [0] max range, [1 + b] per frame-prep block
    int rmax_cap = 0;        // floats in rmax
    float* best_t = nullptr;
    int32_t* best_id = nullptr;
    int best_cap = 0;           // pixels best_t / best_id hold
    float* ztab = nullptr;  // integration z table (3 floats per entry)
    int ztab_cap = 0;
    float* tmax = nullptr;   // maximum range per 8x8 pixel tile, then the minima (2 x tmax_cap)
    int tmax_cap = 0;
    uint8_t* visit = nullptr;  // integration: brick visit mask per item
    int visit_cap = 0;
    int32_t* list = nullptr;   // integration: visited bricks, then deep bricks (8 per item each)
    unsigned long long* list_count = nullptr;  // two count words, zeroed at allocation
    int list_parity = 0;
    uint32_t* tile_cost = nullptr;  // raycast tiles: last duration, then launch order
    int32_t* tile_order = nullptr;
    int tiles_cap = 0;
    int last_tiles = 0;         // tiles of the stream's last raycast (0: none yet)
    int order_ready_tiles = 0;  // an integration ordered that many tiles for the next raycast
    float* rb_lo = nullptr;  // raycast range bounds per 8x8 output-pixel cell
    float* rb_hi = nullptr;
    int rb_cap = 0;
    RayBoundEntry* rb_entries = nullptr;  // plain raycast: footprints of a launch's bricks
    int rb_entries_cap = 0;
    uint32_t* rb_counts = nullptr;        // 2 halves of rb_counts_cap volume slots
    int rb_counts_cap = 0;
    int rb_parity = 0;
};

// Ring of pinned host + device slots for per-launch tables.  A slot is
// reused only after an event recorded behind the launches that read it.
// Captured steps release their slots in batches of kBatch behind one event
// (each event record between two graph launches cost the step 3-6 us); the
// batch's last slot is the latest in ring order, so every slot of a batch is
// reacquired, and has waited, before that slot's event is recorded again.
struct Arena {
    static constexpr int kSlots = 32;
    static constexpr int kBatch = 4;
    static constexpr size_t kSlotBytes = 1 << 20;
    uint8_t* host = nullptr;
    uint8_t* dev = nullptr;
    hipEvent_t ev[kSlots] = {};
    hipEvent_t wait_ev[kSlots] = {};   // the event a pending slot waits on before reuse
    bool pending[kSlots] = {};
    int next = 0;
    int open[kBatch] = {};             // step slots released since the last record
    int n_open = 0;
    hipStream_t open_stream = nullptr;
};

struct Writer {
    uint8_t* host;
    uint8_t* dev;
    size_t used = 0;
    bool overflow = false;
    template <class T>
    T* alloc(size_t n, T** dev_ptr)
    {
        size_t off = align_up(used, 64);
        size_t sz = sizeof(T) * (n ? n : 1);
        if (off + sz > Arena::kSlotBytes) { overflow = true; return nullptr; }
        used = off + sz;
        *dev_ptr = reinterpret_cast<T*>(dev + off);
        return reinterpret_cast<T*>(host + off);
    }
};

struct TimedPair {
    hipEvent_t a, b;
    int kind;  // 0 integrate, 1 raycast, 2 batched step
};

struct StepGraph {
    bool valid = false;
    int n = 0;
    std::vector<int> widths, heights, out_w, out_h;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy_node = nullptr;  // frame preparation, which also uploads the tables (the root)
    // persistent device tables read by the captured kernels
    uint8_t* dev = nullptr;
    size_t dev_bytes = 0;
    size_t off_hdr, off_prep, off_frames, off_vols, off_items, off_lists, off_lbase, off_tbase, off_bbase;
    int max_vols = 0, max_w = 0, max_h = 0;
    int integ_blocks = 0, ray_tiles = 0, ray_blocks = 0;
    float* ztab = nullptr;  // integration z table read by the captured launch
    int ztab_cap = 0;
    uint8_t* visit = nullptr;  // brick visit mask per integration item
    int visit_cap = 0;
    int32_t* list = nullptr;   // integration: visited bricks, then deep bricks (8 per item each)
    unsigned long long* list_count = nullptr;  // two count words, zeroed at allocation
    int list_parity = 0;
    RayBoundEntry* rb_entries = nullptr;  // raycast range-bound footprints (one per brick)
    int rb_entries_cap = 0;
    uint32_t* rb_counts = nullptr;        // 2 * max_vols
    int rb_parity = 0;
    int max_cells_x = 0, max_cells_y = 0;
    mvf_schedule sched{4, 0, kRayLanes, 0};  // schedule the graph was captured with
    uint32_t* tile_cost = nullptr;  // raycast tiles: last duration, then launch order
    int32_t* tile_order = nullptr;
};

}  // namespace

struct mvf_ctx {
    mvf_config cfg{};
    int device = 0;
    hipStream_t d2h_stream = nullptr;  // swap-out copies
    hipStream_t h2d_stream = nullptr;  // swap-in copies
    hipEvent_t h2d_last = nullptr;     // after the latest swap-in copies (swap-outs wait for it)
    std::vector<Grid> grids;
    std::vector<Volume> vols;
    std::map<int, Scratch> scratch;
    unsigned long long* counters = nullptr;
    uint64_t budget = 0;
    uint64_t resident_bytes = 0;  // slabs held by resident volumes
    uint64_t pooled_bytes = 0;    // slabs in the free pool
    std::vector<Slab> pool;
    uint64_t tick = 0;
    // failure injection for tests: this many of the next volume-slab
    // allocations fail as if the device were out of memory (from the
    // environment variable MVF_FAULT_SLAB_ALLOCS at context creation)
    int fault_slab_allocs = 0;
    mvf_stats stats{};
    Arena arena;
    std::vector<TimedPair> timed;
    std::vector<hipEvent_t> event_pool;
    hipEvent_t tail = nullptr;     // recorded by mark_tail
    hipEvent_t tail_ev = nullptr;  // the event that marks the end of the last call (tail or an arena event)
    hipStream_t tail_stream = nullptr;
    bool tail_valid = false;
    bool tail_pending = false;     // the last call was a step whose arena batch is not recorded yet
    int n_cus = 256;
    // step schedule and its autotuner
    mvf_schedule fixed_sched{4, 0, kRayLanes, 0};
    mvf_schedule last_sched{4, 0, kRayLanes, 0};
    int tune_mode = MVF_AUTOTUNE_OFF;
    std::string tune_path;
    std::map<std::string, std::pair<mvf_schedule, double>> tune_cache;  // shape -> (schedule, ms)
    struct Tuning {
        std::string key;
        std::vector<mvf_schedule> cands;
        int next = 0;                                   // launches issued so far
        std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // per launch
    } tuning;
    // placement bookkeeping: per stream, cell -> volume id (volumes created by placement)
    // per stream: volumes created by placement, keyed by (d_v, cell)
    std::map<int, std::map<std::vector<int>, int>> placed;
    unsigned long long* place_table = nullptr;
    int* place_overflow = nullptr;
    float* place_T = nullptr;
    int32_t* place_boxes = nullptr;  // kMaxPlaceBoxes x (h_t, dims)
    static constexpr int kMaxPlaceBoxes = 64;
    static constexpr int kPlaceTable = 8192;
    double* diff_partials = nullptr;
    int diff_partials_n = 0;
    // brick-layout mirror of the caller's dense volume (differentiable
    // raycast forward), and what it was built from
    struct DiffMirror {
        int vol = -1, grid = -1;
        const void* F = nullptr;
        const void* W = nullptr;
        int dims[3] = {0, 0, 0}, off[3] = {0, 0, 0};
        float o[3] = {0, 0, 0}, s = 0.0f;
        uint64_t generation = 0;
    } diff_mirror;
    // camera tracking: pyramid maps, partials and the device state, plus a
    // pinned copy of the state for the result
    struct TrackScratch {
        uint8_t* dev = nullptr;
        size_t bytes = 0;
        TrackState* host = nullptr;
    } track;
    uint8_t* extract_buf = nullptr;   // surface points: per-brick counts (4 B), offsets (8 B), total (8 B)
    size_t extract_buf_n = 0;         // nbricks it holds
    StepGraph step;
    hipStream_t capture_stream = nullptr;
};

namespace {

mvf_status get_event(mvf_ctx* c, hipEvent_t* ev)
{
    if (!c->event_pool.empty()) {
        *ev = c->event_pool.back();
        c->event_pool.pop_back();
        return MVF_OK;
    }
    // pooled events order device work or time it; none makes device memory
    // visible to the host, so they skip the system-scope fence (a cache
    // writeback per record)
    CHECK_HIP(hipEventCreateWithFlags(ev, hipEventDisableSystemFence));
    return MVF_OK;
}

// Record one event behind the step slots released since the last record;
// each of them waits on it before reuse.  When the last call was such a
// step, the event becomes the tail.
mvf_status arena_flush(mvf_ctx* c)
{
    Arena& A = c->arena;
    if (A.n_open == 0) return MVF_OK;
    const int last = A.open[A.n_open - 1];
    CHECK_HIP(hipEventRecord(A.ev[last], A.open_stream));
    for (int i = 0; i < A.n_open; ++i) {
        A.wait_ev[A.open[i]] = A.ev[last];
        A.pending[A.open[i]] = true;
    }
    A.n_open = 0;
    if (c->tail_pending) {
        c->tail_ev = A.ev[last];
        c->tail_stream = A.open_stream;
        c->tail_valid = true;
        c->tail_pending = false;
    }
    return MVF_OK;
}

// Make `stream` run after everything the previous call enqueued.
mvf_status order_after_previous(mvf_ctx* c, hipStream_t stream)
{
    if (c->tail_valid && c->tail_stream != stream) {
        if (c->tail_pending) CHECK_ST(arena_flush(c));
        CHECK_HIP(hipStreamWaitEvent(stream, c->tail_ev, 0));
    }
    return MVF_OK;
}

mvf_status mark_tail(mvf_ctx* c, hipStream_t stream)
{
    CHECK_HIP(hipEventRecord(c->tail, stream));
    c->tail_ev = c->tail;
    c->tail_stream = stream;
    c->tail_valid = true;
    c->tail_pending = false;
    return MVF_OK;
}


mvf_status arena_acquire(mvf_ctx* c, int* slot, Writer* w)
{
    Arena& A = c->arena;
    int s = A.next;
    A.next = (A.next + 1) % Arena::kSlots;
    for (int i = 0; i < A.n_open; ++i)
        if (A.open[i] == s) {
            CHECK_ST(arena_flush(c));
            break;
        }
    if (A.pending[s]) {
        CHECK_HIP(hipEventSynchronize(A.wait_ev[s]));
        A.pending[s] = false;
    }
    *slot = s;
    w->host = A.host + (size_t)s * Arena::kSlotBytes;
    w->dev = A.dev + (size_t)s * Arena::kSlotBytes;
    w->used = 0;
    w->overflow = false;
    return MVF_OK;
}

mvf_status arena_upload(mvf_ctx* c, const Writer& w, hipStream_t stream)
{
    if (w.overflow) return set_error(MVF_ERR_INVALID_ARG, "launch tables exceed %zu bytes", Arena::kSlotBytes);
    if (w.used) CHECK_HIP(hipMemcpyAsync(w.dev, w.host, w.used, hipMemcpyHostToDevice, stream));
    return MVF_OK;
}

mvf_status arena_release(mvf_ctx* c, int slot, hipStream_t stream)
{
    CHECK_ST(arena_flush(c));
    CHECK_HIP(hipEventRecord(c->arena.ev[slot], stream));
    c->arena.wait_ev[slot] = c->arena.ev[slot];
    c->arena.pending[slot] = true;
    return MVF_OK;
}

// A captured step's slot: released with the next kBatch - 1 step slots of
// the same stream behind one event (arena_flush); the call's tail is that
// event once recorded.
mvf_status arena_release_step(mvf_ctx* c, int slot, hipStream_t stream)
{
    Arena& A = c->arena;
    if (A.n_open && A.open_stream != stream) CHECK_ST(arena_flush(c));
    A.open[A.n_open++] = slot;
    A.open_stream = stream;
    c->tail_stream = stream;
    c->tail_valid = true;
    c->tail_pending = true;
    if (A.n_open == Arena::kBatch) CHECK_ST(arena_flush(c));
    return MVF_OK;
}

Volume* find_volume(mvf_ctx* c, int32_t id)
{
    if (id < 0 || id >= (int32_t)c->vols.size() || !c->vols[id].alive || c->vols[id].internal) return nullptr;
    return &c->vols[id];
}

DevVolume make_dev(mvf_ctx* c, const Volume& v)
{
    const Grid& g = c->grids[v.d.grid_id];
    DevVolume d{};
    d.F = reinterpret_cast<float*>(v.dev);
    d.W = reinterpret_cast<uint16_t*>(v.dev + v.off_W);
    d.C = reinterpret_cast<uint32_t*>(v.dev + v.off_C);
    d.flag = v.dev + v.off_flag;
    d.dist = v.dev + v.off_dist;
    d.colm = reinterpret_cast<uint64_t*>(v.dev + v.off_colm);
    d.fmask = reinterpret_cast<uint64_t*>(v.dev + v.off_fmask);
    d.cmask = reinterpret_cast<uint64_t*>(v.dev + v.off_cmask);
    for (int a = 0; a < 3; ++a) {
        d.dims[a] = v.d.dims[a];
        d.off[a] = v.d.offset[a];
        d.bd[a] = v.bd[a];
        d.o[a] = g.d.origin[a];
    }
    d.id = (int32_t)(&v - c->vols.data());
    d.s = g.d.voxel_size;
    d.inv_s = g.inv_s;
    d.mu = g.mu;
    d.inv_mu = g.inv_mu;
    d.w_max = g.d.w_max;
    d.frame = 0;
    return d;
}

// ---- residency ------------------------------------------------------------

mvf_status release_pool(mvf_ctx* c, uint64_t need_room)
{
    // free pooled slabs (oldest first) until `need_room` more bytes fit
    while (!c->pool.empty() && c->resident_bytes + c->pooled_bytes + need_room > c->budget) {
        Slab s = c->pool.front();
        c->pool.erase(c->pool.begin());
        CHECK_HIP(hipEventSynchronize(s.chunk_done.back()));
        for (hipEvent_t e : s.chunk_done) c->event_pool.push_back(e);
        CHECK_HIP(hipFree(s.ptr));
        c->pooled_bytes -= s.bytes;
    }
    return MVF_OK;
}

mvf_status swap_out(mvf_ctx* c, Volume& v, hipStream_t stream, bool keep_slab_pooled = true)
{
    if (v.state != State::Device) return MVF_OK;
    if (!v.host) {
        hipError_t e = hipHostMalloc((void**)&v.host, v.bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            v.host = nullptr;
            return set_error(MVF_ERR_OOM, "pinned host mirror of %zu bytes: %s", v.bytes, hipGetErrorString(e));
        }
    }
    hipEvent_t used;
    CHECK_ST(get_event(c, &used));
    CHECK_HIP(hipEventRecord(used, stream));
    CHECK_HIP(hipStreamWaitEvent(c->d2h_stream, used, 0));
    c->event_pool.push_back(used);  // recorded; safe to reuse after the wait is enqueued
    // the mirror may still be the source of a swap-in copy
    CHECK_HIP(hipStreamWaitEvent(c->d2h_stream, c->h2d_last, 0));
    std::vector<hipEvent_t> chunks;
    for (size_t off = 0; off < v.bytes; off += kSwapChunk) {
        const size_t n = std::min(kSwapChunk, v.bytes - off);
        CHECK_HIP(hipMemcpyAsync(v.host + off, v.dev + off, n, hipMemcpyDeviceToHost, c->d2h_stream));
        hipEvent_t e;
        CHECK_ST(get_event(c, &e));
        CHECK_HIP(hipEventRecord(e, c->d2h_stream));
        chunks.push_back(e);
    }
    if (!v.host_ready) CHECK_HIP(hipEventCreate(&v.host_ready));
    CHECK_HIP(hipEventRecord(v.host_ready, c->d2h_stream));
    v.host_pending = true;
    c->resident_bytes -= v.bytes;
    if (keep_slab_pooled) {
        c->pool.push_back(Slab{v.dev, v.bytes, std::move(chunks)});
        c->pooled_bytes += v.bytes;
    } else {
        CHECK_HIP(hipEventSynchronize(chunks.back()));
        for (hipEvent_t e : chunks) c->event_pool.push_back(e);
        CHECK_HIP(hipFree(v.dev));
    }
    v.dev = nullptr;
    v.state = State::Host;
    c->stats.bytes_d2h += v.bytes;
    c->stats.swaps_out += 1;
    return MVF_OK;
}

// Obtain a slab of v.bytes for v.  With `pending` null the slab is usable
// on `stream`; otherwise the events of a download still filling from it are
// handed over (chunk k free once event k completes) and the caller orders
// its own copies after them.
mvf_status get_slab(mvf_ctx* c, Volume& v, hipStream_t stream, std::vector<hipEvent_t>* pending)
{
    for (size_t i = 0; i < c->pool.size(); ++i) {
        if (c->pool[i].bytes == v.bytes) {
            Slab s = c->pool[i];
            c->pool.erase(c->pool.begin() + i);
            c->pooled_bytes -= s.bytes;
            if (pending) {
                *pending = std::move(s.chunk_done);
            } else {
                CHECK_HIP(hipStreamWaitEvent(stream, s.chunk_done.back(), 0));
                for (hipEvent_t e : s.chunk_done) c->event_pool.push_back(e);
            }
            v.dev = s.ptr;
            return MVF_OK;
        }
    }
    CHECK_ST(release_pool(c, v.bytes));
    auto alloc = [&]() -> hipError_t {
        if (c->fault_slab_allocs > 0) {
            --c->fault_slab_allocs;
            v.dev = nullptr;
            return hipErrorOutOfMemory;
        }
        return hipMalloc((void**)&v.dev, v.bytes);
    };
    hipError_t e = alloc();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // drop every pooled slab and retry once
        uint64_t saved = c->budget;
        c->budget = 0;
        mvf_status st = release_pool(c, 0);
        c->budget = saved;
        if (st != MVF_OK) return st;
        e = alloc();
        if (e != hipSuccess) {
            (void)hipGetLastError();
            v.dev = nullptr;
            return set_error(MVF_ERR_OOM, "device slab of %zu bytes: %s", v.bytes, hipGetErrorString(e));
        }
    }
    return MVF_OK;
}

// Make every volume of `need` resident (evicting least recently used
// volumes outside `need`).  Fails with MVF_ERR_BUDGET if they cannot all fit.
mvf_status ensure_resident(mvf_ctx* c, const std::vector<int>& need, hipStream_t stream)
{
    uint64_t want = 0;
    for (int id : need) {
        Volume& v = c->vols[id];
        if (v.bytes > c->budget)
            return set_error(MVF_ERR_BUDGET, "volume %d needs %zu bytes, budget is %llu", id, v.bytes,
                             (unsigned long long)c->budget);
        if (v.state != State::Device) want += v.bytes;
    }
    if (c->resident_bytes + want > c->budget) {
        std::vector<char> needed(c->vols.size(), 0);
        for (int id : need) needed[id] = 1;
        while (c->resident_bytes + want > c->budget) {
            int victim = -1;
            for (size_t i = 0; i < c->vols.size(); ++i) {
                Volume& v = c->vols[i];
                if (v.alive && v.state == State::Device && !needed[i] &&
                    (victim < 0 || v.last_use < c->vols[victim].last_use))
                    victim = (int)i;
            }
            if (victim < 0)
                return set_error(MVF_ERR_BUDGET, "needed volumes (%llu bytes) exceed the budget",
                                 (unsigned long long)(c->resident_bytes + want));
            CHECK_ST(swap_out(c, c->vols[victim], stream));
        }
    }
    bool copied = false;
    for (int id : need) {
        Volume& v = c->vols[id];
        v.last_use = ++c->tick;
        if (v.state == State::Device) continue;
        std::vector<hipEvent_t> pending;
        CHECK_ST(get_slab(c, v, stream, v.state == State::Host ? &pending : nullptr));
        c->resident_bytes += v.bytes;
        if (v.state == State::Host) {
            // stream-ordered after earlier work on the caller's stream and
            // after the download that wrote the mirror
            hipEvent_t before;
            CHECK_ST(get_event(c, &before));
            CHECK_HIP(hipEventRecord(before, stream));
            CHECK_HIP(hipStreamWaitEvent(c->h2d_stream, before, 0));
            c->event_pool.push_back(before);
            if (v.host_pending) CHECK_HIP(hipStreamWaitEvent(c->h2d_stream, v.host_ready, 0));
            // chunk k after the slab's previous download of chunk k (same
            // slab size, same chunks)
            size_t k = 0;
            for (size_t off = 0; off < v.bytes; off += kSwapChunk, ++k) {
                if (k < pending.size()) CHECK_HIP(hipStreamWaitEvent(c->h2d_stream, pending[k], 0));
                CHECK_HIP(hipMemcpyAsync(v.dev + off, v.host + off, std::min(kSwapChunk, v.bytes - off),
                                         hipMemcpyHostToDevice, c->h2d_stream));
            }
            for (hipEvent_t e : pending) c->event_pool.push_back(e);
            c->stats.bytes_h2d += v.bytes;
            c->stats.swaps_in += 1;
            copied = true;
        } else {
            CHECK_LAUNCH(launch_volume_init(make_dev(c, v), stream));
        }
        v.state = State::Device;
    }
    if (copied) {
        CHECK_HIP(hipEventRecord(c->h2d_last, c->h2d_stream));
        CHECK_HIP(hipStreamWaitEvent(stream, c->h2d_last, 0));
    }
    return MVF_OK;
}

// Split `ids` into consecutive groups that each fit in the budget.
// Volumes already resident go first so the first wave copies least.
std::vector<std::vector<int>> plan_waves(mvf_ctx* c, std::vector<int> ids)
{
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
        return (c->vols[a].state == State::Device) > (c->vols[b].state == State::Device);
    });
    uint64_t total = 0;
    for (int id : ids) total += c->vols[id].bytes;
    std::vector<std::vector<int>> waves;
    if (total <= c->budget) {
        waves.push_back(ids);
        return waves;
    }
    std::vector<int> cur;
    uint64_t cur_bytes = 0;
    for (int id : ids) {
        const uint64_t b = c->vols[id].bytes;
        if (!cur.empty() && cur_bytes + b > c->budget) {
            waves.push_back(cur);
            cur.clear();
            cur_bytes = 0;
        }
        cur.push_back(id);
        cur_bytes += b;
    }
    if (!cur.empty()) waves.push_back(cur);
    return waves;
}

// ---- geometry helpers -------------------------------------------------------

bool finite_pose(const float* T)
{
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(T[i])) return false;
    return true;
}

bool valid_K(const mvf_intrinsics* K)
{
    return K && std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) && std::isfinite(K->cy) &&
           K->fx != 0.0f && K->fy != 0.0f;
}

// Conservative test: can the view frustum (pixels [0,W)x[0,H), in front of
// the camera) meet the volume's voxel box grown by one voxel?
bool volume_in_view(mvf_ctx* c, const Volume& v, const float* T, const mvf_intrinsics& K, int W, int H)
{
    const Grid& g = c->grids[v.d.grid_id];
    const double s = g.d.voxel_size;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.d.origin[a] + s * (v.d.offset[a] + 0.5) - s;
        hi[a] = g.d.origin[a] + s * (v.d.offset[a] + v.d.dims[a] - 0.5) + s;
    }
    double p[8][3];
    for (int k = 0; k < 8; ++k) {
        double x[3] = { (k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2] };
        double d[3] = { x[0] - T[3], x[1] - T[7], x[2] - T[11] };
        for (int cc = 0; cc < 3; ++cc) p[k][cc] = T[cc] * d[0] + T[4 + cc] * d[1] + T[8 + cc] * d[2];
    }
    const double E = 1e-3;
    auto all_out = [&](double ax, double ay, double az, double a0) {
        for (int k = 0; k < 8; ++k)
            if (ax * p[k][0] + ay * p[k][1] + az * p[k][2] + a0 >= 0.0) return false;
        return true;
    };
    if (all_out(0, 0, 1, 2 * s)) return false;
    if (all_out(K.fx, 0, K.cx + 1.5, std::fabs(K.fx) * E)) return false;
    if (all_out(-K.fx, 0, W + 0.5 - K.cx, std::fabs(K.fx) * E)) return false;
    if (all_out(0, K.fy, K.cy + 1.5, std::fabs(K.fy) * E)) return false;
    if (all_out(0, -K.fy, H + 0.5 - K.cy, std::fabs(K.fy) * E)) return false;
    return true;
}

double box_distance(mvf_ctx* c, const Volume& v, const float* T)
{
    const Grid& g = c->grids[v.d.grid_id];
    const double s = g.d.voxel_size;
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double lo = g.d.origin[a] + s * (v.d.offset[a] + 0.5);
        const double hi = g.d.origin[a] + s * (v.d.offset[a] + v.d.dims[a] - 0.5);
        const double t = T[4 * a + 3];
        const double q = t < lo ? lo - t : (t > hi ? t - hi : 0.0);
        d2 += q * q;
    }
    return std::sqrt(d2);
}

// Running best (t*, volume id) of a raycast split into waves, for npix
// output pixels.
mvf_status get_best_buffers(Scratch* s, int npix)
{
    if (npix <= s->best_cap && s->best_t) return MVF_OK;
    if (s->best_t) { CHECK_HIP(hipFree(s->best_t)); s->best_t = nullptr; }
    if (s->best_id) { CHECK_HIP(hipFree(s->best_id)); s->best_id = nullptr; }
    s->best_cap = 0;
    CHECK_HIP(hipMalloc((void**)&s->best_t, (size_t)npix * sizeof(float)));
    CHECK_HIP(hipMalloc((void**)&s->best_id, (size_t)npix * sizeof(int32_t)));
    s->best_cap = npix;
    return MVF_OK;
}

mvf_status get_scratch(mvf_ctx* c, int sid, int w, int h, bool need_best, Scratch** out)
{
    Scratch& s = c->scratch[sid];
    const int parts = ((w + 31) / 32) * ((h + 7) / 8);
    if (1 + parts > s.rmax_cap) {
        if (s.rmax) { CHECK_HIP(hipFree(s.rmax)); s.rmax = nullptr; }
        CHECK_HIP(hipMalloc((void**)&s.rmax, (size_t)(1 + parts) * sizeof(float)));
        s.rmax_cap = 1 + parts;
    }
    const int ntiles = ((w + 7) / 8) * ((h + 7) / 8);
    if (ntiles > s.tmax_cap) {
        if (s.tmax) { CHECK_HIP(hipFree(s.tmax)); s.tmax = nullptr; }
        // maxima, then minima, of the range over each 8x8 tile
        CHECK_HIP(hipMalloc((void**)&s.tmax, 2 * (size_t)ntiles * sizeof(float)));
        s.tmax_cap = ntiles;
    }
    if (w * h > s.w * s.h || !s.range) {
        if (s.range) { CHECK_HIP(hipFree(s.range)); s.range = nullptr; }
        if (s.color) { CHECK_HIP(hipFree(s.color)); s.color = nullptr; }
        const size_t n = (size_t)std::max(w * h, s.w * s.h);
        CHECK_HIP(hipMalloc((void**)&s.range, (n + 64) * sizeof(float)));  // + the zero range behind the image
        CHECK_HIP(hipMalloc((void**)&s.color, n * sizeof(uint32_t)));
        s.w = w;
        s.h = h;
    }
    if (need_best) CHECK_ST(get_best_buffers(&s, w * h));
    *out = &s;
    return MVF_OK;
}

// Raycast cost per tile (padded to whole groups) and launch order per tile
// group, for n tiles.  The costs start at zero; any content still gives a
// valid order (a permutation), the order only decides which tiles start
// first.
mvf_status alloc_tile_buffers(int n, uint32_t** cost, int32_t** order)
{
    const size_t nc = (size_t)ray_groups(n) * kRayGroup;  // whole groups (the padding stays 0)
    CHECK_HIP(hipMalloc((void**)cost, nc * sizeof(uint32_t)));
    CHECK_HIP(hipMalloc((void**)order, (size_t)ray_groups(n) * sizeof(int32_t)));
    CHECK_HIP(hipMemset(*cost, 0, nc * sizeof(uint32_t)));
    return MVF_OK;
}

mvf_status get_tile_buffers(Scratch* s, int n)
{
    if (n <= s->tiles_cap) return MVF_OK;
    if (s->tile_cost) { CHECK_HIP(hipFree(s->tile_cost)); s->tile_cost = nullptr; }
    if (s->tile_order) { CHECK_HIP(hipFree(s->tile_order)); s->tile_order = nullptr; }
    s->tiles_cap = 0;
    CHECK_ST(alloc_tile_buffers(n, &s->tile_cost, &s->tile_order));
    s->tiles_cap = n;
    return MVF_OK;
}

// Range-bound cells for a w x h raycast output (written by every merge
// before the raycast reads them).
mvf_status get_bound_buffers(Scratch* s, int w, int h)
{
    const int n = ((w + kBoundCell - 1) / kBoundCell) * ((h + kBoundCell - 1) / kBoundCell);
    if (n <= s->rb_cap) return MVF_OK;
    if (s->rb_lo) { CHECK_HIP(hipFree(s->rb_lo)); s->rb_lo = nullptr; }
    if (s->rb_hi) { CHECK_HIP(hipFree(s->rb_hi)); s->rb_hi = nullptr; }
    s->rb_cap = 0;
    CHECK_HIP(hipMalloc((void**)&s->rb_lo, (size_t)n * sizeof(float)));
    CHECK_HIP(hipMalloc((void**)&s->rb_hi, (size_t)n * sizeof(float)));
    s->rb_cap = n;
    return MVF_OK;
}

// Footprint list for `bricks` (64-aligned per volume) and zeroed counts for
// `vols` volume slots.
mvf_status get_footprint_buffers(RayBoundEntry** entries, int* entries_cap, uint32_t** counts, int* counts_cap,
                                 int bricks, int vols)
{
    if (bricks > *entries_cap) {
        if (*entries) { CHECK_HIP(hipFree(*entries)); *entries = nullptr; }
        *entries_cap = 0;
        CHECK_HIP(hipMalloc((void**)entries, (size_t)bricks * sizeof(RayBoundEntry)));
        *entries_cap = bricks;
    }
    if (counts_cap && vols > *counts_cap) {
        if (*counts) { CHECK_HIP(hipFree(*counts)); *counts = nullptr; }
        *counts_cap = 0;
        CHECK_HIP(hipMalloc((void**)counts, (size_t)2 * vols * sizeof(uint32_t)));
        CHECK_HIP(hipMemset(*counts, 0, (size_t)2 * vols * sizeof(uint32_t)));
        *counts_cap = vols;
    }
    return MVF_OK;
}

void set_bounds(DevFrame* f, const Scratch* s, int w, int h)
{
    f->rb_lo = s->rb_lo;
    f->rb_hi = s->rb_hi;
    f->cells_x = (w + kBoundCell - 1) / kBoundCell;
    f->cells_y = (h + kBoundCell - 1) / kBoundCell;
}

mvf_status check_frame(const mvf_frame* f)
{
    if (!f || !f->depth) return set_error(MVF_ERR_INVALID_ARG, "frame or frame->depth is NULL");
    if (f->width <= 0 || f->height <= 0 || f->width > 16384 || f->height > 16384)
        return set_error(MVF_ERR_INVALID_ARG, "frame size %dx%d out of range", f->width, f->height);
    if (f->depth_pitch != 0 && f->depth_pitch < f->width)
        return set_error(MVF_ERR_INVALID_ARG, "depth_pitch %d < width %d", f->depth_pitch, f->width);
    if (f->rgb && f->rgb_pitch != 0 && f->rgb_pitch < 3 * f->width)
        return set_error(MVF_ERR_INVALID_ARG, "rgb_pitch %d < 3*width", f->rgb_pitch);
    return MVF_OK;
}

mvf_status timing_begin(mvf_ctx* c, hipStream_t stream, hipEvent_t* a)
{
    *a = nullptr;
    if (!(c->cfg.flags & MVF_FLAG_TIMING)) return MVF_OK;
    CHECK_ST(get_event(c, a));
    CHECK_HIP(hipEventRecord(*a, stream));
    return MVF_OK;
}

// Event pair for a kernel launch that records them itself (timing only).
mvf_status timing_pair(mvf_ctx* c, hipEvent_t* a, hipEvent_t* b)
{
    *a = *b = nullptr;
    if (!(c->cfg.flags & MVF_FLAG_TIMING)) return MVF_OK;
    CHECK_ST(get_event(c, a));
    CHECK_ST(get_event(c, b));
    return MVF_OK;
}

mvf_status timing_push(mvf_ctx* c, hipEvent_t a, hipEvent_t b, int kind)
{
    if (a) c->timed.push_back(TimedPair{a, b, kind});
    return MVF_OK;
}

mvf_status timing_end(mvf_ctx* c, hipStream_t stream, hipEvent_t a, int kind)
{
    if (!a) return MVF_OK;
    hipEvent_t b;
    CHECK_ST(get_event(c, &b));
    CHECK_HIP(hipEventRecord(b, stream));
    c->timed.push_back(TimedPair{a, b, kind});
    return MVF_OK;
}

mvf_status drain_timing(mvf_ctx* c)
{
    for (auto& t : c->timed) {
        CHECK_HIP(hipEventSynchronize(t.b));
        float ms = 0.0f;
        CHECK_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        if (t.kind == 0) c->stats.integrate_ms += ms;
        else if (t.kind == 1) c->stats.raycast_ms += ms;
        else c->stats.step_ms += ms;
        c->event_pool.push_back(t.a);
        c->event_pool.push_back(t.b);
    }
    c->timed.clear();
    return MVF_OK;
}

// bricks per integration item along z (the visit masks hold one byte per brick)
constexpr int kZChunk = 4;
static_assert(kZChunk <= kVisitPerItem, "visit mask too small for the z chunk");
int zchunk_for(const Volume&) { return kZChunk; }

void fill_frame(DevFrame* f, const Scratch* s, int w, int h, const float* T, const mvf_intrinsics& K)
{
    memset(f, 0, sizeof(*f));
    if (s) {
        f->range = s->range;
        f->color = s->color;
        f->rmax = s->rmax;
        f->rmax_parts = ((w + 31) / 32) * ((h + 7) / 8);
        f->tmax = s->tmax;
        f->tiles_x = (w + 7) / 8;
        f->tiles_y = (h + 7) / 8;
    }
    f->width = w;
    f->height = h;
    f->fx = K.fx;
    f->fy = K.fy;
    f->cx = K.cx;
    f->cy = K.cy;
    memcpy(f->T, T, sizeof(float) * 12);
}

RayParams ray_params(mvf_ctx* c, const Grid& g)
{
    RayParams rp;
    rp.delta = c->cfg.ray_step * g.d.voxel_size;
    rp.kmax = (int32_t)std::floor(c->cfg.t_far / rp.delta);
    return rp;
}

// Integration of one frame into the given volumes, one launch per volume
// (the paper's per-volume loop), in budget-sized waves.
mvf_status integrate_plain(mvf_ctx* c, int sid, const mvf_frame* f, const float* T, const mvf_intrinsics& K,
                           const std::vector<int>& ids, hipStream_t stream)
{
    Scratch* sc;
    CHECK_ST(get_scratch(c, sid, f->width, f->height, false, &sc));
    int slot;
    Writer w;
    CHECK_ST(arena_acquire(c, &slot, &w));
    PrepItem* dprep;
    PrepItem* prep = w.alloc<PrepItem>(1, &dprep);
    DevFrame* dframe;
    DevFrame* frame = w.alloc<DevFrame>(1, &dframe);
    if (!prep || !frame) return set_error(MVF_ERR_INVALID_ARG, "arena overflow");
    memset(prep, 0, sizeof(*prep));
    prep->depth = f->depth;
    prep->rgb = f->rgb;
    prep->depth_pitch = f->depth_pitch ? f->depth_pitch : f->width;
    prep->rgb_pitch = f->rgb_pitch ? f->rgb_pitch : 3 * f->width;
    prep->width = f->width;
    prep->height = f->height;
    prep->fx = K.fx; prep->fy = K.fy; prep->cx = K.cx; prep->cy = K.cy;
    prep->range = sc->range;
    prep->color = sc->color;
    prep->rmax = sc->rmax;
    prep->tmax = sc->tmax;
    fill_frame(frame, sc, f->width, f->height, T, K);
    if (!f->rgb) frame->color = nullptr;
    // per-volume tables are filled after residency is known (slab pointers)
    std::vector<std::vector<int>> waves = plan_waves(c, ids);
    // first upload: prep + frame; volume tables go into fresh slots per wave
    CHECK_ST(arena_upload(c, w, stream));
    CHECK_LAUNCH(launch_frame_prep(dprep, 1, f->width, f->height, stream));
    CHECK_ST(arena_release(c, slot, stream));
    int zmax = 0;
    for (int id : ids) zmax = std::max(zmax, kBrick * c->vols[id].bd[2]);
    if (zmax > sc->ztab_cap) {
        // stream-ordered: earlier launches reading the old table have been
        // queued on this stream, so free only after they finish
        if (sc->ztab) {
            CHECK_HIP(hipStreamSynchronize(stream));
            CHECK_HIP(hipFree(sc->ztab));
            sc->ztab = nullptr;
        }
        CHECK_HIP(hipMalloc((void**)&sc->ztab, (size_t)zmax * 3 * sizeof(float)));
        sc->ztab_cap = zmax;
    }
    int max_items = 0;
    for (int id : ids) {
        const Volume& v = c->vols[id];
        max_items = std::max(max_items, v.bd[0] * v.bd[1] * ((v.bd[2] + zchunk_for(v) - 1) / zchunk_for(v)));
    }
    if (max_items > sc->visit_cap) {
        if (sc->visit) {
            CHECK_HIP(hipStreamSynchronize(stream));
            CHECK_HIP(hipFree(sc->visit));
            CHECK_HIP(hipFree(sc->list));
            sc->visit = nullptr;
            sc->list = nullptr;
        }
        CHECK_HIP(hipMalloc((void**)&sc->visit, (size_t)max_items * kVisitPerItem));
        // the visited-brick list, then the deep-brick list (kVisitPerItem per item each)
        CHECK_HIP(hipMalloc((void**)&sc->list, (size_t)max_items * (2 * kVisitPerItem) * sizeof(int32_t)));
        sc->visit_cap = max_items;
    }
    if (!sc->list_count) {
        CHECK_HIP(hipMalloc((void**)&sc->list_count, 2 * sizeof(unsigned long long)));
        CHECK_HIP(hipMemset(sc->list_count, 0, 2 * sizeof(unsigned long long)));
    }
    bool order_pending = sc->tile_cost && sc->last_tiles > 0;  // once per call
    for (auto& wave : waves) {
        CHECK_ST(ensure_resident(c, wave, stream));
        int slot2;
        Writer w2;
        CHECK_ST(arena_acquire(c, &slot2, &w2));
        DevFrame* dfr;
        DevFrame* fr = w2.alloc<DevFrame>(1, &dfr);
        *fr = *frame;
        struct Per { LaunchHeader* dh; DevVolume* dv; int32_t* dib; int32_t* dbb; int items; int bricks; };
        std::vector<Per> per;
        for (int id : wave) {
            Volume& v = c->vols[id];
            Per p;
            LaunchHeader* h = w2.alloc<LaunchHeader>(1, &p.dh);
            DevVolume* dv = w2.alloc<DevVolume>(1, &p.dv);
            int32_t* ib = w2.alloc<int32_t>(2, &p.dib);
            int32_t* bb = w2.alloc<int32_t>(2, &p.dbb);
            if (!h || !dv || !ib || !bb) return set_error(MVF_ERR_INVALID_ARG, "arena overflow");
            *dv = make_dev(c, v);
            dv->frame = 0;
            dv->zt_base = 0;
            const int zc = zchunk_for(v);
            p.items = v.bd[0] * v.bd[1] * ((v.bd[2] + zc - 1) / zc);
            memset(h, 0, sizeof(*h));
            h->nvol = 1;
            h->total_items = p.items;
            h->zchunk = zc;
            h->nstreams = 1;
            p.bricks = (int)v.nbricks;
            h->total_bricks = (int)align_up((size_t)p.bricks, 64);
            h->total_z = kBrick * v.bd[2];
            h->list_parity = sc->list_parity;
            sc->list_parity ^= 1;
            ib[0] = 0;
            ib[1] = p.items;
            bb[0] = 0;
            bb[1] = h->total_bricks;
            per.push_back(p);
        }
        CHECK_ST(arena_upload(c, w2, stream));
        for (size_t pi = 0; pi < per.size(); ++pi) {
            const Per& p = per[pi];
            // the first launch's block 0 orders the tiles of the stream's
            // next raycast from the last one's durations (the raycast then
            // skips its own ordering launch)
            const bool order = pi == 0 && order_pending;
            order_pending = false;
            IntegrateLaunch L{p.dh, p.dv, dfr, p.dib, c->counters, sc->ztab, sc->visit,
                              order ? sc->tile_cost : nullptr, order ? sc->tile_order : nullptr,
                              order ? sc->last_tiles : 0, sc->list, sc->list_count,
                              sc->list + (size_t)sc->visit_cap * kVisitPerItem};
            if (order) sc->order_ready_tiles = sc->last_tiles;
            CHECK_LAUNCH(launch_ztable(L, p.items * kZChunk, stream));
            // with timing, the kernel's dispatch records the event pair
            hipEvent_t t0, t1;
            CHECK_ST(timing_pair(c, &t0, &t1));
            CHECK_LAUNCH(launch_integrate(L, (p.items + 3) / 4 + (order ? 1 : 0), stream, t0, t1));
            CHECK_ST(timing_push(c, t0, t1, 0));
            CHECK_LAUNCH(launch_brick_distance(p.dh, p.dv, p.dbb, std::min(1024, (p.bricks + 255) / 256), stream));
            c->stats.integrate_launches += 1;
        }
        CHECK_ST(arena_release(c, slot2, stream));
    }
    return MVF_OK;
}

mvf_status raycast_plain(mvf_ctx* c, int sid, const float* T, const mvf_intrinsics& K, const mvf_raycast_out* out,
                         const std::vector<int>& ids_in, hipStream_t stream, int32_t* record = nullptr)
{
    std::vector<int> ids = ids_in;
    // nearest first (ties by id) -- only affects speed, not results
    std::vector<double> dist(c->vols.size(), 0.0);
    for (int id : ids) dist[id] = box_distance(c, c->vols[id], T);
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return dist[a] < dist[b] || (dist[a] == dist[b] && a < b); });
    std::vector<std::vector<int>> waves = plan_waves(c, ids);
    if (waves.empty()) waves.push_back({});
    const bool multi = waves.size() > 1;
    Scratch* sc = nullptr;
    CHECK_ST(get_scratch(c, sid, out->width, out->height, multi, &sc));
    RayParams rp{};
    if (!c->grids.empty()) rp = ray_params(c, c->grids[ids.empty() ? 0 : c->vols[ids[0]].d.grid_id]);
    const int tw = ray_tile_w(kRayLanes), th = ray_tile_h(kRayLanes);  // one wavefront per block
    const int tiles = ((out->width + tw - 1) / tw) * ((out->height + th - 1) / th);
    CHECK_ST(get_tile_buffers(sc, tiles));
    CHECK_ST(get_bound_buffers(sc, out->width, out->height));
    // an order the integration computed holds for this many tiles only
    const bool ordered = sc->order_ready_tiles == tiles && sc->last_tiles == tiles;
    sc->order_ready_tiles = 0;
    sc->last_tiles = tiles;
    for (size_t wi = 0; wi < waves.size(); ++wi) {
        auto& wave = waves[wi];
        CHECK_ST(ensure_resident(c, wave, stream));
        // keep nearest-first order inside the wave
        int slot;
        Writer w;
        CHECK_ST(arena_acquire(c, &slot, &w));
        LaunchHeader* dh;
        LaunchHeader* h = w.alloc<LaunchHeader>(1, &dh);
        DevFrame* dfr;
        DevFrame* fr = w.alloc<DevFrame>(1, &dfr);
        DevVolume* dvols;
        DevVolume* vt = w.alloc<DevVolume>(wave.size(), &dvols);
        int32_t* dlists;
        int32_t* lists = w.alloc<int32_t>(wave.size(), &dlists);
        int32_t* dlb;
        int32_t* lb = w.alloc<int32_t>(2, &dlb);
        int32_t* dtb;
        int32_t* tb = w.alloc<int32_t>(2, &dtb);
        if (!h || !fr || !vt || !lists || !lb || !tb) return set_error(MVF_ERR_INVALID_ARG, "arena overflow");
        for (size_t j = 0; j < wave.size(); ++j) {
            vt[j] = make_dev(c, c->vols[wave[j]]);
            lists[j] = (int32_t)j;
        }
        fill_frame(fr, nullptr, out->width, out->height, T, K);
        fr->depth = out->depth;
        fr->vertex = out->vertex;
        fr->normal = out->normal;
        fr->hit = out->hit;
        fr->record = record;
        fr->out_w = out->width;
        fr->out_h = out->height;
        if (multi) {
            fr->best_t = sc->best_t;
            fr->best_id = sc->best_id;
        }
        set_bounds(fr, sc, out->width, out->height);
        // footprint regions: the wave's bricks, 64-aligned per volume
        int32_t* dbb;
        int32_t* bb = w.alloc<int32_t>(wave.size() + 1, &dbb);
        if (!bb) return set_error(MVF_ERR_INVALID_ARG, "arena overflow");
        int nbr = 0;
        for (size_t j = 0; j < wave.size(); ++j) {
            bb[j] = nbr;
            nbr += (int)align_up(c->vols[wave[j]].nbricks, 64);
        }
        bb[wave.size()] = nbr;
        CHECK_ST(get_footprint_buffers(&sc->rb_entries, &sc->rb_entries_cap, &sc->rb_counts, &sc->rb_counts_cap,
                                       std::max(nbr, 64), std::max<int>((int)wave.size(), 16)));
        lb[0] = 0;
        lb[1] = (int32_t)wave.size();
        tb[0] = 0;
        tb[1] = tiles;
        memset(h, 0, sizeof(*h));
        h->nvol = (int32_t)wave.size();
        h->nstreams = 1;
        h->total_tiles = tiles;
        h->first_wave = wi == 0 ? 1 : 0;
        h->rp = rp;
        h->total_bricks = nbr;
        h->rb_parity = sc->rb_parity;
        sc->rb_parity ^= 1;
        CHECK_ST(arena_upload(c, w, stream));
        // slowest tiles of the stream's last raycast first
        RaycastLaunch L{dh, dvols, dfr, dlists, dlb, dtb, tw, th, kRayLanes, sc->tile_cost, sc->tile_order};
        hipEvent_t t0, t1;
        CHECK_ST(timing_pair(c, &t0, &t1));
        const RayBounds RB{sc->rb_entries, sc->rb_counts, sc->rb_counts_cap};
        CHECK_LAUNCH(launch_ray_bounds_collect(dh, dvols, dbb, dfr, RB, std::min(1024, (nbr + 255) / 256), stream));
        CHECK_LAUNCH(launch_ray_bounds_merge(dh, dfr, dlists, dlb, dbb, RB, 1, fr->cells_x, fr->cells_y, stream));
        if (!(ordered && wi == 0)) CHECK_LAUNCH(launch_tile_order(sc->tile_cost, sc->tile_order, tiles, stream));
        CHECK_LAUNCH(launch_raycast(L, ray_blocks(tiles), stream, t0, t1));
        CHECK_ST(timing_push(c, t0, t1, 1));
        CHECK_ST(arena_release(c, slot, stream));
        c->stats.raycast_launches += 1;
    }
    c->stats.pixels_raycast += (uint64_t)out->width * out->height;
    return MVF_OK;
}

// Exact recompute of a resident volume's brick summaries (flags, sub-block
// masks, column words, distances and cell masks) after its planes were
// overwritten, on `stream`.
mvf_status recompute_summaries(mvf_ctx* c, const Volume& v, hipStream_t stream)
{
    const DevVolume dv = make_dev(c, v);
    CHECK_LAUNCH(launch_brick_summary(dv, stream));
    int slot;
    Writer w;
    CHECK_ST(arena_acquire(c, &slot, &w));
    LaunchHeader* dh;
    LaunchHeader* h = w.alloc<LaunchHeader>(1, &dh);
    DevVolume* dvv;
    DevVolume* vt = w.alloc<DevVolume>(1, &dvv);
    int32_t* dbb;
    int32_t* bb = w.alloc<int32_t>(2, &dbb);
    if (!h || !vt || !bb) return set_error(MVF_ERR_INVALID_ARG, "arena overflow");
    memset(h, 0, sizeof(*h));
    h->nvol = 1;
    h->total_bricks = (int)align_up(v.nbricks, 64);
    *vt = dv;
    bb[0] = 0;
    bb[1] = h->total_bricks;
    CHECK_ST(arena_upload(c, w, stream));
    CHECK_LAUNCH(launch_brick_distance(dh, dvv, dbb, std::min<int>(1024, ((int)v.nbricks + 255) / 256), stream));
    return arena_release(c, slot, stream);
}

std::vector<int> stream_volumes(mvf_ctx* c, int sid, const float* T, const mvf_intrinsics& K, int w, int h)
{
    std::vector<int> ids;
    for (size_t i = 0; i < c->vols.size(); ++i) {
        const Volume& v = c->vols[i];
        if (v.alive && v.active && v.d.stream_id == sid && volume_in_view(c, v, T, K, w, h)) ids.push_back((int)i);
    }
    return ids;
}

mvf_status destroy_step_graph(mvf_ctx* c)
{
    StepGraph& g = c->step;
    if (g.exec) { CHECK_HIP(hipGraphExecDestroy(g.exec)); g.exec = nullptr; }
    if (g.graph) { CHECK_HIP(hipGraphDestroy(g.graph)); g.graph = nullptr; }
    g.copy_node = nullptr;
    if (g.dev) { CHECK_HIP(hipFree(g.dev)); g.dev = nullptr; }
    if (g.ztab) { CHECK_HIP(hipFree(g.ztab)); g.ztab = nullptr; }
    if (g.visit) { CHECK_HIP(hipFree(g.visit)); g.visit = nullptr; }
    if (g.list) { CHECK_HIP(hipFree(g.list)); g.list = nullptr; }
    if (g.list_count) { CHECK_HIP(hipFree(g.list_count)); g.list_count = nullptr; }
    g.visit_cap = 0;
    g.list_parity = 0;
    if (g.rb_entries) { CHECK_HIP(hipFree(g.rb_entries)); g.rb_entries = nullptr; }
    if (g.rb_counts) { CHECK_HIP(hipFree(g.rb_counts)); g.rb_counts = nullptr; }
    g.rb_entries_cap = 0;
    if (g.tile_cost) { CHECK_HIP(hipFree(g.tile_cost)); g.tile_cost = nullptr; }
    if (g.tile_order) { CHECK_HIP(hipFree(g.tile_order)); g.tile_order = nullptr; }
    g.ztab_cap = 0;
    g.valid = false;
    return MVF_OK;
}

// ---- step schedules and their autotuner -------------------------------------

// runs per block of one schedule; the first (which pays the graph capture and
// starts the raycast tile order afresh) is not counted, and a block scores
// the mean of the others without their highest and lowest.  The blocks alternate
// between the reference schedule (the first candidate, the default) and the
// other candidates in turn: ref, c1, ref, c2, ..., ref.  A candidate is scored
// by its score over the mean of the two reference scores around it, so that
// the frames' cost, which drifts as the map fills, cancels locally.
constexpr int kTuneReps = 8;

int tune_blocks(int ncand) { return 2 * ncand - 1; }

// candidate run by block b
int tune_block_cand(int b) { return (b & 1) ? (b + 1) / 2 : 0; }

bool valid_schedule(const mvf_schedule& s)
{
    return (s.zchunk == 1 || s.zchunk == 2 || s.zchunk == 4 || s.zchunk == 8) && (s.persistent == 0 || s.persistent == 1) &&
           (s.ray_lanes == 2 || s.ray_lanes == 4 || s.ray_lanes == 8);
}

bool same_schedule(const mvf_schedule& a, const mvf_schedule& b)
{
    return a.zchunk == b.zchunk && a.persistent == b.persistent && a.ray_lanes == b.ray_lanes;
}

// Candidates tried for a new shape: the default first (the reference), then
// every other z chunk and integration grid at 4 lanes per ray, then the other
// lane counts at the default.
std::vector<mvf_schedule> tune_candidates()
{
    std::vector<mvf_schedule> c{mvf_schedule{kZChunk, 0, kRayLanes, 0}};
    for (int z : {2, 4, 8})
        for (int p : {0, 1})
            if (!(z == kZChunk && p == 0)) c.push_back(mvf_schedule{z, p, kRayLanes, 0});
    for (int l : {2, 8}) c.push_back(mvf_schedule{kZChunk, 0, l, 0});
    return c;
}

// Shape of a step: stream count, output sizes, and the brick dimensions of
// its volumes (as a sorted multiset).
std::string step_key(mvf_ctx* c, int n, const mvf_raycast_out* outs, const std::vector<int>& all)
{
    std::string k = "n" + std::to_string(n) + ":";
    for (int i = 0; i < n; ++i) k += std::to_string(outs[i].width) + "x" + std::to_string(outs[i].height) + ",";
    std::map<std::string, int> dims;
    for (int id : all) {
        const Volume& v = c->vols[id];
        dims[std::to_string(v.bd[0]) + "x" + std::to_string(v.bd[1]) + "x" + std::to_string(v.bd[2])] += 1;
    }
    k += "|";
    for (auto& d : dims) k += d.first + "*" + std::to_string(d.second) + ",";
    return k;
}

mvf_status read_tune_cache(mvf_ctx* c, const std::string& path)
{
    FILE* f = fopen(path.c_str(), "r");
    if (!f) return MVF_OK;   // no cache yet
    char line[4096];
    int ln = 0;
    mvf_status st = MVF_OK;
    while (fgets(line, sizeof line, f)) {
        ++ln;
        std::string L(line);
        if (L.find_first_not_of(" \t\r\n") == std::string::npos) continue;
        auto field = [&](const char* name, std::string* sval, double* dval) {
            const std::string pat = std::string("\"") + name + "\":";
            size_t p = L.find(pat);
            if (p == std::string::npos) return false;
            p += pat.size();
            while (p < L.size() && L[p] == ' ') ++p;
            if (sval) {
                if (p >= L.size() || L[p] != '"') return false;
                const size_t e = L.find('"', p + 1);
                if (e == std::string::npos) return false;
                *sval = L.substr(p + 1, e - p - 1);
                return true;
            }
            char* end = nullptr;
            *dval = strtod(L.c_str() + p, &end);
            return end != L.c_str() + p;
        };
        std::string key;
        double z, pe, la, ms = 0.0;
        if (!field("key", &key, nullptr) || !field("zchunk", nullptr, &z) || !field("persistent", nullptr, &pe) ||
            !field("ray_lanes", nullptr, &la)) {
            st = set_error(MVF_ERR_INVALID_ARG, "autotune cache %s line %d does not parse", path.c_str(), ln);
            break;
        }
        field("ms", nullptr, &ms);
        const mvf_schedule sc{(int32_t)z, (int32_t)pe, (int32_t)la, 0};
        if (!valid_schedule(sc)) {
            st = set_error(MVF_ERR_INVALID_ARG, "autotune cache %s line %d: schedule out of range", path.c_str(), ln);
            break;
        }
        c->tune_cache[key] = std::make_pair(sc, ms);
    }
    fclose(f);
    return st;
}

void append_tune_cache(mvf_ctx* c, const std::string& key, const mvf_schedule& sc, double ms)
{
    if (c->tune_path.empty()) return;
    FILE* f = fopen(c->tune_path.c_str(), "a");
    if (!f) return;   // the cache is an optimisation: an unwritable path keeps the result in memory only
    fprintf(f, "{\"key\": \"%s\", \"zchunk\": %d, \"persistent\": %d, \"ray_lanes\": %d, \"ms\": %.5f}\n",
            key.c_str(), sc.zchunk, sc.persistent, sc.ray_lanes, ms);
    fclose(f);
}

// Schedule for a step of shape `key`; *tuning set when this launch is a
// timed candidate run.
mvf_schedule pick_schedule(mvf_ctx* c, const std::string& key, bool* tuning)
{
    *tuning = false;
    if (c->tune_mode == MVF_AUTOTUNE_OFF) return c->fixed_sched;
    auto it = c->tune_cache.find(key);
    if (it != c->tune_cache.end()) return it->second.first;
    if (c->tune_mode == MVF_AUTOTUNE_CACHED) return mvf_schedule{4, 0, kRayLanes, 0};
    mvf_ctx::Tuning& T = c->tuning;
    if (T.key != key) {
        for (auto& e : T.ev) {
            c->event_pool.push_back(e.first);
            c->event_pool.push_back(e.second);
        }
        T = mvf_ctx::Tuning{};
        T.key = key;
        T.cands = tune_candidates();
    }
    *tuning = true;
    const int b = (T.next / kTuneReps) % tune_blocks((int)T.cands.size());
    return T.cands[(size_t)tune_block_cand(b)];
}

// After the last timed launch of a shape: the fastest candidate by median
// becomes the shape's schedule.
mvf_status finish_tuning(mvf_ctx* c)
{
    mvf_ctx::Tuning& T = c->tuning;
    const int nc = (int)T.cands.size(), nb = tune_blocks(nc);
    if (T.next < nb * kTuneReps) return MVF_OK;
    CHECK_HIP(hipEventSynchronize(T.ev.back().second));
    std::vector<double> med(nb);
    for (int b = 0; b < nb; ++b) {
        std::vector<float> ms;
        for (int r = 1; r < kTuneReps; ++r) {
            const auto& e = T.ev[(size_t)(b * kTuneReps + r)];
            float t = 0.0f;
            CHECK_HIP(hipEventElapsedTime(&t, e.first, e.second));
            ms.push_back(t);
        }
        std::sort(ms.begin(), ms.end());
        double sum = 0.0;
        for (size_t i = 1; i + 1 < ms.size(); ++i) sum += ms[i];
        med[b] = sum / (double)(ms.size() - 2);
    }
    // the reference scores 1; candidate j (block 2j - 1) against the
    // reference blocks 2j - 2 and 2j around it.  A candidate replaces the
    // reference only if it is at least kTuneMargin faster: closer scores are
    // within the run-to-run spread (a 4- or 8-brick z chunk on one 512^3
    // volume picked by noise cost the step 1.5 %).
    constexpr double kTuneMargin = 0.01;
    int best = 0;
    double best_score = 1.0 - kTuneMargin, best_ms = med[0];
    for (int j = 1; j < nc; ++j) {
        const double ref = 0.5 * (med[2 * j - 2] + med[2 * j]);
        const double score = med[2 * j - 1] / ref;
        if (score < best_score) {
            best_score = score;
            best = j;
            best_ms = med[2 * j - 1];
        }
    }
    c->tune_cache[T.key] = std::make_pair(T.cands[best], best_ms);
    append_tune_cache(c, T.key, T.cands[best], best_ms);
    for (auto& e : T.ev) {
        c->event_pool.push_back(e.first);
        c->event_pool.push_back(e.second);
    }
    T = mvf_ctx::Tuning{};
    return MVF_OK;
}

}  // namespace

// ============================================================================
// Public API
// ============================================================================

extern "C" {

const char* mvf_version(void) { return "mvf 0.1 (gfx950)"; }

const char* mvf_status_string(mvf_status s)
{
    switch (s) {
    case MVF_OK: return "ok";
    case MVF_ERR_INVALID_ARG: return "invalid argument";
    case MVF_ERR_NOT_FOUND: return "not found";
    case MVF_ERR_OOM: return "out of memory";
    case MVF_ERR_BUDGET: return "exceeds device budget";
    case MVF_ERR_HIP: return "HIP runtime error";
    case MVF_ERR_STATE: return "invalid state";
    case MVF_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char* mvf_last_error(void) { return g_last_error.c_str(); }

mvf_status mvf_create(mvf_ctx** out, const mvf_config* cfg)
{
    if (!out) return set_error(MVF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mvf_config c0{};
    if (cfg) c0 = *cfg;
    if (c0.ray_step == 0.0f) c0.ray_step = 0.5f;
    if (c0.t_far == 0.0f) c0.t_far = 10.0f;
    if (!(c0.ray_step > 0.0f && c0.ray_step < 1.0f))
        return set_error(MVF_ERR_INVALID_ARG, "ray_step must be in (0, 1), got %g", (double)c0.ray_step);
    if (!(c0.t_far > 0.0f && std::isfinite(c0.t_far)))
        return set_error(MVF_ERR_INVALID_ARG, "t_far must be positive");
    int ndev = 0;
    CHECK_HIP(hipGetDeviceCount(&ndev));
    if (c0.device < 0 || c0.device >= ndev)
        return set_error(MVF_ERR_INVALID_ARG, "device %d not present (%d devices)", c0.device, ndev);
    CHECK_HIP(hipSetDevice(c0.device));
    mvf_ctx* c = new mvf_ctx();
    c->cfg = c0;
    c->device = c0.device;
    c->budget = c0.hbm_budget_bytes ? c0.hbm_budget_bytes : ~0ull;
    if (const char* fs = getenv("MVF_FAULT_SLAB_ALLOCS")) c->fault_slab_allocs = std::max(0, atoi(fs));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c0.device) == hipSuccess) c->n_cus = prop.multiProcessorCount;
    auto fail = [&](mvf_status st) {
        mvf_destroy(c);
        return st;
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&c->d2h_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->h2d_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->h2d_last, hipEventDisableTiming | hipEventDisableSystemFence)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipMalloc((void**)&c->counters, sizeof(unsigned long long) * kCntNum * kCntSlots)) != hipSuccess ||
        (e = hipMemset(c->counters, 0, sizeof(unsigned long long) * kCntNum * kCntSlots)) != hipSuccess ||
        (e = hipHostMalloc((void**)&c->arena.host, Arena::kSlots * Arena::kSlotBytes, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc((void**)&c->arena.dev, Arena::kSlots * Arena::kSlotBytes)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->tail, hipEventDisableTiming | hipEventDisableSystemFence)) != hipSuccess)
        return fail(set_error(MVF_ERR_HIP, "context setup: %s", hipGetErrorString(e)));
    for (int i = 0; i < Arena::kSlots; ++i)
        // the host waits on these before rewriting a slot the device has read
        if ((e = hipEventCreateWithFlags(&c->arena.ev[i], hipEventDisableTiming | hipEventDisableSystemFence)) !=
            hipSuccess)
            return fail(set_error(MVF_ERR_HIP, "context setup: %s", hipGetErrorString(e)));
    // device address of the allocation-free backward's static scratch (once
    // per device, with the device current)
    if (int se = diffray_scratch_init(c0.device))
        return fail(set_error(MVF_ERR_HIP, "static scratch address: %s", hipGetErrorString((hipError_t)se)));
    if ((e = hipDeviceSynchronize()) != hipSuccess)
        return fail(set_error(MVF_ERR_HIP, "context setup: %s", hipGetErrorString(e)));
    *out = c;
    return MVF_OK;
}

mvf_status mvf_destroy(mvf_ctx* c)
{
    if (!c) return MVF_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    destroy_step_graph(c);
    for (auto& v : c->vols) {
        if (v.dev) (void)hipFree(v.dev);
        if (v.host) (void)hipHostFree(v.host);
        if (v.host_ready) (void)hipEventDestroy(v.host_ready);
    }
    for (auto& s : c->pool) {
        (void)hipFree(s.ptr);
        for (hipEvent_t e : s.chunk_done) (void)hipEventDestroy(e);
    }
    for (auto& kv : c->scratch) {
        Scratch& s = kv.second;
        if (s.range) (void)hipFree(s.range);
        if (s.color) (void)hipFree(s.color);
        if (s.rmax) (void)hipFree(s.rmax);
        if (s.ztab) (void)hipFree(s.ztab);
        if (s.tmax) (void)hipFree(s.tmax);
        if (s.visit) (void)hipFree(s.visit);
        if (s.list) (void)hipFree(s.list);
        if (s.list_count) (void)hipFree(s.list_count);
        if (s.rb_lo) (void)hipFree(s.rb_lo);
        if (s.rb_hi) (void)hipFree(s.rb_hi);
        if (s.rb_entries) (void)hipFree(s.rb_entries);
        if (s.rb_counts) (void)hipFree(s.rb_counts);
        if (s.tile_cost) (void)hipFree(s.tile_cost);
        if (s.tile_order) (void)hipFree(s.tile_order);
        if (s.best_t) (void)hipFree(s.best_t);
        if (s.best_id) (void)hipFree(s.best_id);
    }
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto ev : c->event_pool) (void)hipEventDestroy(ev);
    for (auto& e : c->tuning.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (int i = 0; i < Arena::kSlots; ++i)
        if (c->arena.ev[i]) (void)hipEventDestroy(c->arena.ev[i]);
    if (c->arena.host) (void)hipHostFree(c->arena.host);
    if (c->arena.dev) (void)hipFree(c->arena.dev);
    if (c->counters) (void)hipFree(c->counters);
    if (c->place_table) (void)hipFree(c->place_table);
    if (c->place_overflow) (void)hipFree(c->place_overflow);
    if (c->place_T) (void)hipFree(c->place_T);
    if (c->place_boxes) (void)hipFree(c->place_boxes);
    if (c->diff_partials) (void)hipFree(c->diff_partials);
    if (c->extract_buf) (void)hipFree(c->extract_buf);
    if (c->track.dev) (void)hipFree(c->track.dev);
    if (c->track.host) (void)hipHostFree(c->track.host);
    if (c->tail) (void)hipEventDestroy(c->tail);
    if (c->d2h_stream) (void)hipStreamDestroy(c->d2h_stream);
    if (c->h2d_stream) (void)hipStreamDestroy(c->h2d_stream);
    if (c->h2d_last) (void)hipEventDestroy(c->h2d_last);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
    return MVF_OK;
}

mvf_status mvf_synchronize(mvf_ctx* c)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    CHECK_HIP(hipSetDevice(c->device));
    CHECK_ST(arena_flush(c));
    if (c->tail_valid) CHECK_HIP(hipEventSynchronize(c->tail_ev));
    CHECK_HIP(hipStreamSynchronize(c->d2h_stream));
    CHECK_HIP(hipStreamSynchronize(c->h2d_stream));
    CHECK_HIP(hipDeviceSynchronize());
    return MVF_OK;
}

mvf_status mvf_set_budget(mvf_ctx* c, uint64_t bytes)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    c->budget = bytes ? bytes : ~0ull;
    c->cfg.hbm_budget_bytes = bytes;
    return MVF_OK;
}

mvf_status mvf_get_stats(mvf_ctx* c, mvf_stats* out)
{
    if (!c || !out) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    CHECK_HIP(hipSetDevice(c->device));
    CHECK_ST(mvf_synchronize(c));
    CHECK_ST(drain_timing(c));
    std::vector<unsigned long long> cnt((size_t)kCntNum * kCntSlots);
    CHECK_HIP(hipMemcpy(cnt.data(), c->counters, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    *out = c->stats;
    out->voxels_updated = 0;
    out->voxels_band = 0;
    out->bricks_projected = 0;
    out->bricks_deep = 0;
    for (int k = 0; k < kCntSlots; ++k) {
        out->voxels_updated += cnt[(size_t)k * kCntNum + kCntUpdated];
        out->voxels_band += cnt[(size_t)k * kCntNum + kCntBand];
        out->bricks_projected += cnt[(size_t)k * kCntNum + kCntBricks];
        out->bricks_deep += cnt[(size_t)k * kCntNum + kCntDeep];
    }
    out->resident_bytes = c->resident_bytes;
    int n = 0;
    for (auto& v : c->vols)
        if (v.alive && v.state == State::Device) ++n;
    out->resident_volumes = n;
    return MVF_OK;
}

mvf_status mvf_reset_stats(mvf_ctx* c)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    CHECK_ST(mvf_synchronize(c));
    CHECK_ST(drain_timing(c));
    c->stats = mvf_stats{};
    CHECK_HIP(hipMemset(c->counters, 0, sizeof(unsigned long long) * kCntNum * kCntSlots));
    CHECK_HIP(hipDeviceSynchronize());
    return MVF_OK;
}

mvf_status mvf_grid_create(mvf_ctx* c, const mvf_grid_desc* d, int32_t* grid_id)
{
    if (!c || !d || !grid_id) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    if (!(d->voxel_size > 0.0f) || !std::isfinite(d->voxel_size))
        return set_error(MVF_ERR_INVALID_ARG, "voxel_size must be positive");
    if (!(d->trunc_voxels > 0.0f) || !std::isfinite(d->trunc_voxels))
        return set_error(MVF_ERR_INVALID_ARG, "trunc_voxels must be positive");
    if (d->w_max < 1) return set_error(MVF_ERR_INVALID_ARG, "w_max must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(d->origin[a])) return set_error(MVF_ERR_INVALID_ARG, "origin not finite");
    Grid g;
    g.d = *d;
    g.mu = d->trunc_voxels * d->voxel_size;
    g.inv_s = 1.0f / d->voxel_size;
    g.inv_mu = 1.0f / g.mu;
    c->grids.push_back(g);
    *grid_id = (int32_t)c->grids.size() - 1;
    return MVF_OK;
}

mvf_status mvf_volume_create(mvf_ctx* c, const mvf_volume_desc* d, int32_t* vol_id)
{
    if (!c || !d || !vol_id) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    if (d->grid_id < 0 || d->grid_id >= (int32_t)c->grids.size())
        return set_error(MVF_ERR_NOT_FOUND, "grid %d", d->grid_id);
    for (int a = 0; a < 3; ++a) {
        if (d->dims[a] < 2 || d->dims[a] > 2048)
            return set_error(MVF_ERR_INVALID_ARG, "dims[%d] = %d outside [2, 2048]", a, d->dims[a]);
        if (d->offset[a] < -(1 << 22) || d->offset[a] > (1 << 22))
            return set_error(MVF_ERR_INVALID_ARG, "offset[%d] = %d out of range", a, d->offset[a]);
    }
    if (d->stream_id < 0) return set_error(MVF_ERR_INVALID_ARG, "stream_id must be >= 0");
    Volume v;
    v.alive = true;
    v.d = *d;
    for (int a = 0; a < 3; ++a) v.bd[a] = (d->dims[a] + kBrick - 1) / kBrick;
    const size_t nb = (size_t)v.bd[0] * v.bd[1] * v.bd[2];
    if (nb * kBrickVox > ((size_t)1 << 30))
        return set_error(MVF_ERR_INVALID_ARG, "volume of %zu padded voxels exceeds 2^30", nb * kBrickVox);
    v.nvox_pad = nb * kBrickVox;
    v.off_W = align_up(v.nvox_pad * 4, kAlign);
    v.off_C = align_up(v.off_W + v.nvox_pad * 2, kAlign);
    v.off_flag = align_up(v.off_C + v.nvox_pad * 4, kAlign);
    v.off_dist = align_up(v.off_flag + nb, kAlign);
    v.off_colm = align_up(v.off_dist + nb, kAlign);
    v.off_fmask = align_up(v.off_colm + 8 * ((size_t)v.bd[0] * v.bd[1] * col_words(v.bd[2]) + 1), kAlign);
    v.off_cmask = align_up(v.off_fmask + 8 * nb, kAlign);
    v.bytes = align_up(v.off_cmask + 8 * nb, kAlign);
    v.nbricks = nb;
    c->vols.push_back(v);
    *vol_id = (int32_t)c->vols.size() - 1;
    return MVF_OK;
}

mvf_status mvf_volume_destroy(mvf_ctx* c, int32_t id)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_ST(mvf_synchronize(c));
    if (v->dev) {
        CHECK_HIP(hipFree(v->dev));
        c->resident_bytes -= v->bytes;
    }
    if (v->host) CHECK_HIP(hipHostFree(v->host));
    if (v->host_ready) CHECK_HIP(hipEventDestroy(v->host_ready));
    *v = Volume();
    for (auto& kv : c->placed)
        for (auto it = kv.second.begin(); it != kv.second.end();)
            it = it->second == id ? kv.second.erase(it) : std::next(it);
    return MVF_OK;
}

mvf_status mvf_volume_place(mvf_ctx* c, int32_t id)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    v->active = true;
    return MVF_OK;
}

mvf_status mvf_volume_evict(mvf_ctx* c, int32_t id, uint32_t flags)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    v->active = false;
    if (flags & MVF_EVICT_SWAP_OUT) {
        hipStream_t s = c->tail_valid ? c->tail_stream : nullptr;
        CHECK_ST(swap_out(c, *v, s));
    }
    return MVF_OK;
}

mvf_status mvf_volume_swap_in(mvf_ctx* c, int32_t id, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    if (!find_volume(c, id)) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    CHECK_ST(ensure_resident(c, std::vector<int>{id}, s));
    return mark_tail(c, s);
}

mvf_status mvf_volume_swap_out(mvf_ctx* c, int32_t id, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    CHECK_ST(swap_out(c, *v, s));
    return mark_tail(c, s);
}

mvf_status mvf_volume_extract(mvf_ctx* c, int32_t id, float* V, float* N, int32_t* G, int64_t cap,
                              int64_t* n_total, void* stream)
{
    if (!c || !n_total) return set_error(MVF_ERR_INVALID_ARG, "ctx or n_total is NULL");
    if (cap < 0) return set_error(MVF_ERR_INVALID_ARG, "cap must be >= 0");
    if (cap > 0 && (!V || !N)) return set_error(MVF_ERR_INVALID_ARG, "V and N are needed when cap > 0");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    *n_total = 0;
    if (v->state == State::Empty) return mark_tail(c, s);  // never observed: no surface
    CHECK_ST(ensure_resident(c, std::vector<int>{id}, s));
    const size_t nb = v->nbricks;
    if (nb > c->extract_buf_n) {
        if (c->extract_buf) {
            CHECK_HIP(hipStreamSynchronize(s));
            CHECK_HIP(hipFree(c->extract_buf));
            c->extract_buf = nullptr;
            c->extract_buf_n = 0;
        }
        if (hipMalloc((void**)&c->extract_buf, align_up(4 * nb, kAlign) + 8 * nb + 8) != hipSuccess) {
            (void)hipGetLastError();
            c->extract_buf = nullptr;
            return set_error(MVF_ERR_OOM, "surface extraction scratch of %zu bricks", nb);
        }
        c->extract_buf_n = nb;
    }
    uint32_t* counts = reinterpret_cast<uint32_t*>(c->extract_buf);
    unsigned long long* offsets = reinterpret_cast<unsigned long long*>(c->extract_buf + align_up(4 * nb, kAlign));
    long long* total = reinterpret_cast<long long*>(offsets + nb);
    DevVolume dv = make_dev(c, *v);
    CHECK_LAUNCH(launch_extract(dv, counts, offsets, total, V, N, G, (long long)cap, s));
    long long n = 0;
    CHECK_HIP(hipMemcpyAsync(&n, total, sizeof(n), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    *n_total = (int64_t)n;
    return mark_tail(c, s);
}

mvf_status mvf_volume_describe(mvf_ctx* c, int32_t id, mvf_volume_desc* out)
{
    if (!c || !out) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    *out = v->d;
    return MVF_OK;
}

mvf_status mvf_volume_query(mvf_ctx* c, int32_t id, int32_t* resident, uint64_t* bytes, int32_t* active)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    if (resident) *resident = v->state == State::Device ? 1 : 0;
    if (bytes) *bytes = v->bytes;
    if (active) *active = v->active ? 1 : 0;
    return MVF_OK;
}

mvf_status mvf_volume_brick_summary(mvf_ctx* c, int32_t id, uint8_t* flag, uint8_t* dist)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    CHECK_ST(mvf_synchronize(c));
    const size_t nb = v->nbricks;
    if (v->state == State::Empty) {
        if (flag) memset(flag, 0, nb);
        if (dist) memset(dist, kDistCap, nb);
        return MVF_OK;
    }
    if (v->state == State::Host) {
        if (flag) memcpy(flag, v->host + v->off_flag, nb);
        if (dist) memcpy(dist, v->host + v->off_dist, nb);
        return MVF_OK;
    }
    if (flag) CHECK_HIP(hipMemcpy(flag, v->dev + v->off_flag, nb, hipMemcpyDeviceToHost));
    if (dist) CHECK_HIP(hipMemcpy(dist, v->dev + v->off_dist, nb, hipMemcpyDeviceToHost));
    return MVF_OK;
}

mvf_status mvf_volume_read(mvf_ctx* c, int32_t id, float* F, uint16_t* W, uint8_t* rgba)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    CHECK_ST(mvf_synchronize(c));
    const size_t n = (size_t)v->d.dims[0] * v->d.dims[1] * v->d.dims[2];
    if (v->state == State::Empty) {
        if (F) memset(F, 0, n * sizeof(float));
        if (W) memset(W, 0, n * sizeof(uint16_t));
        if (rgba) memset(rgba, 0, n * 4);
        return MVF_OK;
    }
    // bring the state to the device (the mirror is in device layout)
    uint8_t* slab = v->dev;
    uint8_t* tmp_slab = nullptr;
    if (v->state == State::Host) {
        CHECK_HIP(hipMalloc((void**)&tmp_slab, v->bytes));
        CHECK_HIP(hipMemcpy(tmp_slab, v->host, v->bytes, hipMemcpyHostToDevice));
        slab = tmp_slab;
    }
    Volume view = *v;
    view.dev = slab;
    DevVolume dv = make_dev(c, view);
    dv.id = id;
    float* dF = nullptr;
    uint16_t* dW = nullptr;
    uint32_t* dC = nullptr;
    mvf_status st = MVF_OK;
    hipError_t e = hipSuccess;
    if (F && (e = hipMalloc((void**)&dF, n * 4)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK && W && (e = hipMalloc((void**)&dW, n * 2)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK && rgba && (e = hipMalloc((void**)&dC, n * 4)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK) {
        int le = launch_to_canonical(dv, dF, dW, dC, nullptr);
        if (le) { st = MVF_ERR_HIP; e = (hipError_t)le; }
    }
    if (st == MVF_OK && (e = hipDeviceSynchronize()) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK && F && (e = hipMemcpy(F, dF, n * 4, hipMemcpyDeviceToHost)) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK && W && (e = hipMemcpy(W, dW, n * 2, hipMemcpyDeviceToHost)) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK && rgba && (e = hipMemcpy(rgba, dC, n * 4, hipMemcpyDeviceToHost)) != hipSuccess) st = MVF_ERR_HIP;
    if (dF) (void)hipFree(dF);
    if (dW) (void)hipFree(dW);
    if (dC) (void)hipFree(dC);
    if (tmp_slab) (void)hipFree(tmp_slab);
    if (st != MVF_OK) return set_error(st, "volume_read: %s", hipGetErrorString(e));
    return MVF_OK;
}

mvf_status mvf_volume_write(mvf_ctx* c, int32_t id, const float* F, const uint16_t* W, const uint8_t* rgba)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    Volume* v = find_volume(c, id);
    if (!v) return set_error(MVF_ERR_NOT_FOUND, "volume %d", id);
    CHECK_HIP(hipSetDevice(c->device));
    CHECK_ST(mvf_synchronize(c));
    CHECK_ST(ensure_resident(c, std::vector<int>{id}, nullptr));
    const size_t n = (size_t)v->d.dims[0] * v->d.dims[1] * v->d.dims[2];
    float* dF = nullptr;
    uint16_t* dW = nullptr;
    uint32_t* dC = nullptr;
    mvf_status st = MVF_OK;
    hipError_t e = hipSuccess;
    if (F && (e = hipMalloc((void**)&dF, n * 4)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK && W && (e = hipMalloc((void**)&dW, n * 2)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK && rgba && (e = hipMalloc((void**)&dC, n * 4)) != hipSuccess) st = MVF_ERR_OOM;
    if (st == MVF_OK && F && (e = hipMemcpy(dF, F, n * 4, hipMemcpyHostToDevice)) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK && W && (e = hipMemcpy(dW, W, n * 2, hipMemcpyHostToDevice)) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK && rgba && (e = hipMemcpy(dC, rgba, n * 4, hipMemcpyHostToDevice)) != hipSuccess) st = MVF_ERR_HIP;
    if (st == MVF_OK) {
        DevVolume dv = make_dev(c, *v);
        int le = launch_volume_init(dv, nullptr);
        if (!le) le = launch_from_canonical(dv, dF, dW, dC, nullptr);
        if (le) { st = MVF_ERR_HIP; e = (hipError_t)le; }
        else {
            const mvf_status sst = recompute_summaries(c, *v, nullptr);
            if (sst != MVF_OK) {
                if (dF) (void)hipFree(dF);
                if (dW) (void)hipFree(dW);
                if (dC) (void)hipFree(dC);
                return sst;
            }
        }
    }
    if (st == MVF_OK && (e = hipDeviceSynchronize()) != hipSuccess) st = MVF_ERR_HIP;
    if (dF) (void)hipFree(dF);
    if (dW) (void)hipFree(dW);
    if (dC) (void)hipFree(dC);
    if (st != MVF_OK) return set_error(st, "volume_write: %s", hipGetErrorString(e));
    return MVF_OK;
}

mvf_status mvf_integrate(mvf_ctx* c, int32_t sid, const mvf_frame* f, const float T_wc[12], const mvf_intrinsics* K,
                         void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    CHECK_ST(check_frame(f));
    if (!T_wc || !finite_pose(T_wc)) return set_error(MVF_ERR_INVALID_ARG, "pose is NULL or not finite");
    if (!valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "intrinsics NULL, not finite or zero focal length");
    if (sid < 0) return set_error(MVF_ERR_INVALID_ARG, "stream_id must be >= 0");
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    std::vector<int> ids = stream_volumes(c, sid, T_wc, *K, f->width, f->height);
    CHECK_ST(integrate_plain(c, sid, f, T_wc, *K, ids, s));
    return mark_tail(c, s);
}

mvf_status mvf_raycast(mvf_ctx* c, int32_t sid, const float T_wc[12], const mvf_intrinsics* K,
                       const mvf_raycast_out* out, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    if (!out || !out->depth) return set_error(MVF_ERR_INVALID_ARG, "out or out->depth is NULL");
    if (out->width <= 0 || out->height <= 0 || out->width > 16384 || out->height > 16384)
        return set_error(MVF_ERR_INVALID_ARG, "output size %dx%d out of range", out->width, out->height);
    if (!T_wc || !finite_pose(T_wc)) return set_error(MVF_ERR_INVALID_ARG, "pose is NULL or not finite");
    if (!valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "intrinsics NULL, not finite or zero focal length");
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    std::vector<int> ids = stream_volumes(c, sid, T_wc, *K, out->width, out->height);
    // all volumes of one raycast must share one grid (one sample lattice)
    for (int id : ids)
        if (c->vols[id].d.grid_id != c->vols[ids[0]].d.grid_id)
            return set_error(MVF_ERR_UNSUPPORTED, "volumes of stream %d lie on different grids", sid);
    CHECK_ST(raycast_plain(c, sid, T_wc, *K, out, ids, s));
    return mark_tail(c, s);
}

// ---- batched step -------------------------------------------------------------

mvf_status mvf_step(mvf_ctx* c, int32_t n, const mvf_stream_frame* frames, const mvf_raycast_out* outs, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    if (n <= 0 || n > 1024 || !frames || !outs) return set_error(MVF_ERR_INVALID_ARG, "bad stream count or NULL arrays");
    for (int i = 0; i < n; ++i) {
        CHECK_ST(check_frame(&frames[i].frame));
        if (!finite_pose(frames[i].T_wc)) return set_error(MVF_ERR_INVALID_ARG, "pose %d not finite", i);
        if (!valid_K(&frames[i].K)) return set_error(MVF_ERR_INVALID_ARG, "intrinsics %d invalid", i);
        if (!outs[i].depth || outs[i].width <= 0 || outs[i].height <= 0 || outs[i].width > 16384 ||
            outs[i].height > 16384)
            return set_error(MVF_ERR_INVALID_ARG, "output %d invalid", i);
        if (frames[i].stream_id < 0) return set_error(MVF_ERR_INVALID_ARG, "stream_id %d", frames[i].stream_id);
        for (int j = 0; j < i; ++j)
            if (frames[j].stream_id == frames[i].stream_id)
                return set_error(MVF_ERR_INVALID_ARG, "stream %d appears twice", frames[i].stream_id);
    }
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));

    // volumes per stream (integration set == raycast set: active and in view)
    std::vector<std::vector<int>> per(n);
    std::vector<int> all;
    int grid0 = -1;
    for (int i = 0; i < n; ++i) {
        const mvf_stream_frame& fr = frames[i];
        per[i] = stream_volumes(c, fr.stream_id, fr.T_wc, fr.K, fr.frame.width, fr.frame.height);
        // raycast view may differ in size from the frame; use the union test
        std::vector<int> rv = stream_volumes(c, fr.stream_id, fr.T_wc, fr.K, outs[i].width, outs[i].height);
        for (int id : rv)
            if (std::find(per[i].begin(), per[i].end(), id) == per[i].end()) per[i].push_back(id);
        std::sort(per[i].begin(), per[i].end());
        for (int id : per[i]) {
            all.push_back(id);
            if (grid0 < 0) grid0 = c->vols[id].d.grid_id;
            if (c->vols[id].d.grid_id != grid0)
                return set_error(MVF_ERR_UNSUPPORTED, "batched step needs all volumes on one grid");
        }
    }
    // volumes that do not all fit the budget are processed in waves (the
    // paper's memory passing, down to one volume at a time): each wave is one
    // replay of the captured step over the wave's volumes, raycasts merged
    // through the per-pixel best (t*, id) of the earlier waves
    std::vector<std::vector<int>> waves = plan_waves(c, all);
    if (waves.empty()) waves.push_back({});
    const bool multi_wave = waves.size() > 1;

    bool tuning = false;
    const std::string key = step_key(c, n, outs, all);
    mvf_schedule sch = pick_schedule(c, key, &tuning);
    if (multi_wave && tuning) {
        // a step split into waves is not a representative sample for the tuner
        tuning = false;
        sch = c->tune_cache.count(key) ? c->tune_cache[key].first : c->fixed_sched;
        if (c->tune_mode != MVF_AUTOTUNE_OFF && !c->tune_cache.count(key)) sch = mvf_schedule{4, 0, kRayLanes, 0};
    }
    StepGraph& G = c->step;
    int max_w = 0, max_h = 0;
    for (int i = 0; i < n; ++i) {
        max_w = std::max(max_w, frames[i].frame.width);
        max_h = std::max(max_h, frames[i].frame.height);
    }
    // capacities from the whole set (every wave is a subset of it)
    int ztotal = 0, items_total = 0, bricks_total = 0;
    for (int id : all) {
        const Volume& v = c->vols[id];
        ztotal += kBrick * v.bd[2];
        items_total += v.bd[0] * v.bd[1] * ((v.bd[2] + sch.zchunk - 1) / sch.zchunk);
        bricks_total += (int)align_up(v.nbricks, 64);
    }
    bool same_shape = G.valid && G.n == n && (int)all.size() <= G.max_vols && max_w <= G.max_w && max_h <= G.max_h &&
                      ztotal <= G.ztab_cap && items_total <= G.visit_cap && bricks_total <= G.rb_entries_cap &&
                      same_schedule(sch, G.sched);
    if (same_shape) {
        for (int i = 0; i < n; ++i)
            if (G.out_w[i] != outs[i].width || G.out_h[i] != outs[i].height) same_shape = false;
    }
    const int tw = ray_tile_w(sch.ray_lanes), th = ray_tile_h(sch.ray_lanes);  // one wavefront per block
    if (!same_shape) {
        CHECK_ST(destroy_step_graph(c));
        G.sched = sch;
        G.n = n;
        G.max_vols = std::max<int>((int)all.size() * 2, 16);
        G.max_w = max_w;
        G.max_h = max_h;
        G.out_w.assign(n, 0);
        G.out_h.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            G.out_w[i] = outs[i].width;
            G.out_h[i] = outs[i].height;
        }
        size_t off = 0;
        auto take = [&](size_t bytes) { size_t o = align_up(off, 256); off = o + bytes; return o; };
        G.off_hdr = take(sizeof(LaunchHeader));
        G.off_prep = take(sizeof(PrepItem) * n);
        G.off_frames = take(sizeof(DevFrame) * n);
        G.off_vols = take(sizeof(DevVolume) * G.max_vols);
        G.off_items = take(sizeof(int32_t) * (G.max_vols + 1));
        G.off_lists = take(sizeof(int32_t) * G.max_vols);
        G.off_lbase = take(sizeof(int32_t) * (n + 1));
        G.off_tbase = take(sizeof(int32_t) * (n + 1));
        G.off_bbase = take(sizeof(int32_t) * (G.max_vols + 1));
        G.dev_bytes = align_up(off, 256);
        if (G.dev_bytes > Arena::kSlotBytes) return set_error(MVF_ERR_INVALID_ARG, "step tables too large");
        CHECK_HIP(hipMalloc((void**)&G.dev, G.dev_bytes));
        G.ztab_cap = std::max(ztotal * 2, 1024);
        CHECK_HIP(hipMalloc((void**)&G.ztab, (size_t)G.ztab_cap * 3 * sizeof(float)));
        G.visit_cap = std::max(items_total * 2, 1024);
        CHECK_HIP(hipMalloc((void**)&G.visit, (size_t)G.visit_cap * kVisitPerItem));
        CHECK_HIP(hipMalloc((void**)&G.list, (size_t)G.visit_cap * (2 * kVisitPerItem) * sizeof(int32_t)));
        CHECK_HIP(hipMalloc((void**)&G.list_count, 2 * sizeof(unsigned long long)));
        CHECK_HIP(hipMemset(G.list_count, 0, 2 * sizeof(unsigned long long)));
        int counts_cap = 0;
        CHECK_ST(get_footprint_buffers(&G.rb_entries, &G.rb_entries_cap, &G.rb_counts, &counts_cap,
                                       std::max(bricks_total * 2, 1024), G.max_vols));
        G.max_cells_x = G.max_cells_y = 0;
        for (int i = 0; i < n; ++i) {
            G.max_cells_x = std::max(G.max_cells_x, (outs[i].width + kBoundCell - 1) / kBoundCell);
            G.max_cells_y = std::max(G.max_cells_y, (outs[i].height + kBoundCell - 1) / kBoundCell);
        }
        G.integ_blocks = c->n_cus * 8;
        int tiles = 0;
        for (int i = 0; i < n; ++i) tiles += ((outs[i].width + tw - 1) / tw) * ((outs[i].height + th - 1) / th);
        G.ray_tiles = tiles;
        G.ray_blocks = ray_blocks(tiles);
        CHECK_ST(alloc_tile_buffers(tiles, &G.tile_cost, &G.tile_order));
    }
    // scratch per stream (with the running best of a multi-wave raycast)
    std::vector<Scratch*> sc(n);
    for (int i = 0; i < n; ++i)
    {
        CHECK_ST(get_scratch(c, frames[i].stream_id, frames[i].frame.width, frames[i].frame.height, false, &sc[i]));
        CHECK_ST(get_bound_buffers(sc[i], outs[i].width, outs[i].height));
        if (multi_wave) CHECK_ST(get_best_buffers(sc[i], outs[i].width * outs[i].height));
    }
    // nearest-first order of each stream's volumes (raycast lists; only speed)
    std::vector<std::vector<int>> order(n);
    for (int i = 0; i < n; ++i) {
        std::vector<double> dist;
        for (int id : per[i]) dist.push_back(box_distance(c, c->vols[id], frames[i].T_wc));
        std::vector<int> ord(per[i].size());
        for (size_t j = 0; j < ord.size(); ++j) ord[j] = (int)j;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
            return dist[a] < dist[b] || (dist[a] == dist[b] && per[i][a] < per[i][b]);
        });
        for (int j : ord) order[i].push_back(per[i][j]);
    }
    const RayParams rp = grid0 >= 0 ? ray_params(c, c->grids[grid0]) : RayParams{1.0f, 0};

    hipEvent_t t0;
    CHECK_ST(timing_begin(c, s, &t0));
    for (size_t wi = 0; wi < waves.size(); ++wi) {
        const std::vector<int>& wave = waves[wi];
        CHECK_ST(ensure_resident(c, wave, s));
        std::vector<char> in_wave(c->vols.size(), 0);
        for (int id : wave) in_wave[id] = 1;
        // host image of the tables, uploaded to G.dev by the graph's first node
        int slot;
        Writer w;
        CHECK_ST(arena_acquire(c, &slot, &w));
        uint8_t* img = w.host;
        memset(img, 0, G.dev_bytes);
        w.used = G.dev_bytes;
        LaunchHeader* h = reinterpret_cast<LaunchHeader*>(img + G.off_hdr);
        PrepItem* prep = reinterpret_cast<PrepItem*>(img + G.off_prep);
        DevFrame* dfr = reinterpret_cast<DevFrame*>(img + G.off_frames);
        DevVolume* vt = reinterpret_cast<DevVolume*>(img + G.off_vols);
        int32_t* ib = reinterpret_cast<int32_t*>(img + G.off_items);
        int32_t* lists = reinterpret_cast<int32_t*>(img + G.off_lists);
        int32_t* lb = reinterpret_cast<int32_t*>(img + G.off_lbase);
        int32_t* tb = reinterpret_cast<int32_t*>(img + G.off_tbase);
        int32_t* bbase = reinterpret_cast<int32_t*>(img + G.off_bbase);
        int nbr = 0, nv = 0, items = 0, zt = 0, tiles = 0;
        const int zc = sch.zchunk;
        lb[0] = 0;
        tb[0] = 0;
        for (int i = 0; i < n; ++i) {
            const mvf_stream_frame& fr = frames[i];
            PrepItem& p = prep[i];
            p.depth = fr.frame.depth;
            p.rgb = fr.frame.rgb;
            p.depth_pitch = fr.frame.depth_pitch ? fr.frame.depth_pitch : fr.frame.width;
            p.rgb_pitch = fr.frame.rgb_pitch ? fr.frame.rgb_pitch : 3 * fr.frame.width;
            p.width = fr.frame.width;
            p.height = fr.frame.height;
            p.fx = fr.K.fx; p.fy = fr.K.fy; p.cx = fr.K.cx; p.cy = fr.K.cy;
            p.range = sc[i]->range;
            p.color = sc[i]->color;
            p.rmax = sc[i]->rmax;
            p.tmax = sc[i]->tmax;
            fill_frame(&dfr[i], sc[i], fr.frame.width, fr.frame.height, fr.T_wc, fr.K);
            set_bounds(&dfr[i], sc[i], outs[i].width, outs[i].height);
            if (!fr.frame.rgb) dfr[i].color = nullptr;
            dfr[i].depth = outs[i].depth;
            dfr[i].vertex = outs[i].vertex;
            dfr[i].normal = outs[i].normal;
            dfr[i].hit = outs[i].hit;
            dfr[i].out_w = outs[i].width;
            dfr[i].out_h = outs[i].height;
            if (multi_wave) {
                dfr[i].best_t = sc[i]->best_t;
                dfr[i].best_id = sc[i]->best_id;
            }
            // this stream's volumes of the wave: table entries in id order,
            // the raycast list nearest first
            const int first = nv;
            std::vector<int> slot_of(c->vols.size(), -1);
            for (int id : per[i]) {
                if (!in_wave[id]) continue;
                Volume& v = c->vols[id];
                vt[nv] = make_dev(c, v);
                vt[nv].frame = i;
                vt[nv].zt_base = zt;
                zt += kBrick * v.bd[2];
                ib[nv] = items;
                bbase[nv] = nbr;
                nbr += (int)align_up(v.nbricks, 64);  // volumes start on a wavefront
                items += v.bd[0] * v.bd[1] * ((v.bd[2] + zc - 1) / zc);
                slot_of[id] = nv;
                ++nv;
            }
            int li = first;
            for (int id : order[i])
                if (slot_of[id] >= 0) lists[li++] = slot_of[id];
            lb[i + 1] = nv;
            tiles += ((outs[i].width + tw - 1) / tw) * ((outs[i].height + th - 1) / th);
            tb[i + 1] = tiles;
        }
        ib[nv] = items;
        bbase[nv] = nbr;
        h->nvol = nv;
        h->total_bricks = nbr;
        h->total_items = items;
        h->total_z = zt;
        h->zchunk = zc;
        h->nstreams = n;
        h->total_tiles = tiles;
        h->first_wave = wi == 0 ? 1 : 0;
        h->rp = rp;
        h->rb_parity = G.rb_parity;
        G.rb_parity ^= 1;
        h->list_parity = G.list_parity;
        G.list_parity ^= 1;
        // The graph's first node (frame preparation) copies this image into the
        // fixed tables; its source is pointed at this wave's arena slot.
        if (!G.valid) {
            hipStream_t cs = c->capture_stream;
            const LaunchHeader* dh = reinterpret_cast<const LaunchHeader*>(G.dev + G.off_hdr);
            const DevFrame* dframes = reinterpret_cast<const DevFrame*>(G.dev + G.off_frames);
            const DevVolume* dvols = reinterpret_cast<const DevVolume*>(G.dev + G.off_vols);
            const int32_t* ditems = reinterpret_cast<const int32_t*>(G.dev + G.off_items);
            const int32_t* dlists = reinterpret_cast<const int32_t*>(G.dev + G.off_lists);
            const int32_t* dlb = reinterpret_cast<const int32_t*>(G.dev + G.off_lbase);
            const int32_t* dtb = reinterpret_cast<const int32_t*>(G.dev + G.off_tbase);
            const int32_t* dbb = reinterpret_cast<const int32_t*>(G.dev + G.off_bbase);
            CHECK_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            // the first node reads this step's prep items from the slot and
            // copies the slot's tables to G.dev
            int e1 = launch_frame_prep(reinterpret_cast<const PrepItem*>(w.host + G.off_prep), n, G.max_w, G.max_h, cs,
                                       w.host, G.dev, G.dev_bytes);
            // integration's block 0 orders the raycast's tile groups (slowest of
            // the last step first)
            IntegrateLaunch IL{dh, dvols, dframes, ditems, c->counters, G.ztab, G.visit,
                               G.tile_cost, G.tile_order, G.ray_tiles, G.list, G.list_count,
                               G.list + (size_t)G.visit_cap * kVisitPerItem};
            int e2 = e1 ? e1 : launch_ztable(IL, items_total * zc, cs);
            // one wavefront per work item of the whole volume set (a larger
            // set later is walked by the kernel's grid-stride loop)
            G.integ_blocks = (sch.persistent ? c->n_cus * 8 : std::max(c->n_cus * 8, (items_total + 3) / 4)) + 1;
            if (!e2) e2 = launch_integrate(IL, G.integ_blocks, cs);
            // the last distance pass also collects the raycast range-bound
            // footprints; the merge folds them per cell
            const RayBounds RB{G.rb_entries, G.rb_counts, G.max_vols};
            if (!e2) e2 = launch_brick_distance(dh, dvols, dbb, c->n_cus * 4, cs, dframes, RB);
            if (!e2) e2 = launch_ray_bounds_merge(dh, dframes, dlists, dlb, dbb, RB, n, G.max_cells_x, G.max_cells_y, cs);
            RaycastLaunch RL{dh, dvols, dframes, dlists, dlb, dtb, tw, th, sch.ray_lanes, G.tile_cost, G.tile_order};
            int e3 = e2 ? e2 : launch_raycast(RL, G.ray_blocks, cs);
            hipError_t ee = hipStreamEndCapture(cs, &G.graph);
            if (e3) return set_error(MVF_ERR_HIP, "step capture: %s", hipGetErrorString((hipError_t)e3));
            if (ee != hipSuccess) return set_error(MVF_ERR_HIP, "step capture: %s", hipGetErrorString(ee));
            CHECK_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
            // frame preparation (with the table upload) is the graph's only root
            G.copy_node = nullptr;
            size_t nr = 1;
            CHECK_HIP(hipGraphGetRootNodes(G.graph, &G.copy_node, &nr));
            if (nr != 1 || !G.copy_node) return set_error(MVF_ERR_HIP, "step capture: no frame preparation node");
            G.valid = true;
        } else {
            CHECK_HIP((hipError_t)set_frame_prep_node(G.exec, G.copy_node,
                                                      reinterpret_cast<const PrepItem*>(w.host + G.off_prep), n,
                                                      G.max_w, G.max_h, w.host, G.dev, G.dev_bytes));
        }
        hipEvent_t tune_a = nullptr, tune_b = nullptr;
        if (tuning) {
            CHECK_ST(get_event(c, &tune_a));
            CHECK_ST(get_event(c, &tune_b));
            CHECK_HIP(hipEventRecord(tune_a, s));
        }
        CHECK_HIP(hipGraphLaunch(G.exec, s));
        if (tuning) {
            CHECK_HIP(hipEventRecord(tune_b, s));
            c->tuning.ev.push_back(std::make_pair(tune_a, tune_b));
            c->tuning.next += 1;
        }
        CHECK_ST(arena_release_step(c, slot, s));  // reused once the replay that reads it is done
    }
    CHECK_ST(timing_end(c, s, t0, 2));
    c->last_sched = sch;
    if (tuning) CHECK_ST(finish_tuning(c));
    c->stats.step_launches += 1;
    for (int i = 0; i < n; ++i) c->stats.pixels_raycast += (uint64_t)outs[i].width * outs[i].height;
    return MVF_OK;
}

mvf_status mvf_set_schedule(mvf_ctx* c, const mvf_schedule* sched)
{
    if (!c || !sched) return set_error(MVF_ERR_INVALID_ARG, "ctx or schedule is NULL");
    if (!valid_schedule(*sched) || sched->reserved != 0)
        return set_error(MVF_ERR_INVALID_ARG, "schedule {%d, %d, %d} out of range", sched->zchunk, sched->persistent,
                         sched->ray_lanes);
    c->fixed_sched = *sched;
    c->tune_mode = MVF_AUTOTUNE_OFF;
    return MVF_OK;
}

mvf_status mvf_get_schedule(mvf_ctx* c, mvf_schedule* out)
{
    if (!c || !out) return set_error(MVF_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = c->last_sched;
    return MVF_OK;
}

mvf_status mvf_autotune(mvf_ctx* c, int32_t mode, const char* cache_path)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    if (mode != MVF_AUTOTUNE_OFF && mode != MVF_AUTOTUNE_TUNE && mode != MVF_AUTOTUNE_CACHED)
        return set_error(MVF_ERR_INVALID_ARG, "autotune mode %d", mode);
    c->tune_path = cache_path ? cache_path : "";
    if (!c->tune_path.empty()) CHECK_ST(read_tune_cache(c, c->tune_path));
    c->tune_mode = mode;
    return MVF_OK;
}

// ---- placement ------------------------------------------------------------------

mvf_status mvf_placement_policy(const int32_t* active, int32_t n_active, const int32_t* cells,
                                const int32_t* counts, int32_t n_cells, int32_t n_max, float beta,
                                int32_t* out_active, int32_t* n_out, int32_t* added, int32_t* n_added,
                                int32_t* removed, int32_t* n_removed)
{
    if (n_active < 0 || n_cells < 0 || n_max < 0 || !(beta >= 1.0f) || !n_out || !n_added || !n_removed ||
        (n_active && !active) || (n_cells && (!cells || !counts)) || (n_max && !out_active))
        return set_error(MVF_ERR_INVALID_ARG, "placement_policy: bad arguments");
    typedef std::vector<int> Key;
    auto key_of = [](const int32_t* p) { return Key{p[0], p[1], p[2]}; };
    std::map<Key, long long> cnt;
    for (int i = 0; i < n_cells; ++i) {
        if (counts[i] < 0) return set_error(MVF_ERR_INVALID_ARG, "negative count");
        cnt[key_of(cells + 3 * i)] += counts[i];
    }
    std::vector<Key> H;
    for (int i = 0; i < n_active; ++i) {
        Key k = key_of(active + 3 * i);
        if (std::find(H.begin(), H.end(), k) == H.end()) H.push_back(k);
    }
    // candidates: counted cells not in H, count desc then cell asc
    std::vector<std::pair<long long, Key>> cand;
    for (auto& kv : cnt)
        if (kv.second > 0 && std::find(H.begin(), H.end(), kv.first) == H.end()) cand.push_back({kv.second, kv.first});
    std::sort(cand.begin(), cand.end(), [](const std::pair<long long, Key>& a, const std::pair<long long, Key>& b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    std::vector<Key> add, rem;
    size_t ci = 0;
    while ((int)H.size() < n_max && ci < cand.size()) {
        H.push_back(cand[ci].second);
        add.push_back(cand[ci].second);
        ++ci;
    }
    auto count_of = [&](const Key& k) { auto it = cnt.find(k); return it == cnt.end() ? 0LL : it->second; };
    while (ci < cand.size() && !H.empty()) {
        // lowest-count member; ties go to the lexicographically larger cell
        size_t low = 0;
        for (size_t i = 1; i < H.size(); ++i) {
            const long long a = count_of(H[i]), b = count_of(H[low]);
            if (a < b || (a == b && H[i] > H[low])) low = i;
        }
        if ((double)cand[ci].first > (double)beta * (double)count_of(H[low])) {
            Key gone = H[low];
            H.erase(H.begin() + low);
            auto it = std::find(add.begin(), add.end(), gone);
            if (it != add.end()) add.erase(it); else rem.push_back(gone);
            H.push_back(cand[ci].second);
            add.push_back(cand[ci].second);
            ++ci;
        } else {
            break;
        }
    }
    if ((int)H.size() > n_max) return set_error(MVF_ERR_STATE, "placement_policy: internal size error");
    for (size_t i = 0; i < H.size(); ++i)
        for (int a = 0; a < 3; ++a) out_active[3 * i + a] = H[i][a];
    *n_out = (int32_t)H.size();
    for (size_t i = 0; i < add.size(); ++i)
        if (added) for (int a = 0; a < 3; ++a) added[3 * i + a] = add[i][a];
    for (size_t i = 0; i < rem.size(); ++i)
        if (removed) for (int a = 0; a < 3; ++a) removed[3 * i + a] = rem[i][a];
    *n_added = (int32_t)add.size();
    *n_removed = (int32_t)rem.size();
    return MVF_OK;
}

// Endpoint counts per cell of the lattice of side d_v - 2 voxels, leaving out
// endpoints inside any of `boxes` (h_t[3], dims[3] each; at most
// kMaxPlaceBoxes).  Synchronises on s.
static mvf_status placement_count_impl(mvf_ctx* c, const mvf_frame* f, const float* T, const mvf_intrinsics* K,
                                       const Grid& g, int d_v, const std::vector<int32_t>& boxes,
                                       std::vector<std::pair<std::vector<int>, int>>* out, hipStream_t s)
{
    if (!c->place_table) {
        CHECK_HIP(hipMalloc((void**)&c->place_table, sizeof(unsigned long long) * 2 * mvf_ctx::kPlaceTable));
        CHECK_HIP(hipMalloc((void**)&c->place_overflow, 256));
        CHECK_HIP(hipMalloc((void**)&c->place_T, 256));
        CHECK_HIP(hipMalloc((void**)&c->place_boxes, sizeof(int32_t) * 6 * mvf_ctx::kMaxPlaceBoxes));
    }
    const int n_boxes = (int)boxes.size() / 6;
    if (n_boxes > mvf_ctx::kMaxPlaceBoxes) return set_error(MVF_ERR_INVALID_ARG, "too many placement boxes");
    const float cell = g.d.voxel_size * (float)(d_v - 2);
    CHECK_HIP(hipMemcpyAsync(c->place_T, T, sizeof(float) * 12, hipMemcpyHostToDevice, s));
    if (n_boxes)
        CHECK_HIP(hipMemcpyAsync(c->place_boxes, boxes.data(), sizeof(int32_t) * boxes.size(), hipMemcpyHostToDevice,
                                 s));
    CHECK_LAUNCH(launch_placement_clear(c->place_table, mvf_ctx::kPlaceTable, s));
    CHECK_HIP(hipMemsetAsync(c->place_overflow, 0, sizeof(int), s));
    CHECK_LAUNCH(launch_placement_count(f->depth, f->depth_pitch ? f->depth_pitch : f->width, f->width, f->height,
                                        K->fx, K->fy, K->cx, K->cy, c->place_T, g.d.origin[0], g.d.origin[1],
                                        g.d.origin[2], cell, c->place_table, mvf_ctx::kPlaceTable,
                                        c->place_overflow, c->place_boxes, n_boxes, g.d.voxel_size, s));
    std::vector<unsigned long long> tab(2 * mvf_ctx::kPlaceTable);
    int ovf = 0;
    CHECK_HIP(hipMemcpyAsync(tab.data(), c->place_table, tab.size() * 8, hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipMemcpyAsync(&ovf, c->place_overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (ovf & 1) return set_error(MVF_ERR_STATE, "more than %d distinct placement cells", mvf_ctx::kPlaceTable);
    if (ovf & 2) return set_error(MVF_ERR_INVALID_ARG, "placement cell index out of range");
    out->clear();
    for (int i = 0; i < mvf_ctx::kPlaceTable; ++i) {
        const unsigned long long key = tab[2 * i];
        if (key == ~0ull) continue;
        const long long nrays = (long long)tab[2 * i + 1];
        std::vector<int> k = { (int)((key >> 42) & 0x1FFFFF) - (1 << 20), (int)((key >> 21) & 0x1FFFFF) - (1 << 20),
                               (int)(key & 0x1FFFFF) - (1 << 20) };
        out->push_back({k, (int)nrays});
    }
    std::sort(out->begin(), out->end());
    return MVF_OK;
}

mvf_status mvf_placement_count(mvf_ctx* c, const mvf_frame* f, const float T_wc[12], const mvf_intrinsics* K,
                               int32_t grid_id, int32_t d_v, int32_t* cells, int32_t* counts, int32_t max_cells,
                               int32_t* n_cells, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    CHECK_ST(check_frame(f));
    if (!T_wc || !finite_pose(T_wc) || !valid_K(K) || !n_cells || max_cells < 0 || (max_cells && (!cells || !counts)))
        return set_error(MVF_ERR_INVALID_ARG, "bad pose, intrinsics or output arrays");
    if (grid_id < 0 || grid_id >= (int32_t)c->grids.size()) return set_error(MVF_ERR_NOT_FOUND, "grid %d", grid_id);
    if (d_v < 3) return set_error(MVF_ERR_INVALID_ARG, "d_v must be >= 3");
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    std::vector<std::pair<std::vector<int>, int>> res;
    CHECK_ST(placement_count_impl(c, f, T_wc, K, c->grids[grid_id], d_v, {}, &res, s));
    *n_cells = (int32_t)res.size();
    for (int i = 0; i < (int)res.size() && i < max_cells; ++i) {
        for (int a = 0; a < 3; ++a) cells[3 * i + a] = res[i].first[a];
        counts[i] = res[i].second;
    }
    return mark_tail(c, s);
}

// Insertion and removal over the classes of p, with the new live cells of
// each class chosen by the built-in rule (custom == null) or by the caller's
// function.
static mvf_status placement_update_impl(mvf_ctx* c, int32_t sid, const mvf_frame* f, const float T_wc[12],
                                        const mvf_intrinsics* K, const mvf_placement_class_params* p,
                                        mvf_placement_fn custom, void* user, mvf_placement_result* r,
                                        void* stream)
{
    if (!c || !p || !r) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    CHECK_ST(check_frame(f));
    if (!T_wc || !finite_pose(T_wc) || !valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "bad pose or intrinsics");
    if (p->grid_id < 0 || p->grid_id >= (int32_t)c->grids.size()) return set_error(MVF_ERR_NOT_FOUND, "grid %d", p->grid_id);
    if (p->n_classes < 1 || p->n_classes > MVF_MAX_PLACEMENT_CLASSES)
        return set_error(MVF_ERR_INVALID_ARG, "n_classes must be in [1, %d]", MVF_MAX_PLACEMENT_CLASSES);
    int quota_sum = 0;
    for (int ci = 0; ci < p->n_classes; ++ci) {
        const mvf_placement_class& pc = p->classes[ci];
        if (pc.d_v < 3 || pc.d_v > 2048) return set_error(MVF_ERR_INVALID_ARG, "class %d: d_v out of range", ci);
        if (pc.quota < 0) return set_error(MVF_ERR_INVALID_ARG, "class %d: negative quota", ci);
        for (int cj = 0; cj < ci; ++cj)
            if (p->classes[cj].d_v == pc.d_v) return set_error(MVF_ERR_INVALID_ARG, "class d_v %d twice", pc.d_v);
        quota_sum += pc.quota;
    }
    if (quota_sum > 64) return set_error(MVF_ERR_INVALID_ARG, "the quotas sum to %d > 64", quota_sum);
    if (!custom && !(p->beta >= 1.0f)) return set_error(MVF_ERR_INVALID_ARG, "beta must be >= 1");
    if (sid < 0) return set_error(MVF_ERR_INVALID_ARG, "stream_id must be >= 0");
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    memset(r, 0, sizeof(*r));
    auto& placed = c->placed[sid];
    // live volumes of the classes already updated this frame: their
    // endpoints are not counted for the later classes
    std::vector<int32_t> boxes;
    std::set<std::vector<int>> cells_seen;
    for (int ci = 0; ci < p->n_classes; ++ci) {
        const int d_v = p->classes[ci].d_v;
        std::vector<std::pair<std::vector<int>, int>> res;
        CHECK_ST(placement_count_impl(c, f, T_wc, K, c->grids[p->grid_id], d_v, boxes, &res, s));
        for (auto& e : res) cells_seen.insert({d_v, e.first[0], e.first[1], e.first[2]});
        std::vector<int32_t> act, cellv, cntv;
        for (auto& kv : placed) {
            if (kv.first[0] != d_v) continue;
            Volume* v = find_volume(c, kv.second);
            if (v && v->active) act.insert(act.end(), kv.first.begin() + 1, kv.first.end());
        }
        for (auto& e : res) {
            cellv.insert(cellv.end(), e.first.begin(), e.first.end());
            cntv.push_back(e.second);
        }
        const int n_act = (int)act.size() / 3;
        const int quota = p->classes[ci].quota;
        std::vector<int32_t> out(3 * std::max(1, std::max(quota, n_act))), add(3 * (n_act + (int)res.size() + 1)),
            rem(3 * (n_act + (int)res.size() + 1));
        int32_t n_out = 0, n_add = 0, n_rem = 0;
        if (!custom) {
            CHECK_ST(mvf_placement_policy(act.data(), n_act, cellv.data(), cntv.data(), (int32_t)res.size(), quota,
                                          p->beta, out.data(), &n_out, add.data(), &n_add, rem.data(), &n_rem));
        } else {
            // the caller's f: the class's live cells after this frame
            std::vector<int32_t> keep(3 * std::max(1, quota));
            int32_t n_keep = -1;
            const int32_t rc = custom(user, ci, d_v, act.data(), n_act, cellv.data(), cntv.data(),
                                      (int32_t)res.size(), quota, keep.data(), &n_keep);
            if (rc != 0) return set_error(MVF_ERR_STATE, "placement function returned %d (class %d)", rc, ci);
            if (n_keep < 0 || n_keep > quota)
                return set_error(MVF_ERR_INVALID_ARG, "placement function kept %d cells, quota %d", n_keep, quota);
            std::set<std::vector<int>> kept, live;
            for (int i = 0; i < n_act; ++i) live.insert({act[3 * i], act[3 * i + 1], act[3 * i + 2]});
            for (int i = 0; i < n_keep; ++i) {
                const std::vector<int> k = { keep[3 * i], keep[3 * i + 1], keep[3 * i + 2] };
                for (int a = 0; a < 3; ++a)
                    if ((int64_t)k[a] * (d_v - 2) < -(1 << 22) || (int64_t)k[a] * (d_v - 2) > (1 << 22))
                        return set_error(MVF_ERR_INVALID_ARG, "placement function kept a cell out of range");
                if (!kept.insert(k).second)
                    return set_error(MVF_ERR_INVALID_ARG, "placement function kept a cell twice");
                for (int a = 0; a < 3; ++a) out[3 * i + a] = k[a];
                if (!live.count(k)) {
                    for (int a = 0; a < 3; ++a) add[3 * n_add + a] = k[a];
                    ++n_add;
                }
            }
            n_out = n_keep;
            for (int i = 0; i < n_act; ++i) {
                const std::vector<int> k = { act[3 * i], act[3 * i + 1], act[3 * i + 2] };
                if (!kept.count(k)) {
                    for (int a = 0; a < 3; ++a) rem[3 * n_rem + a] = k[a];
                    ++n_rem;
                }
            }
        }
        for (int i = 0; i < n_rem; ++i) {
            const std::vector<int> k = { d_v, rem[3 * i], rem[3 * i + 1], rem[3 * i + 2] };
            const int id = placed[k];
            CHECK_ST(mvf_volume_evict(c, id, MVF_EVICT_SWAP_OUT));
            if (r->n_removed < 64) r->removed[r->n_removed++] = id;
        }
        for (int i = 0; i < n_add; ++i) {
            const std::vector<int> k = { d_v, add[3 * i], add[3 * i + 1], add[3 * i + 2] };
            int id;
            auto it = placed.find(k);
            if (it != placed.end() && find_volume(c, it->second)) {
                id = it->second;  // seen before: state kept on the host
            } else {
                mvf_volume_desc d{};
                d.grid_id = p->grid_id;
                for (int a = 0; a < 3; ++a) {
                    d.offset[a] = k[1 + a] * (d_v - 2);
                    d.dims[a] = d_v;
                }
                d.stream_id = sid;
                CHECK_ST(mvf_volume_create(c, &d, &id));
                placed[k] = id;
            }
            CHECK_ST(mvf_volume_place(c, id));
            if (r->n_added < 64) r->added[r->n_added++] = id;
        }
        for (int i = 0; i < n_out; ++i) {
            const int32_t hb[6] = { out[3 * i] * (d_v - 2), out[3 * i + 1] * (d_v - 2), out[3 * i + 2] * (d_v - 2),
                                    d_v, d_v, d_v };
            boxes.insert(boxes.end(), hb, hb + 6);
        }
    }
    r->n_cells = (int32_t)cells_seen.size();
    return mark_tail(c, s);
}

mvf_status mvf_placement_update_classes(mvf_ctx* c, int32_t sid, const mvf_frame* f, const float T_wc[12],
                                        const mvf_intrinsics* K, const mvf_placement_class_params* p,
                                        mvf_placement_result* r, void* stream)
{
    return placement_update_impl(c, sid, f, T_wc, K, p, nullptr, nullptr, r, stream);
}

mvf_status mvf_placement_update_custom(mvf_ctx* c, int32_t sid, const mvf_frame* f, const float T_wc[12],
                                       const mvf_intrinsics* K, const mvf_placement_class_params* p,
                                       mvf_placement_fn fn, void* user, mvf_placement_result* r, void* stream)
{
    if (!fn) return set_error(MVF_ERR_INVALID_ARG, "placement function is NULL");
    return placement_update_impl(c, sid, f, T_wc, K, p, fn, user, r, stream);
}

mvf_status mvf_placement_update(mvf_ctx* c, int32_t sid, const mvf_frame* f, const float T_wc[12],
                                const mvf_intrinsics* K, const mvf_placement_params* p, mvf_placement_result* r,
                                void* stream)
{
    if (!c || !p || !r) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    if (p->n_max < 0 || p->n_max > 64) return set_error(MVF_ERR_INVALID_ARG, "n_max must be in [0, 64]");
    mvf_placement_class_params q{};
    q.grid_id = p->grid_id;
    q.n_classes = 1;
    q.classes[0].d_v = p->d_v;
    q.classes[0].quota = p->n_max;
    q.beta = p->beta;
    return mvf_placement_update_classes(c, sid, f, T_wc, K, &q, r, stream);
}

// ---- checkpoint and resume ---------------------------------------------------------

namespace {
constexpr char kCkptMagic[8] = {'M', 'V', 'F', 'C', 'K', 'P', 'T', 1};
constexpr uint32_t kCkptVersion = 1;

struct CkptVolume {
    int32_t alive, active, has_state, reserved;
    mvf_volume_desc d;
    uint64_t bytes, nbricks;
};

struct CkptPlaced {
    int32_t stream, d_v, cell[3], vol;
};

struct FileCloser {
    FILE* f;
    ~FileCloser() { if (f) fclose(f); }
};
}  // namespace

mvf_status mvf_checkpoint_save(mvf_ctx* c, const char* path)
{
    if (!c || !path) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    CHECK_ST(mvf_synchronize(c));
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) return set_error(MVF_ERR_INVALID_ARG, "cannot open %s for writing", path);
    std::vector<CkptPlaced> placed;
    for (auto& kv : c->placed)
        for (auto& e : kv.second)
            placed.push_back(CkptPlaced{kv.first, e.first[0], {e.first[1], e.first[2], e.first[3]}, e.second});
    const uint32_t hdr[4] = {kCkptVersion, (uint32_t)c->grids.size(), (uint32_t)c->vols.size(),
                             (uint32_t)placed.size()};
    bool ok = fwrite(kCkptMagic, 1, 8, fc.f) == 8 && fwrite(hdr, sizeof(hdr), 1, fc.f) == 1;
    for (const Grid& g : c->grids) ok = ok && fwrite(&g.d, sizeof(g.d), 1, fc.f) == 1;
    std::vector<uint8_t> buf;
    for (const Volume& v : c->vols) {
        CkptVolume cv{};
        cv.alive = v.alive && !v.internal;
        cv.active = v.active;
        cv.has_state = cv.alive && v.state != State::Empty;
        cv.d = v.d;
        cv.bytes = v.bytes;
        cv.nbricks = v.nbricks;
        ok = ok && fwrite(&cv, sizeof(cv), 1, fc.f) == 1;
        if (!cv.has_state || !ok) continue;
        const uint8_t* src = v.host;
        if (v.state == State::Device) {
            buf.resize(v.bytes);
            CHECK_HIP(hipMemcpy(buf.data(), v.dev, v.bytes, hipMemcpyDeviceToHost));
            src = buf.data();
        }
        ok = ok && fwrite(src, 1, v.bytes, fc.f) == v.bytes;
    }
    if (!placed.empty()) ok = ok && fwrite(placed.data(), sizeof(CkptPlaced), placed.size(), fc.f) == placed.size();
    if (!ok) return set_error(MVF_ERR_INVALID_ARG, "writing %s failed", path);
    return MVF_OK;
}

mvf_status mvf_checkpoint_load(mvf_ctx* c, const char* path)
{
    if (!c || !path) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    if (!c->grids.empty() || !c->vols.empty())
        return set_error(MVF_ERR_STATE, "a checkpoint loads into a context without grids or volumes");
    CHECK_HIP(hipSetDevice(c->device));
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) return set_error(MVF_ERR_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    uint32_t hdr[4];
    if (fread(magic, 1, 8, fc.f) != 8 || memcmp(magic, kCkptMagic, 8) != 0 || fread(hdr, sizeof(hdr), 1, fc.f) != 1 ||
        hdr[0] != kCkptVersion || hdr[1] > (1u << 20) || hdr[2] > (1u << 24) || hdr[3] > (1u << 24))
        return set_error(MVF_ERR_INVALID_ARG, "%s is not a checkpoint of this version", path);
    mvf_status st = MVF_OK;
    for (uint32_t i = 0; i < hdr[1] && st == MVF_OK; ++i) {
        mvf_grid_desc d;
        int32_t gid;
        if (fread(&d, sizeof(d), 1, fc.f) != 1) st = set_error(MVF_ERR_INVALID_ARG, "%s: truncated grids", path);
        else st = mvf_grid_create(c, &d, &gid);
    }
    for (uint32_t i = 0; i < hdr[2] && st == MVF_OK; ++i) {
        CkptVolume cv;
        if (fread(&cv, sizeof(cv), 1, fc.f) != 1) { st = set_error(MVF_ERR_INVALID_ARG, "%s: truncated volumes", path); break; }
        if (!cv.alive) {
            c->vols.push_back(Volume());  // keeps the ids of the later volumes
            continue;
        }
        int32_t id;
        st = mvf_volume_create(c, &cv.d, &id);
        if (st != MVF_OK) break;
        Volume& v = c->vols[id];
        if (id != (int32_t)i || v.bytes != cv.bytes || v.nbricks != cv.nbricks) {
            st = set_error(MVF_ERR_INVALID_ARG, "%s: volume %u does not match this library's layout", path, i);
            break;
        }
        v.active = cv.active != 0;
        if (!cv.has_state) continue;
        if (hipHostMalloc((void**)&v.host, v.bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            v.host = nullptr;
            st = set_error(MVF_ERR_OOM, "pinned host memory of %zu bytes", v.bytes);
            break;
        }
        if (fread(v.host, 1, v.bytes, fc.f) != v.bytes) { st = set_error(MVF_ERR_INVALID_ARG, "%s: truncated state", path); break; }
        v.state = State::Host;
        v.host_pending = false;
    }
    for (uint32_t i = 0; i < hdr[3] && st == MVF_OK; ++i) {
        CkptPlaced e;
        if (fread(&e, sizeof(e), 1, fc.f) != 1) { st = set_error(MVF_ERR_INVALID_ARG, "%s: truncated placement", path); break; }
        if (e.vol < 0 || e.vol >= (int32_t)c->vols.size() || !c->vols[e.vol].alive) {
            st = set_error(MVF_ERR_INVALID_ARG, "%s: placement entry names no volume", path);
            break;
        }
        c->placed[e.stream][std::vector<int>{e.d_v, e.cell[0], e.cell[1], e.cell[2]}] = e.vol;
    }
    if (st != MVF_OK) {
        // leave the context empty again
        for (Volume& v : c->vols)
            if (v.host) (void)hipHostFree(v.host);
        c->vols.clear();
        c->grids.clear();
        c->placed.clear();
    }
    return st;
}

// ---- camera tracking ---------------------------------------------------------------

mvf_status mvf_depth_maps(mvf_ctx* c, const mvf_frame* f, const mvf_intrinsics* K, int32_t level, float tau,
                          float smooth, float* V, float* N, void* stream)
{
    if (!c || !V || !N) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    CHECK_ST(check_frame(f));
    if (!valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "intrinsics NULL, not finite or zero focal length");
    if (level < 0 || level > 2) return set_error(MVF_ERR_INVALID_ARG, "level must be in [0, 2]");
    if (!(tau >= 0.0f) || !(smooth >= 0.0f)) return set_error(MVF_ERR_INVALID_ARG, "tau and smooth must be >= 0");
    if ((f->width >> level) < 1 || (f->height >> level) < 1)
        return set_error(MVF_ERR_INVALID_ARG, "image too small for level %d", level);
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    int w = f->width, h = f->height, pitch = f->depth_pitch ? f->depth_pitch : f->width;
    const float* D = f->depth;
    float* tmp[3] = {nullptr, nullptr, nullptr};
    mvf_status st = MVF_OK;
    if (smooth > 0.0f) {
        if (hipMalloc((void**)&tmp[2], sizeof(float) * (size_t)w * h) != hipSuccess) {
            (void)hipGetLastError();
            st = set_error(MVF_ERR_OOM, "smoothed depth");
        } else {
            const int le = launch_track_smooth(D, pitch, w, h, smooth, tmp[2], s);
            if (le) st = set_error(MVF_ERR_HIP, "launch: %s", hipGetErrorString((hipError_t)le));
            D = tmp[2];
            pitch = w;
        }
    }
    for (int l = 1; l <= level && st == MVF_OK; ++l) {
        if (hipMalloc((void**)&tmp[l - 1], sizeof(float) * (size_t)(w / 2) * (h / 2)) != hipSuccess) {
            (void)hipGetLastError();
            st = set_error(MVF_ERR_OOM, "depth pyramid level %d", l);
            break;
        }
        const int le = launch_track_down(D, pitch, w, h, tau, tmp[l - 1], s);
        if (le) st = set_error(MVF_ERR_HIP, "launch: %s", hipGetErrorString((hipError_t)le));
        D = tmp[l - 1];
        w /= 2;
        h /= 2;
        pitch = w;
    }
    if (st == MVF_OK) {
        const float sc = std::ldexp(1.0f, -level);
        const float Kl[4] = { K->fx * sc, K->fy * sc, (K->cx + 0.5f) * sc - 0.5f, (K->cy + 0.5f) * sc - 0.5f };
        const int le = launch_track_vn(D, pitch, w, h, Kl, V, N, s);
        if (le) st = set_error(MVF_ERR_HIP, "launch: %s", hipGetErrorString((hipError_t)le));
    }
    if (tmp[0] || tmp[1] || tmp[2]) {
        const hipError_t e = hipStreamSynchronize(s);
        for (float* t : tmp)
            if (t) (void)hipFree(t);
        if (st == MVF_OK && e != hipSuccess) st = set_error(MVF_ERR_HIP, "%s", hipGetErrorString(e));
    }
    if (st != MVF_OK) return st;
    return mark_tail(c, s);
}

mvf_status mvf_track(mvf_ctx* c, const mvf_frame* f, const mvf_intrinsics* K, const mvf_track_model* m,
                     const double T_init[12], const mvf_track_params* p, double T_out[12], mvf_track_stats* st,
                     void* stream)
{
    if (!c || !m || !p || !T_init || !T_out) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    CHECK_ST(check_frame(f));
    if (!valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "intrinsics NULL, not finite or zero focal length");
    if (!m->vertex || !m->normal) return set_error(MVF_ERR_INVALID_ARG, "model maps NULL");
    if (m->width != f->width || m->height != f->height)
        return set_error(MVF_ERR_INVALID_ARG, "model maps %dx%d differ from the frame %dx%d", m->width, m->height,
                         f->width, f->height);
    if (!finite_pose(m->T_wc)) return set_error(MVF_ERR_INVALID_ARG, "model pose not finite");
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(T_init[i])) return set_error(MVF_ERR_INVALID_ARG, "T_init not finite");
    if (p->levels < 1 || p->levels > 3) return set_error(MVF_ERR_INVALID_ARG, "levels must be in [1, 3]");
    int nsteps = 0;
    for (int l = 0; l < p->levels; ++l) {
        if (p->iters[l] < 0) return set_error(MVF_ERR_INVALID_ARG, "negative iteration count");
        nsteps += p->iters[l];
    }
    if (nsteps > kTrackMaxSteps) return set_error(MVF_ERR_INVALID_ARG, "more than %d steps", kTrackMaxSteps);
    if (!(p->eps_d > 0.0f) || !(p->cos_theta >= 0.0f && p->cos_theta <= 1.0f) || !(p->tau >= 0.0f) ||
        !(p->smooth >= 0.0f))
        return set_error(MVF_ERR_INVALID_ARG, "eps_d > 0, cos_theta in [0, 1], tau >= 0 and smooth >= 0 required");
    if ((f->width >> (p->levels - 1)) < 1 || (f->height >> (p->levels - 1)) < 1)
        return set_error(MVF_ERR_INVALID_ARG, "image too small for %d levels", p->levels);
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    // scratch: per level depth (levels >= 1), current V and N, model V and N
    // (levels >= 1); then the partials and the state
    int w[3], h[3];
    w[0] = f->width;
    h[0] = f->height;
    for (int l = 1; l < 3; ++l) { w[l] = w[l - 1] / 2; h[l] = h[l - 1] / 2; }
    size_t off = 0;
    size_t o_d[3] = {0, 0, 0}, o_v[3], o_n[3], o_vm[3] = {0, 0, 0}, o_nm[3] = {0, 0, 0};
    const size_t o_smooth = off;   // the smoothed full-size depth
    if (p->smooth > 0.0f) off = align_up(off + 4 * (size_t)w[0] * h[0], kAlign);
    for (int l = 0; l < p->levels; ++l) {
        const size_t npx = (size_t)w[l] * h[l];
        if (l) { o_d[l] = off; off = align_up(off + 4 * npx, kAlign); }
        o_v[l] = off; off = align_up(off + 12 * npx, kAlign);
        o_n[l] = off; off = align_up(off + 12 * npx, kAlign);
        if (l) {
            o_vm[l] = off; off = align_up(off + 12 * npx, kAlign);
            o_nm[l] = off; off = align_up(off + 12 * npx, kAlign);
        }
    }
    const size_t o_part = off;
    off = align_up(off + sizeof(double) * kTrackSums * (size_t)track_blocks(w[0], h[0]), kAlign);
    const size_t o_state = off;
    off = align_up(off + sizeof(TrackState), kAlign);
    auto& tk = c->track;
    if (off > tk.bytes) {
        if (tk.dev) {
            CHECK_HIP(hipStreamSynchronize(s));
            CHECK_HIP(hipFree(tk.dev));
            tk.dev = nullptr;
            tk.bytes = 0;
        }
        if (hipMalloc((void**)&tk.dev, off) != hipSuccess) {
            (void)hipGetLastError();
            tk.dev = nullptr;
            return set_error(MVF_ERR_OOM, "tracking scratch of %zu bytes", off);
        }
        tk.bytes = off;
    }
    if (!tk.host) CHECK_HIP(hipHostMalloc((void**)&tk.host, sizeof(TrackState), hipHostMallocDefault));
    uint8_t* B = tk.dev;
    TrackState* dstate = reinterpret_cast<TrackState*>(B + o_state);
    double* partials = reinterpret_cast<double*>(B + o_part);
    for (int i = 0; i < 12; ++i) tk.host->T[i] = T_init[i];
    CHECK_HIP(hipMemcpyAsync(dstate->T, tk.host->T, sizeof(double) * 12, hipMemcpyHostToDevice, s));
    CHECK_LAUNCH(launch_track_init(dstate, s));
    // pyramid and maps
    const float* D[3];
    int pitch[3];
    float Kl[3][4];
    D[0] = f->depth;
    pitch[0] = f->depth_pitch ? f->depth_pitch : f->width;
    if (p->smooth > 0.0f) {
        float* Ds = reinterpret_cast<float*>(B + o_smooth);
        CHECK_LAUNCH(launch_track_smooth(D[0], pitch[0], w[0], h[0], p->smooth, Ds, s));
        D[0] = Ds;
        pitch[0] = w[0];
    }
    for (int l = 0; l < p->levels; ++l) {
        if (l) {
            float* Dl = reinterpret_cast<float*>(B + o_d[l]);
            CHECK_LAUNCH(launch_track_down(D[l - 1], pitch[l - 1], w[l - 1], h[l - 1], p->tau, Dl, s));
            D[l] = Dl;
            pitch[l] = w[l];
        }
        // f / 2^l and (c + 1/2) / 2^l - 1/2 in binary32
        const float sc = std::ldexp(1.0f, -l);
        Kl[l][0] = K->fx * sc;
        Kl[l][1] = K->fy * sc;
        Kl[l][2] = (K->cx + 0.5f) * sc - 0.5f;
        Kl[l][3] = (K->cy + 0.5f) * sc - 0.5f;
        CHECK_LAUNCH(launch_track_vn(D[l], pitch[l], w[l], h[l], Kl[l], reinterpret_cast<float*>(B + o_v[l]),
                                     reinterpret_cast<float*>(B + o_n[l]), s));
    }
    const float* Vm[3];
    const float* Nm[3];
    Vm[0] = m->vertex;
    Nm[0] = m->normal;
    for (int l = 1; l < p->levels; ++l) {
        float* v2 = reinterpret_cast<float*>(B + o_vm[l]);
        float* n2 = reinterpret_cast<float*>(B + o_nm[l]);
        CHECK_LAUNCH(launch_track_model_down(Vm[l - 1], Nm[l - 1], w[l - 1], h[l - 1], v2, n2, s));
        Vm[l] = v2;
        Nm[l] = n2;
    }
    // coarse to fine
    int step = 0;
    for (int l = p->levels - 1; l >= 0; --l) {
        for (int it = 0; it < p->iters[l]; ++it) {
            TrackLaunch L{};
            L.V = reinterpret_cast<const float*>(B + o_v[l]);
            L.N = reinterpret_cast<const float*>(B + o_n[l]);
            L.w = w[l];
            L.h = h[l];
            L.Vm = Vm[l];
            L.Nm = Nm[l];
            L.fx = Kl[l][0];
            L.fy = Kl[l][1];
            L.cx = Kl[l][2];
            L.cy = Kl[l][3];
            for (int i = 0; i < 12; ++i) L.Tm[i] = m->T_wc[i];
            L.eps_d = p->eps_d;
            L.cos_theta = p->cos_theta;
            L.state = dstate;
            L.partials = partials;
            L.inlier = nullptr;
            CHECK_LAUNCH(launch_icp_step(L, dstate, step++, s));
        }
    }
    CHECK_HIP(hipMemcpyAsync(tk.host, dstate, sizeof(TrackState), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < 12; ++i) T_out[i] = tk.host->T[i];
    if (st) {
        memset(st, 0, sizeof(*st));
        st->steps = tk.host->steps;
        for (int i = 0; i < tk.host->steps && i < kTrackMaxSteps; ++i) {
            st->pairs[i] = tk.host->pairs[i];
            st->sq_err[i] = tk.host->sq_err[i];
        }
    }
    return mark_tail(c, s);
}

// ---- differentiable raycast --------------------------------------------------------

static mvf_status diff_volume(mvf_ctx* c, const mvf_dense_tsdf* v, DiffVolume* out)
{
    if (!v || !v->F || !v->W) return set_error(MVF_ERR_INVALID_ARG, "dense volume or its planes NULL");
    for (int a = 0; a < 3; ++a)
        if (v->dims[a] < 2 || v->dims[a] > 4096) return set_error(MVF_ERR_INVALID_ARG, "dense dims out of range");
    if (!(v->voxel_size > 0.0f)) return set_error(MVF_ERR_INVALID_ARG, "voxel_size must be positive");
    out->F = v->F;
    out->W = v->W;
    for (int a = 0; a < 3; ++a) {
        out->dims[a] = v->dims[a];
        out->off[a] = v->offset[a];
        out->o[a] = v->origin[a];
    }
    out->s = v->voxel_size;
    out->inv_s = 1.0f / v->voxel_size;
    (void)c;
    return MVF_OK;
}

// The differentiable forward raycasts a brick-layout mirror of the caller's
// dense volume with the plain raycast (same rules, same exact skipping) and
// records the crossing.  The mirror is an internal volume of the context,
// rebuilt when the dense volume's description changes, on every call with
// generation 0, and when the generation differs from the last build's.
static mvf_status build_diff_mirror(mvf_ctx* c, const mvf_dense_tsdf* v, hipStream_t s)
{
    mvf_ctx::DiffMirror& m = c->diff_mirror;
    const bool same_shape = m.vol >= 0 && m.dims[0] == v->dims[0] && m.dims[1] == v->dims[1] &&
                            m.dims[2] == v->dims[2];
    const bool same = same_shape && m.F == v->F && m.W == v->W && v->generation != 0 &&
                      m.generation == v->generation && m.s == v->voxel_size && m.off[0] == v->offset[0] &&
                      m.off[1] == v->offset[1] && m.off[2] == v->offset[2] && m.o[0] == v->origin[0] &&
                      m.o[1] == v->origin[1] && m.o[2] == v->origin[2];
    if (same) return MVF_OK;
    if (m.grid < 0) {
        mvf_grid_desc gd{};
        gd.voxel_size = v->voxel_size;
        gd.trunc_voxels = 4.0f;  // unused: the raycast reads F in truncation units
        gd.w_max = 65535;
        for (int a = 0; a < 3; ++a) gd.origin[a] = v->origin[a];
        CHECK_ST(mvf_grid_create(c, &gd, &m.grid));
    }
    Grid& g = c->grids[m.grid];
    g.d.voxel_size = v->voxel_size;
    for (int a = 0; a < 3; ++a) g.d.origin[a] = v->origin[a];
    g.mu = g.d.trunc_voxels * g.d.voxel_size;
    g.inv_s = 1.0f / g.d.voxel_size;
    g.inv_mu = 1.0f / g.mu;
    if (!same_shape) {
        if (m.vol >= 0) {
            c->vols[m.vol].internal = false;
            CHECK_ST(mvf_volume_destroy(c, m.vol));
            m.vol = -1;
        }
        mvf_volume_desc d{};
        d.grid_id = m.grid;
        for (int a = 0; a < 3; ++a) d.dims[a] = v->dims[a];
        CHECK_ST(mvf_volume_create(c, &d, &m.vol));
        c->vols[m.vol].internal = true;
    }
    Volume& mv = c->vols[m.vol];
    for (int a = 0; a < 3; ++a) mv.d.offset[a] = v->offset[a];
    m.F = nullptr;  // invalid until the import below is enqueued
    CHECK_ST(ensure_resident(c, std::vector<int>{m.vol}, s));
    CHECK_LAUNCH(launch_from_canonical(make_dev(c, mv), v->F, v->W, nullptr, s));
    CHECK_ST(recompute_summaries(c, mv, s));
    m.F = v->F;
    m.W = v->W;
    m.generation = v->generation;
    m.s = v->voxel_size;
    for (int a = 0; a < 3; ++a) {
        m.dims[a] = v->dims[a];
        m.off[a] = v->offset[a];
        m.o[a] = v->origin[a];
    }
    return MVF_OK;
}

mvf_status mvf_diffray_forward(mvf_ctx* c, const mvf_dense_tsdf* v, const float T_wc[12], const mvf_intrinsics* K,
                               int32_t width, int32_t height, float* depth, int32_t* record, void* stream)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    DiffVolume dv;
    CHECK_ST(diff_volume(c, v, &dv));
    for (int a = 0; a < 3; ++a)
        if (v->dims[a] > 2048) return set_error(MVF_ERR_INVALID_ARG, "dense dims above 2048 (forward)");
    if (!T_wc || !finite_pose(T_wc) || !valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "bad pose or intrinsics");
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384 || !depth || !record)
        return set_error(MVF_ERR_INVALID_ARG, "bad output");
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    CHECK_ST(build_diff_mirror(c, v, s));
    mvf_raycast_out out{};
    out.depth = depth;
    out.width = width;
    out.height = height;
    CHECK_ST(raycast_plain(c, kDiffStream, T_wc, *K, &out, std::vector<int>{c->diff_mirror.vol}, s, record));
    return mark_tail(c, s);
}

// Argument checks shared by the two backward entry points.
static mvf_status diffray_backward_args(mvf_ctx* c, const mvf_dense_tsdf* v, const float T_wc[12],
                                        const mvf_intrinsics* K, int32_t width, int32_t height,
                                        const float* grad_depth, const int32_t* record, const double* grad_xi,
                                        DiffVolume* dv)
{
    if (!c) return set_error(MVF_ERR_INVALID_ARG, "ctx is NULL");
    CHECK_ST(diff_volume(c, v, dv));
    if (!T_wc || !finite_pose(T_wc) || !valid_K(K)) return set_error(MVF_ERR_INVALID_ARG, "bad pose or intrinsics");
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384 || !grad_depth || !record || !grad_xi)
        return set_error(MVF_ERR_INVALID_ARG, "bad gradient buffers");
    return MVF_OK;
}

static RayParams diff_ray_params(mvf_ctx* c, const mvf_dense_tsdf* v)
{
    RayParams rp;
    rp.delta = c->cfg.ray_step * v->voxel_size;
    rp.kmax = (int32_t)std::floor(c->cfg.t_far / rp.delta);
    return rp;
}

mvf_status mvf_diffray_backward(mvf_ctx* c, const mvf_dense_tsdf* v, const float T_wc[12], const mvf_intrinsics* K,
                                int32_t width, int32_t height, const float* grad_depth, const int32_t* record,
                                float* grad_F, double* grad_xi, void* stream)
{
    DiffVolume dv;
    CHECK_ST(diffray_backward_args(c, v, T_wc, K, width, height, grad_depth, record, grad_xi, &dv));
    CHECK_HIP(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    const int need = diffray_partials_needed(width, height);
    if (need > c->diff_partials_n) {
        if (c->diff_partials) {
            CHECK_HIP(hipStreamSynchronize(s));
            CHECK_HIP(hipFree(c->diff_partials));
        }
        CHECK_HIP(hipMalloc((void**)&c->diff_partials, sizeof(double) * 6 * need));
        c->diff_partials_n = need;
    }
    CHECK_LAUNCH(launch_diffray_backward(dv, T_wc, K->fx, K->fy, K->cx, K->cy, width, height, diff_ray_params(c, v),
                                         grad_depth, record, grad_F, c->diff_partials, c->diff_partials_n, grad_xi, s));
    return mark_tail(c, s);
}

mvf_status mvf_diffray_backward_noalloc(mvf_ctx* c, const mvf_dense_tsdf* v, const float T_wc[12],
                                        const mvf_intrinsics* K, int32_t width, int32_t height,
                                        const float* grad_depth, const int32_t* record, float* grad_F,
                                        double* grad_xi, void* stream)
{
    DiffVolume dv;
    CHECK_ST(diffray_backward_args(c, v, T_wc, K, width, height, grad_depth, record, grad_xi, &dv));
    const int need = diffray_partials_needed(width, height);
    if (need > kDiffScratchBlocks)
        return set_error(MVF_ERR_INVALID_ARG,
                         "a %dx%d image needs %d partial blocks of 16x16 pixels; the static scratch holds %d",
                         width, height, need, kDiffScratchBlocks);
    CHECK_HIP(hipSetDevice(c->device));
    double* partials = diffray_scratch(c->device);
    if (!partials) return set_error(MVF_ERR_STATE, "static scratch of device %d not set up", c->device);
    hipStream_t s = (hipStream_t)stream;
    CHECK_ST(order_after_previous(c, s));
    CHECK_LAUNCH(launch_diffray_backward(dv, T_wc, K->fx, K->fy, K->cx, K->cy, width, height, diff_ray_params(c, v),
                                         grad_depth, record, grad_F, partials, kDiffScratchBlocks, grad_xi, s));
    return mark_tail(c, s);
}

mvf_status mvf_pose_retract(const double T[12], const double xi[6], double T_out[12])
{
    if (!T || !xi || !T_out) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    const double* rho = xi;
    const double* w = xi + 3;
    const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double Wx[9] = { 0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0 };
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += Wx[3 * i + k] * Wx[3 * k + j];
            W2[3 * i + j] = acc;
        }
    double A, B, C;
    if (th < 1e-10) {
        A = 1.0; B = 0.5; C = 1.0 / 6.0;
    } else {
        A = std::sin(th) / th;
        B = (1.0 - std::cos(th)) / (th * th);
        C = (th - std::sin(th)) / (th * th * th);
    }
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * Wx[i] + B * W2[i];
        V[i] = I + B * Wx[i] + C * W2[i];
    }
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = V[3 * i] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
    double out[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            out[4 * i + j] = T[4 * i] * R[j] + T[4 * i + 1] * R[3 + j] + T[4 * i + 2] * R[6 + j];
        out[4 * i + 3] = T[4 * i] * t[0] + T[4 * i + 1] * t[1] + T[4 * i + 2] * t[2] + T[4 * i + 3];
    }
    memcpy(T_out, out, sizeof(out));
    return MVF_OK;
}

// Right Jacobian of Exp on SE(3) with xi = (rho, omega): Exp(xi + d) =
// Exp(xi) Exp(J d) to first order in d.  J_r(xi) is the left Jacobian at
// -xi, [[J(w), Q(rho, w)], [0, J(w)]] with J the SO(3) left Jacobian
// (the V of Exp) and Q the closed-form coupling block (Barfoot, State
// Estimation for Robotics, SE(3) kinematics); series below 1e-2 rad.
mvf_status mvf_pose_right_jacobian(const double xi[6], double J_out[36])
{
    if (!xi || !J_out) return set_error(MVF_ERR_INVALID_ARG, "NULL argument");
    double r[3], w[3];
    for (int i = 0; i < 3; ++i) {
        r[i] = -xi[i];
        w[i] = -xi[3 + i];
    }
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = std::sqrt(th2);
    double b1, a1, a2, a3;
    if (th < 1e-2) {
        const double t4 = th2 * th2;
        b1 = 0.5 - th2 / 24.0 + t4 / 720.0;
        a1 = 1.0 / 6.0 - th2 / 120.0 + t4 / 5040.0;
        a2 = 1.0 / 24.0 - th2 / 720.0 + t4 / 40320.0;
        a3 = 1.0 / 120.0 - th2 / 2520.0;
    } else {
        const double sn = std::sin(th), cs = std::cos(th);
        b1 = (1.0 - cs) / th2;
        a1 = (th - sn) / (th2 * th);
        a2 = (th2 + 2.0 * cs - 2.0) / (2.0 * th2 * th2);
        a3 = (2.0 * th - 3.0 * sn + th * cs) / (2.0 * th2 * th2 * th);
    }
    typedef double M3[9];
    auto hat = [](const double v[3], double* m) {
        const double t[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
        memcpy(m, t, sizeof(t));
    };
    auto mul = [](const double* a, const double* b, double* out) {
        double t[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) t[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
        memcpy(out, t, sizeof(t));
    };
    M3 W, P, WW, WP, PW, WPW, WWP, PWW, WPWW, WWPW, Jw, Q;
    hat(w, W);
    hat(r, P);
    mul(W, W, WW);
    mul(W, P, WP);
    mul(P, W, PW);
    mul(WP, W, WPW);
    mul(WW, P, WWP);
    mul(P, WW, PWW);
    mul(WPW, W, WPWW);
    mul(WW, PW, WWPW);
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        Jw[i] = I + b1 * W[i] + a1 * WW[i];
        Q[i] = 0.5 * P[i] + a1 * (WP[i] + PW[i] + WPW[i]) + a2 * (WWP[i] + PWW[i] - 3.0 * WPW[i]) +
               a3 * (WPWW[i] + WWPW[i]);
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double v = 0.0;
            if (i < 3 && j < 3) v = Jw[3 * i + j];
            else if (i < 3) v = Q[3 * i + (j - 3)];
            else if (j >= 3) v = Jw[3 * (i - 3) + (j - 3)];
            J_out[6 * i + j] = v;
        }
    return MVF_OK;
}

}  // extern "C"
