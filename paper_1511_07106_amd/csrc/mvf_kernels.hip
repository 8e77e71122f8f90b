// HIP kernels for gfx950 (MI355X): TSDF integration, multi-volume raycast,
// brick summaries, layout conversion, placement counting, differentiable
// raycast.  Built with -ffp-contract=off and IEEE division/sqrt so the
// decision path reproduces the binary32 contract of the CPU reference
// bit for bit.  Paper: Salvato, Finman, Leonard, arXiv 1511.07106.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "mvf_internal.h"
#include "mvf_masks.h"

namespace mvf {

static __host__ __device__ __forceinline__ float qnan() { return __builtin_nanf(""); }
static __host__ __device__ __forceinline__ float pinf() { return __builtin_inff(); }

// Pointers into global memory.  Volume and frame pointers reach the kernels
// through tables in memory, so the compiler cannot infer their address space
// and would emit flat accesses; the cast makes them global accesses.
#if defined(__HIP_DEVICE_COMPILE__)
#define GPTR(T) __attribute__((address_space(1))) T*
template <class T>
static __device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}
#else
#define GPTR(T) T*
template <class T>
static __host__ __device__ inline T* gptr(T* p) { return p; }
#endif

// Read-only tables written before the launch (volume, frame and z tables):
// in the constant address space a load with a wave-uniform address becomes
// a scalar load.
#if defined(__HIP_DEVICE_COMPILE__)
#define CPTR(T) const __attribute__((address_space(4))) T*
template <class T>
static __device__ __forceinline__ const __attribute__((address_space(4))) T* cptr(const T* p)
{
    return (const __attribute__((address_space(4))) T*)p;
}
#else
#define CPTR(T) const T*
template <class T>
static __host__ __device__ inline const T* cptr(const T* p) { return p; }
#endif

static __device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

static __host__ __device__ __forceinline__ size_t brick_index(const int bd[3], int bx, int by, int bz) {
    return ((size_t)bx * bd[1] + by) * bd[2] + bz;
}

// ---------------------------------------------------------------------------
// Frame preparation: per pixel the range R = D * lambda along the pixel ray
// (lambda = |K^-1 [u v 1]|, the same binary32 operations the voxel test
// uses), 0 for an invalid depth; packed RGB; the frame's maximum range.
// The range map holds one more element, range[W * H] = 0, read by voxels
// that project outside the image.  The maximum range is reduced from
// per-block maxima by the z-table kernel, which runs before integration.
// In a captured step the items are read from the step's pinned host slot,
// and every thread of the launch also copies one 16-byte word of the slot's
// table image to the tables' device home (tsrc, tdst: n16 words), which the
// later kernels of the step read.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mvf_frame_prep_kernel(const PrepItem* __restrict__ items, const uint4* tsrc,
                                                             uint4* tdst, uint32_t n16)
{
    if (tsrc) {
        const uint32_t nt = gridDim.x * gridDim.y * gridDim.z * 256u;
        const uint32_t t = ((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 256u + threadIdx.x;
        for (uint32_t i = t; i < n16; i += nt) tdst[i] = tsrc[i];
    }
    const PrepItem& it = items[blockIdx.z];
    const int u = blockIdx.x * 32 + (threadIdx.x & 31);
    const int v = blockIdx.y * 8 + (threadIdx.x >> 5);
    float R = 0.0f;
    if (u < it.width && v < it.height) {
        const float Dz = it.depth[(size_t)v * it.depth_pitch + u];
        if (Dz > 0.0f && Dz < INFINITY) {
            const float a = ((float)u - it.cx) / it.fx;
            const float b = ((float)v - it.cy) / it.fy;
            const float lam = sqrtf(((a * a) + (b * b)) + 1.0f);
            R = Dz * lam;
        }
        it.range[(size_t)v * it.width + u] = R;
        uint32_t c = 0;
        if (it.rgb) {
            const uint8_t* q = it.rgb + (size_t)v * it.rgb_pitch + 3 * u;
            c = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16);
        }
        it.color[(size_t)v * it.width + u] = c;
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
        it.range[(size_t)it.width * it.height] = 0.0f;
    // maxima and minima of the block's four 8x8 tiles: a wavefront holds
    // two rows of 32 pixels, a tile's part of it is 8 consecutive lanes in
    // each half (pixels outside the image count as range 0)
    float tm = R, tn = R;
    for (int o = 1; o <= 4; o <<= 1) {
        tm = fmaxf(tm, __shfl_xor(tm, o));
        tn = fminf(tn, __shfl_xor(tn, o));
    }
    tm = fmaxf(tm, __shfl_xor(tm, 32));
    tn = fminf(tn, __shfl_xor(tn, 32));
    // block maximum into this block's slot; the z-table kernel reduces the
    // slots (no atomics on one address)
    float m = tm;
    for (int o = 8; o <= 16; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    __shared__ float wmax[4];
    __shared__ float tw[4][4], tnw[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wmax[wv] = m;
    if (lane < 32 && (lane & 7) == 0) {
        tw[wv][lane >> 3] = tm;
        tnw[wv][lane >> 3] = tn;
    }
    __syncthreads();
    const int gx = (it.width + 31) / 32, gy = (it.height + 7) / 8;
    if (threadIdx.x == 0 && (int)blockIdx.x < gx && (int)blockIdx.y < gy) {
        m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        it.rmax[1 + blockIdx.y * gx + blockIdx.x] = m;
    }
    const int tiles_x = (it.width + 7) / 8;
    const int tx = (int)blockIdx.x * 4 + (int)threadIdx.x;
    if (it.tmax && threadIdx.x < 4 && tx < tiles_x && (int)blockIdx.y < gy) {
        const int t = threadIdx.x;
        it.tmax[blockIdx.y * tiles_x + tx] = fmaxf(fmaxf(tw[0][t], tw[1][t]), fmaxf(tw[2][t], tw[3][t]));
        // the minima follow the maxima (tiles_x * tiles_y of each)
        it.tmax[(size_t)tiles_x * gy + blockIdx.y * tiles_x + tx] =
            fminf(fminf(tnw[0][t], tnw[1][t]), fminf(tnw[2][t], tnw[3][t]));
    }
}

int launch_frame_prep(const PrepItem* items, int n, int max_w, int max_h, void* stream, const void* tsrc,
                      void* tdst, size_t tbytes)
{
    if (n <= 0) return 0;
    if (tsrc && ((tbytes & 15) || ((uintptr_t)tsrc & 15) || ((uintptr_t)tdst & 15))) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((max_w + 31) / 32, (max_h + 7) / 8, n);
    hipLaunchKernelGGL(mvf_frame_prep_kernel, grid, dim3(256), 0, s, items, (const uint4*)tsrc, (uint4*)tdst,
                       (uint32_t)(tsrc ? tbytes / 16 : 0));
    return (int)hipGetLastError();
}

int set_frame_prep_node(void* exec, void* node, const PrepItem* items, int n, int max_w, int max_h, const void* tsrc,
                        void* tdst, size_t tbytes)
{
    if (n <= 0 || !tsrc || (tbytes & 15) || ((uintptr_t)tsrc & 15) || ((uintptr_t)tdst & 15))
        return (int)hipErrorInvalidValue;
    const PrepItem* a0 = items;
    const uint4* a1 = (const uint4*)tsrc;
    uint4* a2 = (uint4*)tdst;
    uint32_t a3 = (uint32_t)(tbytes / 16);
    void* args[] = {(void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3};
    hipKernelNodeParams p{};
    p.func = reinterpret_cast<void*>(mvf_frame_prep_kernel);
    p.gridDim = dim3((max_w + 31) / 32, (max_h + 7) / 8, n);
    p.blockDim = dim3(256);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return (int)hipGraphExecKernelNodeSetParams((hipGraphExec_t)exec, (hipGraphNode_t)node, &p);
}

// ---------------------------------------------------------------------------
// Volume initialisation: F = NaN (unobserved), W = 0, C = 0, flags = 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mvf_volume_init_kernel(DevVolume v, size_t nvox, size_t nbricks)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t ncolw = (size_t)v.bd[0] * v.bd[1] * col_words(v.bd[2]);  // <= nbricks
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvox; i += stride) {
        v.F[i] = __uint_as_float(0x7fc00000u);
        v.W[i] = 0;
        v.C[i] = 0;
        if (i < nbricks) {
            v.flag[i] = 0;
            v.dist[i] = kDistCap;
            v.fmask[i] = 0;
            v.cmask[i] = 0;
        }
        if (i <= ncolw) v.colm[i] = 0;  // word ncolw stays zero (read for absent neighbours)
    }
}

int launch_volume_init(DevVolume v, void* stream)
{
    const size_t nb = (size_t)v.bd[0] * v.bd[1] * v.bd[2];
    const size_t nvox = nb * kBrickVox;
    int blocks = (int)((nvox + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(mvf_volume_init_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, v,
                       nvox, nb);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch order of the raycast tile groups: counting sort of their summed
// last durations, longest first, by half octaves (the leading two bits).
// Run by one block of any size: each thread takes kOrderBatch groups per
// round with all their loads in flight, and counts and places them with
// LDS atomics (aggregating a wavefront's lanes per bin with ballots first
// serialised the block: up to ~90 us per order in the integration launch's
// block 0, longer than the integration it runs beside).  The cost array holds
// ray_groups(n) * kRayGroup entries (zero past n).
constexpr int kOrderBins = 64;
constexpr int kOrderBatch = 4;

static __device__ __forceinline__ int cost_bin(uint4 c)
{
    const uint64_t t = (uint64_t)c.x + c.y + c.z + c.w;
    if (t < 2) return (int)t;
    const int e = 63 - __clzll(t);
    return min(2 * e + (int)((t >> (e - 1)) & 1), kOrderBins - 1);
}

static __device__ void tile_order_block(const uint32_t* __restrict__ cost, int32_t* __restrict__ order, int ntiles,
                                        int* hist)
{
    static_assert(kRayGroup == 4, "one uint4 of costs per group");
    const int ng = ray_groups(ntiles);
    const int nt = blockDim.x;
    const uint4* c4 = reinterpret_cast<const uint4*>(cost);
    for (int i = threadIdx.x; i < kOrderBins; i += nt) hist[i] = 0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int g0 = 0; g0 < ng; g0 += kOrderBatch * nt) {
            uint4 c[kOrderBatch];
#pragma unroll
            for (int k = 0; k < kOrderBatch; ++k) {
                const int g = g0 + k * nt + (int)threadIdx.x;
                c[k] = g < ng ? c4[g] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < kOrderBatch; ++k) {
                const int g = g0 + k * nt + (int)threadIdx.x;
                if (g >= ng) continue;
                const int bin = cost_bin(c[k]);
                // the place within a bin is the atomics' order (the launch
                // order only steers the timing)
                if (pass == 0) atomicAdd(&hist[bin], 1);
                else order[atomicAdd(&hist[bin], 1)] = g;
            }
        }
        __syncthreads();
        if (pass == 0 && threadIdx.x == 0) {
            // start of each bin, longest first
            int acc = 0;
            for (int b = kOrderBins - 1; b >= 0; --b) {
                const int h = hist[b];
                hist[b] = acc;
                acc += h;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Integration.  A wavefront owns the 8x8 voxel columns of a brick and walks
// its 8 z-slices; each lane is one column (Volumetric Integration section:
// one thread per (x, y), iterating z).  A z-slice of a brick is 64
// consecutive voxels, so every load/store of the wave is one contiguous
// 256-byte (F, C) or 128-byte (W) access.  The visit pass before the launch
// lists the bricks to decide voxel by voxel and the "deep" ones, updated
// wholesale with phi = 1; a conservative per-column z interval (frustum,
// near plane, farthest range of the frame) masks lanes, and the exact
// binary32 test decides every voxel of a visited brick.
//
// Per voxel the work is the projection (one division), a gather of the
// measured range, a square root and the running average.  The camera-frame
// offset of each z, the same for all lanes, comes from a table computed by
// a small kernel before the launch (scalar loads).  The square root uses
// the hardware estimate and takes the correctly rounded value only in lanes
// where the estimate lies within its error bound of the truncation band:
// elsewhere the update test, the band test and the stored value (phi = 1,
// or no update) do not depend on which of the two roots is used.
// ---------------------------------------------------------------------------

// n / d for n < 2^17 and 1 <= d <= 256 exactly: a quotient from the
// reciprocal estimate, then one correction step each way.
static __device__ __forceinline__ uint32_t udiv_small(uint32_t n, uint32_t d, float rd)
{
    int q = (int)((float)n * rd);
    int r = (int)n - q * (int)d;
    q += (r >= (int)d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return (uint32_t)q;
}

// Conservative interval of local z (inclusive lo, exclusive hi) for which a
// voxel of this column can pass the exact test.  Each condition is a
// half-line a + b z >= 0 of the affine camera-frame position p(z); margins
// (1 px, 1 mm, 2 voxels, and 1-2 voxels on the bound itself) dominate the
// binary32 rounding of the exact test and the 2^-22 relative error of the
// estimated quotient; a bound beyond the volume is clamped away.
static __device__ __forceinline__ void clip_halfline(float a, float b, float& zl, float& zh)
{
    if (b > 0.0f) {
        zl = fmaxf(zl, -a * __builtin_amdgcn_rcpf(b) - 1.0f);
    } else if (b < 0.0f) {
        zh = fminf(zh, -a * __builtin_amdgcn_rcpf(b) + 2.0f);
    } else if (a < 0.0f) {
        zh = -1e30f;
    }
}

// The flags of brick (bxi, byi, bz) after an update that may have written
// F <= 2^-100 in the lanes with flag_here (fz: per pair of z-slices).
static __device__ __forceinline__ void mark_brick(const DevVolume& V, int bxi, int byi, int bz, bool flag_here,
                                                  const bool (&fz)[kBrick / 2], int lane)
{
    if (__ballot(flag_here) != 0) {
        uint64_t fm = 0;
#pragma unroll
        for (int zp = 0; zp < kBrick / 2; ++zp)
            fm |= (uint64_t)subblock_bits(__ballot(fz[zp])) << (16 * zp);
        if (lane == 0) {
            const size_t b = brick_index(V.bd, bxi, byi, bz);
            V.flag[b] = 1;
            atomicOr((unsigned long long*)&V.fmask[b], (unsigned long long)fm);
            const size_t cw = (size_t)(bxi * V.bd[1] + byi) * col_words(V.bd[2]) + (bz >> 6);
            atomicOr((unsigned long long*)&V.colm[cw], 1ull << (bz & 63));
        }
    }
}

// NB deep bricks (entries e = item * 8 + j of the deep list: brick j of the
// item; e < 0 for none): the visit pass proved R - rho > mu for every voxel,
// so each voxel inside the volume is updated with phi = 1 and none is in the
// colour band; neither the projection nor the range gathers are needed.
// The F and W loads of all NB bricks (3 KB each) are issued before any is
// used: two bricks a wavefront were 3 % faster than one on the large room
// (more bytes in flight per wave slot), four spilled scalar registers.
template <int NB>
static __device__ __forceinline__ void integrate_deep_bricks(const IntegrateLaunch& L, const int (&es)[NB], int zchunk,
                                                             int nvol, int lane, unsigned& n_upd)
{
    CPTR(int32_t) const item_base = cptr(L.item_base);
    int vi[NB], bxi[NB], byi[NB], bzv[NB];
    size_t base[NB];
    bool uv[NB][kBrick];
    float Fo[NB][kBrick];
    uint16_t Wo[NB][kBrick];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int e = es[b] < 0 ? 0 : es[b];
        const int item = e >> 3, j = e & 7;
        int lo = 0, hi = nvol - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_base[mid] <= item) lo = mid; else hi = mid - 1;
        }
        lo = wave_uniform(lo);
        vi[b] = lo;
        const DevVolume& V = cptr(L.vols)[lo];
        const int local = item - item_base[lo];
        const int ncols = V.bd[0] * V.bd[1];
        const int zc = local / ncols;
        const int col = local - zc * ncols;
        byi[b] = col / V.bd[0];
        bxi[b] = col - byi[b] * V.bd[0];
        bzv[b] = zc * zchunk + j;
        const int x = bxi[b] * kBrick + (lane & 7);
        const int y = byi[b] * kBrick + (lane >> 3);
        const bool col_ok = es[b] >= 0 && x < V.dims[0] && y < V.dims[1];
        const int nz_here = min(kBrick, V.dims[2] - bzv[b] * kBrick);
        base[b] = brick_index(V.bd, bxi[b], byi[b], bzv[b]) * kBrickVox + lane;
        GPTR(float) const pF = gptr(V.F) + base[b];
        GPTR(uint16_t) const pW = gptr(V.W) + base[b];
#pragma unroll
        for (int zz = 0; zz < kBrick; ++zz) {
            uv[b][zz] = col_ok & (zz < nz_here);
            Fo[b][zz] = 0.0f;
            Wo[b][zz] = 0;
            if (uv[b][zz]) {
                Fo[b][zz] = __builtin_nontemporal_load(&pF[zz * 64]);
                Wo[b][zz] = __builtin_nontemporal_load(&pW[zz * 64]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const DevVolume V = cptr(L.vols)[vi[b]];
        GPTR(float) const pF = gptr(V.F) + base[b];
        GPTR(uint16_t) const pW = gptr(V.W) + base[b];
        bool flag_here = false;
        bool fz[kBrick / 2] = {false, false, false, false};
#pragma unroll
        for (int zz = 0; zz < kBrick; ++zz) {
            n_upd += (unsigned)__popcll(__ballot(uv[b][zz]));
            const int w = Wo[b][zz];
            const float Wf = (float)w;
            const float den = Wf + 1.0f;
            float r = __builtin_amdgcn_rcpf(den);
            r = fmaf(r, fmaf(-den, r, 1.0f), r);
            const float Fn = (w == 0) ? 1.0f : fmaf(Fo[b][zz], Wf, 1.0f) * r;
            if (uv[b][zz]) {
                pF[zz * 64] = Fn;
                pW[zz * 64] = (uint16_t)min(w + 1, V.w_max);
            }
            const bool fl = uv[b][zz] & (Fn <= kFlagThreshold);
            flag_here |= fl;
            fz[zz >> 1] |= fl;
        }
        if (es[b] >= 0) mark_brick(V, bxi[b], byi[b], bzv[b], flag_here, fz, lane);
    }
}

// eight wavefronts per SIMD: the kernel is latency-bound, and its state fits 64 VGPRs
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void mvf_integrate_kernel(IntegrateLaunch L)
{
    // with a tile order to compute (captured step), block 0 sorts the next
    // raycast's tile groups while the others integrate
    const int b0 = L.tile_order ? 1 : 0;
    if ((int)blockIdx.x < b0) {
        __shared__ int hist[kOrderBins];
        tile_order_block(L.tile_cost, L.tile_order, L.order_tiles, hist);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int total_waves = ((int)gridDim.x - b0) * wpb;
    unsigned n_upd = 0, n_band = 0, n_brk = 0, n_deep = 0;  // wave totals
    const int nvol = L.hdr->nvol;
    const int zchunk = L.hdr->zchunk;
    CPTR(float) const ztab = cptr(L.ztab);
    // with a list, every brick to visit voxel by voxel gets a wavefront, and
    // the deep bricks come after them (a wavefront per visited brick: items
    // of several visited bricks, walked by one wavefront, were the launch's
    // longest waves)
    const unsigned long long lc = L.list ? cptr(L.list_count)[L.hdr->list_parity] : 0ull;
    // visited bricks (or, without a list, items), then deep bricks
    const int n_vis = L.list ? (int)(lc & 0xffffffffull) : L.hdr->total_items;
    // deep bricks two to a wavefront when the grid covers all the work in
    // one pass (large room: 3 % faster), else one (a full-frustum frame,
    // where every wavefront walks several deep bricks anyway: pairs were
    // 2.5 % slower there)
    constexpr int kDeepPerWave = 2;
    const int n_deep_all = (int)(lc >> 32);
    const int per = (n_vis + n_deep_all <= total_waves) ? kDeepPerWave : 1;
    const int n_work = n_vis + (n_deep_all + per - 1) / per;

    for (int w = wave_uniform(((int)blockIdx.x - b0) * wpb + wib); w < n_work; w += total_waves) {
        if (w >= n_vis) {
            const int m = per * (w - n_vis);
            int es[kDeepPerWave];
#pragma unroll
            for (int b = 0; b < kDeepPerWave; ++b) es[b] = b < per && m + b < n_deep_all ? cptr(L.deep_list)[m + b] : -1;
            integrate_deep_bricks<kDeepPerWave>(L, es, zchunk, nvol, lane, n_upd);
#pragma unroll
            for (int b = 0; b < kDeepPerWave; ++b) n_deep += es[b] >= 0 ? 1 : 0;
            continue;
        }
        // brick j0 of the item from a list entry, else the whole item
        const int e = L.list ? cptr(L.list)[w] : 0;
        const int item = L.list ? e >> 3 : w;
        const int j0 = L.list ? e & 7 : 0;
        const int j1 = L.list ? j0 + 1 : zchunk;
        // bricks of the item that may hold an updated voxel (bytes from
        // zchunk on are not written by the visit pass)
        const uint64_t vis = L.visit ? cptr((const uint64_t*)L.visit)[item] &
                                           (zchunk >= kVisitPerItem ? ~0ull : (1ull << (8 * zchunk)) - 1ull)
                                     : 0x0101010101010101ull;
        if (vis == 0) continue;
        // volume owning this item
        CPTR(int32_t) const item_base = cptr(L.item_base);
        int lo = 0, hi = nvol - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_base[mid] <= item) lo = mid; else hi = mid - 1;
        }
        lo = wave_uniform(lo);
        const DevVolume V = cptr(L.vols)[lo];
        const int local = item - item_base[lo];
        const int ncols = V.bd[0] * V.bd[1];
        const int zc = local / ncols;
        const int col = local - zc * ncols;
        const int byi = col / V.bd[0];
        const int bxi = col - byi * V.bd[0];
        const int bz0 = zc * zchunk;
        const int bz1 = min(bz0 + zchunk, V.bd[2]);

        // frame parameters, held in registers for the whole item
        CPTR(DevFrame) const Fp = cptr(L.frames) + V.frame;
        GPTR(const float) const range = gptr(Fp->range);
        GPTR(const uint32_t) const color = gptr(Fp->color);
        const float rmax = *Fp->rmax;
        const float T0 = Fp->T[0], T1 = Fp->T[1], T2 = Fp->T[2], T3 = Fp->T[3];
        const float T4 = Fp->T[4], T5 = Fp->T[5], T6 = Fp->T[6], T7 = Fp->T[7];
        const float T8 = Fp->T[8], T9 = Fp->T[9], T10 = Fp->T[10], T11 = Fp->T[11];
        const float fx = Fp->fx, fy = Fp->fy, cx = Fp->cx, cy = Fp->cy;
        const int W = Fp->width, H = Fp->height;
        const float fW = (float)W, fH = (float)H;
        const float fW1 = (float)(W - 1), fH1 = (float)(H - 1);
        const uint32_t npix = (uint32_t)W * (uint32_t)H;  // index of the zero range
        const bool has_color = Fp->color != nullptr;
        GPTR(float) vF = gptr(V.F);
        GPTR(uint16_t) vW = gptr(V.W);
        GPTR(uint32_t) vC = gptr(V.C);

        const int x = bxi * kBrick + (lane & 7);
        const int y = byi * kBrick + (lane >> 3);
        const bool col_ok = x < V.dims[0] && y < V.dims[1];
        // column constants of the binary32 contract
        const float xw_x = V.o[0] + (V.s * ((float)(V.off[0] + x) + 0.5f));
        const float xw_y = V.o[1] + (V.s * ((float)(V.off[1] + y) + 0.5f));
        const float dx = xw_x - T3;
        const float dy = xw_y - T7;
        const float Px = (T0 * dx) + (T4 * dy);
        const float Py = (T1 * dx) + (T5 * dy);
        const float Pz = (T2 * dx) + (T6 * dy);

        // conservative z interval of this column
        float zl = (float)(bz0 * kBrick), zh = (float)min(bz1 * kBrick, V.dims[2]);
        {
            const float A = (V.o[2] + V.s * ((float)V.off[2] + 0.5f)) - T11;
            const float ax = Px + T8 * A, bx = T8 * V.s;
            const float ay = Py + T9 * A, by = T9 * V.s;
            const float az = Pz + T10 * A, bzc = T10 * V.s;
            const float E = 1e-3f;
            clip_halfline(az + 2.0f * V.s, bzc, zl, zh);
            clip_halfline(fx * ax + (cx + 1.5f) * az + fx * E, fx * bx + (cx + 1.5f) * bzc, zl, zh);
            clip_halfline(-fx * ax + (fW + 0.5f - cx) * az + fx * E, -fx * bx + (fW + 0.5f - cx) * bzc, zl, zh);
            clip_halfline(fy * ay + (cy + 1.5f) * az + fy * E, fy * by + (cy + 1.5f) * bzc, zl, zh);
            clip_halfline(-fy * ay + (fH + 0.5f - cy) * az + fy * E, -fy * by + (fH + 0.5f - cy) * bzc, zl, zh);
            const float rfar = rmax + V.mu + 2.0f * V.s;
            clip_halfline(rfar - az, -bzc, zl, zh);
        }
        int zlo = (int)fmaxf(zl, -1.0f), zhi = (int)fminf(fmaxf(zh, -1.0f), 1e8f);
        if (!col_ok) { zlo = 0; zhi = 0; }
        zlo = max(zlo, bz0 * kBrick);
        zhi = min(zhi, min(bz1 * kBrick, V.dims[2]));
        // threshold of the square-root filter: the estimate is within 2 ulp
        // of the correctly rounded root (within 2^-48 below 2^-96); 8 ulp of
        // margin plus the absolute term cover both roundings of sdf
        const float mu_f = V.mu + 0x1p-46f;

        const size_t colbase = brick_index(V.bd, bxi, byi, 0) * kBrickVox + lane;
        for (int bz = bz0 + j0; bz < min(bz0 + j1, bz1); ++bz) {
            const int zb = bz * kBrick;
            const bool mine = zlo < zb + kBrick && zhi > zb;
            if (!((vis >> (8 * (bz - bz0))) & 1ull) || __ballot(mine) == 0) continue;
            const size_t base = colbase + (size_t)bz * kBrickVox;
            GPTR(float) const pF = vF + base;
            GPTR(uint16_t) const pW = vW + base;
            // a deep brick has a wavefront of its own (integrate_deep_brick)
            if ((vis >> (8 * (bz - bz0) + 1)) & 1ull) continue;
            // the brick's 8 z-table entries, one scalar block
            struct ZRow { float v[3 * kBrick]; };
            const ZRow zr = *(CPTR(ZRow))(ztab + 3 * (V.zt_base + zb));
            const int nz_here = min(kBrick, V.dims[2] - zb);
            ++n_brk;
            // phase 1: camera-frame position and nearest pixel of 8 voxels.
            // The pixel coordinates are clamped into the image (a NaN goes
            // to 0); the voxel projects into the image iff clamping left them
            // unchanged.  A voxel that does not reads the zero range behind
            // the image, so R > 0 below carries the projection test.
            float rho2v[kBrick], Rv[kBrick];
#pragma unroll
            for (int zz = 0; zz < kBrick; ++zz) {
                const float px = Px + zr.v[3 * zz];
                const float py = Py + zr.v[3 * zz + 1];
                const float pz = Pz + zr.v[3 * zz + 2];
                const float iz = 1.0f / pz;
                const float uf = ((fx * px) * iz) + cx;
                const float vf = ((fy * py) * iz) + cy;
                const float ur = floorf(uf + 0.5f);
                const float vr = floorf(vf + 0.5f);
                const float uc = __builtin_amdgcn_fmed3f(ur, 0.0f, fW1);
                const float vc = __builtin_amdgcn_fmed3f(vr, 0.0f, fH1);
                const bool ok = col_ok & (zz < nz_here) & (pz > 0.0f) & (uc == ur) & (vc == vr);
                rho2v[zz] = ((px * px) + (py * py)) + (pz * pz);
                const uint32_t pix = ok ? __umul24((uint32_t)vc, (uint32_t)W) + (uint32_t)uc : npix;
                Rv[zz] = *(GPTR(const float))((GPTR(const uint8_t))range + (pix << 2));
            }
            // phase 2: projective signed distance and the truncation test
            float sdfv[kBrick];
            bool nearv[kBrick];
            bool any_near = false;
#pragma unroll
            for (int zz = 0; zz < kBrick; ++zz) {
                const float rho = __builtin_amdgcn_sqrtf(rho2v[zz]);
                const float sdf = Rv[zz] - rho;
                sdfv[zz] = sdf;
                nearv[zz] = !(fabsf(sdf) > fmaf(rho, 0x1p-20f, mu_f));
                any_near |= nearv[zz];
            }
            if (__ballot(any_near) != 0) {
#pragma unroll
                for (int zz = 0; zz < kBrick; ++zz)
                    if (nearv[zz]) sdfv[zz] = Rv[zz] - sqrtf(rho2v[zz]);
            }
            bool updv[kBrick], bandv[kBrick];
            bool any_upd = false, any_band = false;
#pragma unroll
            for (int zz = 0; zz < kBrick; ++zz) {
                const float sdf = sdfv[zz];
                updv[zz] = (Rv[zz] > 0.0f) & !(sdf < -V.mu);
                bandv[zz] = updv[zz] & (sdf <= V.mu);
                n_upd += (unsigned)__popcll(__ballot(updv[zz]));
                n_band += (unsigned)__popcll(__ballot(bandv[zz]));
                any_upd |= updv[zz];
                any_band |= bandv[zz];
            }
            if (__ballot(any_upd) == 0) continue;
            // phase 3: running average (value path) and weights; F and W are
            // read only in the lanes that update them
            float Fo[kBrick];
            uint16_t Wo[kBrick];
#pragma unroll
            for (int zz = 0; zz < kBrick; ++zz) {
                Fo[zz] = 0.0f;
                Wo[zz] = 0;
                if (updv[zz]) {
                    Fo[zz] = __builtin_nontemporal_load(&pF[zz * 64]);
                    Wo[zz] = __builtin_nontemporal_load(&pW[zz * 64]);
                }
            }
            bool flag_here = false;
            bool fz[kBrick / 2] = {false, false, false, false};
#pragma unroll
            for (int zz = 0; zz < kBrick; ++zz) {
                const float phi = fminf(1.0f, sdfv[zz] * V.inv_mu);
                const int w = Wo[zz];
                const float Wf = (float)w;
                // reciprocal of (W + 1) by the hardware estimate refined with
                // one Newton step (error ~1 ulp)
                const float den = Wf + 1.0f;
                float r = __builtin_amdgcn_rcpf(den);
                r = fmaf(r, fmaf(-den, r, 1.0f), r);
                const float Fn = (w == 0) ? phi : fmaf(Fo[zz], Wf, phi) * r;
                // plain (cache-allocating) stores: the raycast that follows
                // reads the updated surface band
                if (updv[zz]) {
                    pF[zz * 64] = Fn;
                    pW[zz * 64] = (uint16_t)min(w + 1, V.w_max);
                }
                const bool fl = updv[zz] & (Fn <= kFlagThreshold);
                flag_here |= fl;
                fz[zz >> 1] |= fl;
            }
            // phase 4: colour in the band |sdf| <= mu (rounded running mean)
            if (has_color && __ballot(any_band) != 0) {
#pragma unroll
                for (int zz = 0; zz < kBrick; ++zz) {
                    if (bandv[zz]) {
                        // the voxel's pixel again (band voxels are few)
                        const float xw_z = V.o[2] + (V.s * ((float)(V.off[2] + zb + zz) + 0.5f));
                        const float dz = xw_z - T11;
                        const float px = Px + (T8 * dz);
                        const float py = Py + (T9 * dz);
                        const float pz = Pz + (T10 * dz);
                        const float iz = 1.0f / pz;
                        const float ur = floorf((((fx * px) * iz) + cx) + 0.5f);
                        const float vr = floorf((((fy * py) * iz) + cy) + 0.5f);
                        const size_t i = base + zz * 64;
                        const uint32_t obs = color[__umul24((uint32_t)vr, (uint32_t)W) + (uint32_t)ur];
                        const uint32_t c = vC[i];
                        const uint32_t Aw = c >> 24;
                        const uint32_t d = Aw + 1u;
                        const float rd = __builtin_amdgcn_rcpf((float)d);
                        const uint32_t half = d >> 1;
                        const uint32_t r = udiv_small((c & 255u) * Aw + (obs & 255u) + half, d, rd);
                        const uint32_t g = udiv_small(((c >> 8) & 255u) * Aw + ((obs >> 8) & 255u) + half, d, rd);
                        const uint32_t b = udiv_small(((c >> 16) & 255u) * Aw + ((obs >> 16) & 255u) + half, d, rd);
                        const uint32_t An = Aw + 1u < 255u ? Aw + 1u : 255u;
                        vC[i] = r | (g << 8) | (b << 16) | (An << 24);
                    }
                }
            }
            mark_brick(V, bxi, byi, bz, flag_here, fz, lane);
        }
    }
    // counters: the wave's totals (the same in every lane), one atomic each
    // into one of kCntSlots copies; no block barrier, so a wavefront that
    // finishes early frees its slot at once
    if (lane == 0 && L.counters && (n_upd | n_band | n_brk | n_deep)) {
        unsigned long long* slot = L.counters + ((((int)blockIdx.x - b0) * wpb + wib) % kCntSlots) * kCntNum;
        if (n_upd) atomicAdd(&slot[kCntUpdated], (unsigned long long)n_upd);
        if (n_band) atomicAdd(&slot[kCntBand], (unsigned long long)n_band);
        if (n_brk) atomicAdd(&slot[kCntBricks], (unsigned long long)n_brk);
        if (n_deep) atomicAdd(&slot[kCntDeep], (unsigned long long)n_deep);
    }
}

// Class of brick [lo, hi] (the box of its voxel centres, world frame) for
// the frame: 0 when no voxel of it can be updated, 2 when every voxel of it
// inside the volume is updated with phi = 1 and lies outside the colour band
// ("deep": in front of the measured surface by more than mu everywhere),
// else 1 (visited, decided voxel by voxel).
// - 0: the box projects outside the image, or the pixels it projects to
//   hold no measurement, or every voxel centre lies farther from the camera
//   than mu beyond the largest range of those pixels (then R - rho < -mu).
// - 2: the box lies in front of the camera and its projection, grown by a
//   pixel, inside the image, so every voxel's nearest pixel is in the image
//   and among the tiles read; those tiles hold valid ranges only, and their
//   smallest range exceeds the farthest voxel distance by more than mu.
//   Then R - rho > mu for every voxel: the update test passes, phi = 1 and
//   the band test fails, whatever the voxel.
// The pixels are bounded by the 8x8 tiles (maxima and minima of the range)
// under the projected box grown by one pixel (at most 4x4 tiles are read; a
// larger footprint is class 1); margins of 1e-4 m plus 1e-5 of the distance
// cover the binary32 rounding of the voxel test.
static __device__ int brick_class(const DevVolume& V, const DevFrame& Fr, const float lo[3], const float hi[3])
{
    const float c[3] = {Fr.T[3], Fr.T[7], Fr.T[11]};
    float d2 = 0.0f, d2f = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float e = fmaxf(fmaxf(lo[a] - c[a], c[a] - hi[a]), 0.0f);
        const float f = fmaxf(fabsf(lo[a] - c[a]), fabsf(hi[a] - c[a]));
        d2 += e * e;
        d2f += f * f;
    }
    const float dmin = sqrtf(d2) * (1.0f - 1e-5f) - 1e-4f;
    if (!(dmin > V.mu)) return 1;
    {
        // cheap rejection of a box wholly outside the view (most bricks of a
        // volume): the largest value over the box of each side plane's
        // linear form, the planes one pixel beyond the image; a box with a
        // negative maximum (by a margin far above the rounding) projects
        // nowhere into the image, and one wholly behind the camera holds no
        // voxel with pz > 0
        float cw[3], ew[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cw[a] = 0.5f * (lo[a] + hi[a]) - c[a];
            ew[a] = 0.5f * (hi[a] - lo[a]);
        }
        const float* T = Fr.T;
        const float pcx = T[0] * cw[0] + T[4] * cw[1] + T[8] * cw[2];
        const float pcy = T[1] * cw[0] + T[5] * cw[1] + T[9] * cw[2];
        const float pcz = T[2] * cw[0] + T[6] * cw[1] + T[10] * cw[2];
        const float ecz = fabsf(T[2]) * ew[0] + fabsf(T[6]) * ew[1] + fabsf(T[10]) * ew[2];
        if (pcz + ecz < -1e-3f) return 0;
        // the side planes pass through the camera centre: a point with pz > 0
        // projects inside the grown image iff all four forms are >= 0, so the
        // test also holds for a box across the camera plane (around a camera
        // inside the volume; such boxes were all visited before, and most of
        // them have no column in the view)
        const float A[4] = {Fr.fx, -Fr.fx, 0.0f, 0.0f};
        const float B[4] = {0.0f, 0.0f, Fr.fy, -Fr.fy};
        const float Cc[4] = {Fr.cx + 1.5f, (float)Fr.width + 0.5f - Fr.cx, Fr.cy + 1.5f,
                             (float)Fr.height + 0.5f - Fr.cy};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float Lc = A[q] * pcx + B[q] * pcy + Cc[q] * pcz;
            float Le = 0.0f;
#pragma unroll
            for (int b = 0; b < 3; ++b)
                Le += fabsf(A[q] * T[4 * b] + B[q] * T[4 * b + 1] + Cc[q] * T[4 * b + 2]) * ew[b];
            const float margin = 1e-4f * (fabsf(A[q]) + fabsf(B[q]) + fabsf(Cc[q])) * (fabsf(pcz) + ecz + 1.0f);
            if (Lc + Le < -margin) return 0;
        }
    }
    float u0 = INFINITY, u1 = -INFINITY, v0 = INFINITY, v1 = -INFINITY;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float dx = ((k & 1) ? hi[0] : lo[0]) - c[0];
        const float dy = ((k & 2) ? hi[1] : lo[1]) - c[1];
        const float dz = ((k & 4) ? hi[2] : lo[2]) - c[2];
        const float px = Fr.T[0] * dx + Fr.T[4] * dy + Fr.T[8] * dz;
        const float py = Fr.T[1] * dx + Fr.T[5] * dy + Fr.T[9] * dz;
        const float pz = Fr.T[2] * dx + Fr.T[6] * dy + Fr.T[10] * dz;
        if (!(pz > 0.01f)) return 1;
        const float iz = __builtin_amdgcn_rcpf(pz);  // relative error 2^-22: far inside the margin
        const float u = Fr.fx * px * iz + Fr.cx;
        const float v = Fr.fy * py * iz + Fr.cy;
        u0 = fminf(u0, u); u1 = fmaxf(u1, u);
        v0 = fminf(v0, v); v1 = fmaxf(v1, v);
    }
    const float g0 = floorf(u0 - 0.5f), g1 = floorf(u1 + 1.5f);
    const float h0 = floorf(v0 - 0.5f), h1 = floorf(v1 + 1.5f);
    const bool inside = g0 >= 0.0f && g1 <= (float)(Fr.width - 1) && h0 >= 0.0f && h1 <= (float)(Fr.height - 1);
    const float a0 = fmaxf(g0, 0.0f), a1 = fminf(g1, (float)(Fr.width - 1));
    const float b0 = fmaxf(h0, 0.0f), b1 = fminf(h1, (float)(Fr.height - 1));
    if (!(a0 <= a1 && b0 <= b1)) return 0;  // outside the image
    const int ta0 = (int)a0 >> 3, tb0 = (int)b0 >> 3;
    const int nx = ((int)a1 >> 3) - ta0 + 1, ny = ((int)b1 >> 3) - tb0 + 1;
    if (nx > 4 || ny > 4) return 1;
    const float* tmin = Fr.tmax + (size_t)Fr.tiles_x * Fr.tiles_y;
    // 16 tiles, each index clamped into the nx x ny rectangle (repeats of its
    // tiles leave the maximum and minimum as they are): the loads carry no
    // condition, so all of them are in flight at once
    float tx[16], tn[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int t = (tb0 + min(k >> 2, ny - 1)) * Fr.tiles_x + ta0 + min(k & 3, nx - 1);
        tx[k] = Fr.tmax[t];
        tn[k] = tmin[t];
    }
    float mR = 0.0f, mn = INFINITY;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        mR = fmaxf(mR, tx[k]);
        mn = fminf(mn, tn[k]);
    }
    if (mR == 0.0f) return 0;  // no measurement under the brick
    if (dmin > mR + V.mu) return 0;
    const float dmax = sqrtf(d2f) * (1.0f + 1e-5f) + 1e-4f;
    if (inside && mn - dmax > V.mu * (1.0f + 1e-5f) + 1e-4f) return 2;
    return 1;
}

// Blocks [0, kZtBlocks): the z table of every volume of the launch (see
// IntegrateLaunch) and each frame's maximum range from the frame-preparation
// block maxima.  Blocks beyond: the items' brick visit masks.
constexpr int kZtBlocks = 16;
// visited items a z-table block holds in LDS before appending them
constexpr int kZtListBuf = 1024;
// most blocks of the visit pass (each appends its bricks with one atomic per
// flush): one brick per thread up to 1M bricks (the 32-room workload's 73
// volumes: 90 us of visit pass with 512 blocks, each thread walking about
// eleven bricks in turn)
constexpr int kZtCullBlocksMax = 2048;
// threads of a z-table launch's blocks: a visit block of 512 threads takes one
// brick per thread on a 512^3 volume (10.7 us per frame on the large room,
// against 13.2 us with 256 threads and two bricks each, 11.4 with 1024)
constexpr int kZtThreads = 512;

__global__ __launch_bounds__(kZtThreads) void mvf_ztable_kernel(IntegrateLaunch L)
{
    const LaunchHeader* hdr = L.hdr;
    const DevVolume* vols = L.vols;
    const DevFrame* frames = L.frames;
    const int nvol = hdr->nvol;
    if (blockIdx.x >= kZtBlocks) {
        // one thread per brick of an item (zchunk per item; the item's
        // bytes from zchunk on are never read)
        const int zchunk = hdr->zchunk;
        const int total = hdr->total_items * zchunk;
        const int stride = (gridDim.x - kZtBlocks) * blockDim.x;
        const int lane = threadIdx.x & 63;
        const int wib = threadIdx.x >> 6;
        // the block's visited and deep bricks, gathered in LDS over its
        // iterations and appended with one counter atomic per flush: one
        // atomic per wavefront on a single address serialised in the L2 and
        // cost ~20 us per frame
        __shared__ int32_t blk_items[kZtListBuf];
        __shared__ int32_t blk_deep[kZtListBuf];
        __shared__ int blk_n, blk_base, blk_dn, blk_dbase;
        __shared__ int wave_n[kZtThreads / 64], wave_dn[kZtThreads / 64];
        if (threadIdx.x == 0) {
            blk_n = 0;
            blk_dn = 0;
        }
        __syncthreads();
        auto flush = [&]() {
            if (threadIdx.x == 0) {
                // both counts in one 64-bit word: one atomic per flush
                const unsigned long long add = (unsigned long long)blk_n | ((unsigned long long)blk_dn << 32);
                const unsigned long long old = add ? atomicAdd(&L.list_count[L.hdr->list_parity], add) : 0ull;
                blk_base = (int)(old & 0xffffffffull);
                blk_dbase = (int)(old >> 32);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < blk_n; i += blockDim.x) L.list[blk_base + i] = blk_items[i];
            for (int i = threadIdx.x; i < blk_dn; i += blockDim.x) L.deep_list[blk_dbase + i] = blk_deep[i];
            __syncthreads();
            if (threadIdx.x == 0) {
                blk_n = 0;
                blk_dn = 0;
            }
            __syncthreads();
        };
        for (int t0 = (blockIdx.x - kZtBlocks) * blockDim.x; t0 < total; t0 += stride) {
            const int t = min(t0 + (int)threadIdx.x, total - 1);
            const int item = t / zchunk, j = t - item * zchunk;
            int lo = 0, hi = nvol - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.item_base[mid] <= item) lo = mid; else hi = mid - 1;
            }
            auto test = [&](const DevVolume& V, const DevFrame& Fr) -> int {
                const int local = item - L.item_base[lo];
                const int ncols = V.bd[0] * V.bd[1];
                const int zc = local / ncols;
                const int col = local - zc * ncols;
                const int byi = col / V.bd[0];
                const int bxi = col - byi * V.bd[0];
                const int bz = zc * zchunk + j;
                if (bz >= V.bd[2]) return 0;
                if (!Fr.tmax) return 1;
                const int i0[3] = {bxi * kBrick, byi * kBrick, bz * kBrick};
                float blo[3], bhi[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int i1 = min(i0[a] + kBrick - 1, V.dims[a] - 1);
                    blo[a] = V.o[a] + (V.s * ((float)(V.off[a] + i0[a]) + 0.5f));
                    bhi[a] = V.o[a] + (V.s * ((float)(V.off[a] + i1) + 0.5f));
                }
                return brick_class(V, Fr, blo, bhi);
            };
            // a wavefront whose bricks share one volume reads the volume
            // and frame tables with scalar loads
            const int lo0 = wave_uniform(lo);
            int cls;
            if (__ballot(lo != lo0) == 0) {
                const DevVolume V = cptr(vols)[lo0];
                cls = test(V, cptr(frames)[V.frame]);
            } else {
                cls = test(vols[lo], frames[vols[lo].frame]);
            }
            // deep bricks get wavefronts of their own only with the lists
            const bool deep = cls == 2 && L.list != nullptr;
            const bool visit = cls != 0;
            const bool valid = t0 + (int)threadIdx.x < total;
            // byte: bit 0 visit, bit 1 deep (done by a wavefront of its own)
            if (valid) L.visit[(size_t)item * kVisitPerItem + j] = deep ? 3 : (visit ? 1 : 0);
            if (L.list) {
                // the bricks of this wavefront to visit voxel by voxel, and
                // the deep ones, each in brick order within the block
                const bool proj = valid && visit && !deep;
                const uint64_t hm = __ballot(proj);
                const uint64_t dm = __ballot(valid && deep);
                if (lane == 0) {
                    wave_n[wib] = (int)__popcll(hm);
                    wave_dn[wib] = (int)__popcll(dm);
                }
                __syncthreads();
                int off = blk_n, sum = 0, doff = blk_dn, dsum = 0;
                for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                    if (w < wib) {
                        off += wave_n[w];
                        doff += wave_dn[w];
                    }
                    sum += wave_n[w];
                    dsum += wave_dn[w];
                }
                const uint64_t below = (1ull << lane) - 1ull;
                if (proj) blk_items[off + __popcll(hm & below)] = item * 8 + j;
                if (valid && deep) blk_deep[doff + __popcll(dm & below)] = item * 8 + j;
                __syncthreads();
                if (threadIdx.x == 0) {
                    blk_n += sum;
                    blk_dn += dsum;
                }
                __syncthreads();
                // room for the next iteration's entries (at most one per thread)
                if (blk_n + (int)blockDim.x > kZtListBuf || blk_dn + (int)blockDim.x > kZtListBuf) flush();
            }
        }
        if (L.list) flush();
        return;
    }
    // the other count, for the next launch (the previous one, which used it,
    // has finished)
    if (L.list_count && blockIdx.x == 0 && threadIdx.x == 0) L.list_count[L.hdr->list_parity ^ 1] = 0ull;
    const int total = hdr->total_z;
    for (int f = blockIdx.x; f < hdr->nstreams; f += kZtBlocks) {
        float* rm = frames[f].rmax;
        if (!rm) continue;
        const int np = frames[f].rmax_parts;
        float m = 0.0f;
        for (int j = threadIdx.x; j < np; j += blockDim.x) m = fmaxf(m, rm[1 + j]);
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        __shared__ float wmax[kZtThreads / 64];
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            float mm = 0.0f;
            for (int q = 0; q < kZtThreads / 64; ++q) mm = fmaxf(mm, wmax[q]);
            rm[0] = mm;
        }
        __syncthreads();
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += kZtBlocks * blockDim.x) {
        int lo = 0, hi = nvol - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (vols[mid].zt_base <= i) lo = mid; else hi = mid - 1;
        }
        const DevVolume& V = vols[lo];
        const DevFrame& Fr = frames[V.frame];
        const int z = i - V.zt_base;
        const float xw_z = V.o[2] + (V.s * ((float)(V.off[2] + z) + 0.5f));
        const float dz = xw_z - Fr.T[11];
        L.ztab[3 * i] = Fr.T[8] * dz;
        L.ztab[3 * i + 1] = Fr.T[9] * dz;
        L.ztab[3 * i + 2] = Fr.T[10] * dz;
    }
}

int launch_ztable(const IntegrateLaunch& L, int bricks, void* stream)
{
    const int need = (bricks + kZtThreads - 1) / kZtThreads;
    const int cb = need < 1 ? 1 : (need > kZtCullBlocksMax ? kZtCullBlocksMax : need);
    const int blocks = kZtBlocks + (L.visit ? cb : 0);
    hipLaunchKernelGGL(mvf_ztable_kernel, dim3(blocks), dim3(kZtThreads), 0, (hipStream_t)stream, L);
    return (int)hipGetLastError();
}

int launch_integrate(const IntegrateLaunch& L, int blocks, void* stream, void* ev_start, void* ev_stop)
{
    if (blocks <= 0) return 0;
    if (ev_start)
        hipExtLaunchKernelGGL(mvf_integrate_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                              (hipEvent_t)ev_start, (hipEvent_t)ev_stop, 0, L);
    else
        hipLaunchKernelGGL(mvf_integrate_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, L);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Raycast.  One thread per pixel; a one-wavefront block covers an 8x8 pixel
// tile of coherent rays (a free wave slot is refilled as soon as any ray
// tile finishes); tiles are assigned so that neighbouring tiles land on the
// same XCD (shared L2 for the voxels they gather).  Each ray walks the global sample lattice t_k = k delta through
// every volume of its stream (nearest first), skipping runs of samples
// whose cell lies in bricks flagged "no F <= 0" (exact: such samples can
// never be the far end of a plus-to-minus crossing), and keeps the nearest
// crossing over all volumes.
// ---------------------------------------------------------------------------
static __host__ __device__ __forceinline__ float lerp32(float a, float b, float t) { return (a * (1.0f - t)) + (b * t); }

struct Ray {
    float C[3];
    float dw[3];
    float inv_dw[3];   // approximate 1/dw (conservative uses only)
    float inv_delta;   // approximate 1/delta
    float t_lo, t_hi;  // every sample that may end a crossing lies in [t_lo, t_hi]
};

static __host__ __device__ __forceinline__ float approx_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// local continuous voxel coordinate of sample k in volume V (binary32 contract)
static __host__ __device__ __forceinline__ void sample_coord(const DevVolume& V, const Ray& r, float tk, float l[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = r.C[a] + (tk * r.dw[a]);
        const float c = ((x - V.o[a]) * V.inv_s) - 0.5f;
        l[a] = c - (float)V.off[a];
    }
}

static __host__ __device__ __forceinline__ bool in_domain(const DevVolume& V, const float l[3])
{
    return l[0] >= 0.0f && l[0] < (float)(V.dims[0] - 1) && l[1] >= 0.0f &&
           l[1] < (float)(V.dims[1] - 1) && l[2] >= 0.0f && l[2] < (float)(V.dims[2] - 1);
}

// 32-bit brick-linear addressing: a volume holds at most 2^30 padded
// voxels, so element and byte offsets of its planes fit in 32 bits.
static __host__ __device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return a * b;
#endif
}

static __host__ __device__ __forceinline__ uint32_t brick_index32(const DevVolume& V, int bx, int by, int bz)
{
    return mul24(mul24((uint32_t)bx, (uint32_t)V.bd[1]) + (uint32_t)by, (uint32_t)V.bd[2]) + (uint32_t)bz;
}

static __host__ __device__ __forceinline__ uint32_t voxel_index32(const DevVolume& V, const int i[3])
{
    return brick_index32(V, i[0] >> 3, i[1] >> 3, i[2] >> 3) * (uint32_t)kBrickVox +
           (uint32_t)(((i[2] & 7) << 6) | ((i[1] & 7) << 3) | (i[0] & 7));
}

// element e of a plane, addressed as base + 32-bit byte offset
template <class T>
static __host__ __device__ __forceinline__ T ld_elem(GPTR(const T) base, uint32_t e)
{
    return *(GPTR(const T))((GPTR(const uint8_t))base + e * (uint32_t)sizeof(T));
}

// 8 corner values of the cell with base i (brick-linear addressing)
static __host__ __device__ __forceinline__ void gather8(const DevVolume& V, const int i[3], float c[8])
{
    const uint32_t base = voxel_index32(V, i);
    const uint32_t sx = ((i[0] & 7) == 7) ? (uint32_t)V.bd[1] * (uint32_t)V.bd[2] * kBrickVox - 7u : 1u;
    const uint32_t sy = ((i[1] & 7) == 7) ? (uint32_t)V.bd[2] * kBrickVox - 56u : 8u;
    const uint32_t sz = ((i[2] & 7) == 7) ? (uint32_t)(kBrickVox - 448) : 64u;
    GPTR(const float) const F = gptr((const float*)V.F);
    c[0] = ld_elem(F, base);
    c[1] = ld_elem(F, base + sx);
    c[2] = ld_elem(F, base + sy);
    c[3] = ld_elem(F, base + sy + sx);
    c[4] = ld_elem(F, base + sz);
    c[5] = ld_elem(F, base + sz + sx);
    c[6] = ld_elem(F, base + sz + sy);
    c[7] = ld_elem(F, base + sz + sy + sx);
}

// trilinear value in the contract's order (x, then y, then z); NaN when a
// corner is unobserved
static __host__ __device__ __forceinline__ float trilinear(const float c[8], const float f[3])
{
    const float c00 = lerp32(c[0], c[1], f[0]);
    const float c10 = lerp32(c[2], c[3], f[0]);
    const float c01 = lerp32(c[4], c[5], f[0]);
    const float c11 = lerp32(c[6], c[7], f[0]);
    const float c0 = lerp32(c00, c10, f[1]);
    const float c1 = lerp32(c01, c11, f[1]);
    return lerp32(c0, c1, f[2]);
}

// The 8 corner values of the last cell gathered by a ray; consecutive
// samples half a voxel apart often share a cell.
struct CellCache {
    int i[3];
    float c[8];
};

static __host__ __device__ __forceinline__ bool eval_sample_cached(const DevVolume& V, const float l[3], float& Fk,
                                                                   CellCache& cc)
{
    int i[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float fl = floorf(l[a]);
        i[a] = (int)fl;
        f[a] = l[a] - fl;
    }
    if (i[0] != cc.i[0] || i[1] != cc.i[1] || i[2] != cc.i[2]) {
        gather8(V, i, cc.c);
        cc.i[0] = i[0];
        cc.i[1] = i[1];
        cc.i[2] = i[2];
    }
    Fk = trilinear(cc.c, f);
    return !isnan(Fk);
}

// Conservative sample range [k0, k1] of the ray inside V's domain box grown
// by one voxel, plus two samples each side.
// Raycast range bounds.  Every sample the march must evaluate (a possible
// far end of a crossing) lies in a cell with a corner that may hold F <= 0:
// a cell whose base voxel lies in a sub-block set in its brick's cell mask,
// at local coordinates in [8 b + 2 s0, 8 b + 2 s1 + 2) along each axis for
// the set sub-blocks s0 .. s1 (the near end of a crossing is one sample
// before; rays keep two samples of margin).  Each brick with a non-empty
// cell mask records the distance range of that box (grown by 0.1 voxel)
// from the camera centre and the 8x8-pixel cells its projection can reach
// (grown by one pixel; all cells when the box reaches behind the camera); a
// merge folds these footprints into per-cell ranges, and a ray marches only
// within the range of its cell (a cell no brick reaches is empty).
static __device__ bool brick_footprint(const DevVolume& V, const DevFrame& Fr, int bx, int by, int bz, uint64_t cm,
                                       RayBoundEntry& e)
{
    const int ib[3] = {bx, by, bz};
    const float c[3] = {Fr.T[3], Fr.T[7], Fr.T[11]};
    // the box of the cell mask's sub-blocks (cm != 0), in voxel-centre
    // coordinates
    const uint32_t occ[3] = {occupancy_x(cm), occupancy_y(cm), occupancy_z(cm)};
    float lo[3], hi[3];
    float dn2 = 0.0f, df2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s0 = __builtin_ctz(occ[a]), s1 = 31 - __builtin_clz(occ[a]);
        lo[a] = V.o[a] + V.s * ((float)(V.off[a] + kBrick * ib[a] + 2 * s0) + 0.4f);
        hi[a] = V.o[a] + V.s * ((float)(V.off[a] + kBrick * ib[a] + 2 * s1 + 2) + 0.6f);
        const float en = fmaxf(fmaxf(lo[a] - c[a], c[a] - hi[a]), 0.0f);
        const float ef = fmaxf(fabsf(lo[a] - c[a]), fabsf(hi[a] - c[a]));
        dn2 += en * en;
        df2 += ef * ef;
    }
    e.dn = fmaxf(sqrtf(dn2) * (1.0f - 1e-5f) - 1e-4f, 0.0f);
    e.df = sqrtf(df2) * (1.0f + 1e-5f) + 1e-4f;
    float u0 = INFINITY, u1 = -INFINITY, v0 = INFINITY, v1 = -INFINITY;
    bool behind = false, front = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float dx = ((k & 1) ? hi[0] : lo[0]) - c[0];
        const float dy = ((k & 2) ? hi[1] : lo[1]) - c[1];
        const float dz = ((k & 4) ? hi[2] : lo[2]) - c[2];
        const float px = Fr.T[0] * dx + Fr.T[4] * dy + Fr.T[8] * dz;
        const float py = Fr.T[1] * dx + Fr.T[5] * dy + Fr.T[9] * dz;
        const float pz = Fr.T[2] * dx + Fr.T[6] * dy + Fr.T[10] * dz;
        behind |= !(pz > 1e-3f);
        front |= pz > -1e-3f;
        const float iz = __builtin_amdgcn_rcpf(pz);
        const float u = Fr.fx * px * iz + Fr.cx;
        const float v = Fr.fy * py * iz + Fr.cy;
        u0 = fminf(u0, u); u1 = fmaxf(u1, u);
        v0 = fminf(v0, v); v1 = fmaxf(v1, v);
    }
    // every ray sample lies in front of the camera (z > 0): a box wholly
    // behind it is seen by no ray, one across the camera plane by any
    if (!front) return false;
    if (behind) {
        e.x0 = 0; e.x1 = (uint16_t)(Fr.cells_x - 1);
        e.y0 = 0; e.y1 = (uint16_t)(Fr.cells_y - 1);
        return true;
    }
    const float a0 = fmaxf(floorf(u0 - 1.0f), 0.0f), a1 = fminf(ceilf(u1 + 1.0f), (float)(Fr.out_w - 1));
    const float b0 = fmaxf(floorf(v0 - 1.0f), 0.0f), b1 = fminf(ceilf(v1 + 1.0f), (float)(Fr.out_h - 1));
    if (!(a0 <= a1 && b0 <= b1)) return false;   // no pixel of the image sees the box
    e.x0 = (uint16_t)((int)a0 / kBoundCell); e.x1 = (uint16_t)((int)a1 / kBoundCell);
    e.y0 = (uint16_t)((int)b0 / kBoundCell); e.y1 = (uint16_t)((int)b1 / kBoundCell);
    return true;
}

// Footprint of brick (bx, by, bz) of volume v appended to the volume's list
// (if its cell mask is not empty).  Called by every active lane of a
// wavefront whose lanes all serve volume v; one counter atomic per wavefront.
static __device__ void collect_footprint(const DevVolume& V, const DevFrame& Fr, int v, uint64_t cm, int bx, int by,
                                         int bz, const int32_t* brick_base, const LaunchHeader* hdr, RayBounds rb)
{
    RayBoundEntry e;
    const bool has = Fr.rb_lo && cm != 0ull && brick_footprint(V, Fr, bx, by, bz, cm, e);
    const unsigned long long m = __ballot(has);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll(m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&rb.counts[hdr->rb_parity * rb.cap + v], (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    if (has) rb.entries[brick_base[v] + base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = e;
}

static __host__ __device__ __forceinline__ void ray_k_range(const DevVolume& V, const Ray& r, float delta, int kmax,
                                                   int& k0, int& k1)
{
    float t0 = fmaxf(0.0f, r.t_lo), t1 = fminf((float)kmax * delta, r.t_hi);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = V.o[a] + V.s * ((float)V.off[a] + 0.5f) - V.s;
        const float hi = V.o[a] + V.s * ((float)V.off[a] + (float)V.dims[a] - 0.5f) + V.s;
        if (r.dw[a] == 0.0f) {
            if (r.C[a] < lo || r.C[a] > hi) { k0 = 1; k1 = 0; return; }
        } else {
            // approximate reciprocal: the range is grown by a voxel and two
            // samples, far beyond its rounding error
            float ta = (lo - r.C[a]) * r.inv_dw[a], tb = (hi - r.C[a]) * r.inv_dw[a];
            if (ta > tb) { const float t = ta; ta = tb; tb = t; }
            t0 = fmaxf(t0, ta);
            t1 = fminf(t1, tb);
        }
    }
    if (!(t0 <= t1)) { k0 = 1; k1 = 0; return; }
    k0 = max(1, (int)floorf(t0 * r.inv_delta) - 2);
    k1 = min(kmax, (int)ceilf(t1 * r.inv_delta) + 2);
}

// Empty-space skip.  Samples whose cells have no corner that may hold F <= 0
// (flags are conservative) cannot be the far end of a plus-to-minus
// crossing and are skipped while their cells stay in such a region: the
// bricks within dist - 1 of the sample's brick, else clear cell sub-blocks
// of its brick grown along the ray.  Returns how many samples, from this
// one (local coordinate l, cell base i, in the domain), can be skipped, or 0
// when it must be evaluated.  The jump keeps a 0.01-voxel margin to the box
// [A, B) of cell base coordinates.
struct SkipCache {
    uint32_t b;    // brick whose distance and cell mask are held
    int D;
    uint64_t cm;
};

static __host__ __device__ __forceinline__ int skip_run(const DevVolume& V, const float l[3], const int i[3],
                                                        const float dl[3], const float inv_dl[3],
                                                        GPTR(const uint8_t) distp, GPTR(const uint64_t) cmaskp,
                                                        SkipCache& sc)
{
    int A[3], B[3];
    bool skip = false;
    const uint32_t bi = brick_index32(V, i[0] >> 3, i[1] >> 3, i[2] >> 3);
    if (bi != sc.b) {
        sc.b = bi;
        sc.D = ld_elem(distp, bi);
        sc.cm = ld_elem(cmaskp, bi);
    }
    const int D = sc.D;
    if (D >= 2) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            A[a] = 8 * ((i[a] >> 3) - (D - 1));
            B[a] = 8 * ((i[a] >> 3) + (D - 1)) + 7;
        }
        skip = true;
    } else {
        int lo[3], hi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = (i[a] & 7) >> 1;
        if ((subblock_box(lo, hi) & sc.cm) == 0) {
            skip = true;
            // grown over clear sub-blocks along the ray (x, then y, then z)
            grow_clear_box(sc.cm, lo, hi, dl);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                A[a] = (i[a] & ~7) + 2 * lo[a];
                B[a] = (i[a] & ~7) + 2 * hi[a] + 2;
            }
        }
    }
    if (!skip) return 0;
    float m = 1e30f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dl[a] > 0.0f) m = fminf(m, ((float)B[a] - 0.01f - l[a]) * inv_dl[a]);
        else if (dl[a] < 0.0f) m = fminf(m, (l[a] - ((float)A[a] + 0.01f)) * -inv_dl[a]);
    }
    const int jump = (int)fminf(fmaxf(m, 0.0f), 4096.0f);
    return jump < 1 ? 1 : jump;
}

// March one volume.  Returns true with t* and k when a crossing nearer than
// (best_t, best_id) exists.
static __host__ __device__ bool march_volume(const DevVolume& V, const Ray& r, float delta, int kmax,
                                    float best_t, int best_id, float& tstar, int& kstar, int cell[3])
{
    int k0, k1;
    ray_k_range(V, r, delta, kmax, k0, k1);
    if (k0 > k1) return false;
    {
        const float t0 = (float)k0 * delta;
        if (t0 > best_t || (t0 == best_t && V.id > best_id)) return false;
    }
    // per-sample advance in local voxel units and its reciprocal (for
    // skipping only; the 0.01-voxel shrink of the skip box absorbs rounding)
    float dl[3], inv_dl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dl[a] = delta * r.dw[a] * V.inv_s;
        inv_dl[a] = approx_rcp(dl[a]);
    }

    int prev_k = -2;     // index of the last evaluated sample
    bool prev_ok = false;
    float Fprev = 0.0f;
    GPTR(const uint8_t) const distp = gptr((const uint8_t*)V.dist);
    GPTR(const uint64_t) const cmaskp = gptr((const uint64_t*)V.cmask);
    SkipCache sc;
    sc.b = 0xffffffffu;
    sc.D = 0;
    sc.cm = 0;
    CellCache cc;
    cc.i[0] = -1; cc.i[1] = -1; cc.i[2] = -1;
    int k = k0;
    while (k <= k1) {
        if ((float)(k - 1) * delta > best_t) break;   // nothing nearer can follow
        const float tk = (float)k * delta;
        float l[3];
        sample_coord(V, r, tk, l);
        if (!in_domain(V, l)) {
            prev_k = k; prev_ok = false;
            ++k;
            continue;
        }
        int i[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) i[a] = (int)floorf(l[a]);
        {
            const int jump = skip_run(V, l, i, dl, inv_dl, distp, cmaskp, sc);
            if (jump) {
                prev_ok = false;
                prev_k = -2;
                k += jump;
                continue;
            }
        }
        if (prev_k != k - 1) {
            // re-evaluate the previous sample (skipped or never seen)
            float lp[3];
            sample_coord(V, r, (float)(k - 1) * delta, lp);
            prev_ok = in_domain(V, lp) && eval_sample_cached(V, lp, Fprev, cc);
        }
        float Fk;
        const bool ok = eval_sample_cached(V, l, Fk, cc);
        if (prev_ok && ok && Fprev > 0.0f && Fk <= 0.0f) {
            const float ta = (float)(k - 1) * delta;
            const float ts = ta + ((delta * Fprev) / (Fprev - Fk));
            if (ts < best_t || (ts == best_t && V.id < best_id)) {
                tstar = ts;
                kstar = k;
                cell[0] = i[0]; cell[1] = i[1]; cell[2] = i[2];
                return true;
            }
            return false;
        }
        prev_k = k;
        prev_ok = ok;
        Fprev = Fk;
        ++k;
    }
    return false;
}

#if defined(__HIP_DEVICE_COMPILE__)
// March one volume with the P lanes of a group (lane j of the group; all P
// lanes carry the same ray and take the same path through the loop).  A
// round starts at sample w0: every lane makes the skip decision of sample
// w0 + j; if no sample of that window may be the far end of a crossing the
// group jumps past the longest clear run, otherwise the group evaluates
// kEvalWindows consecutive windows (lane j: samples w0 + w*P + j, all their
// gathers in flight together) and takes the first crossing in sample order,
// exactly as the sequential march would find it.  When the sample before
// the round was not evaluated, w0 is that sample so that it serves as the
// near end.  Rays that graze a surface evaluate long stretches of samples;
// two windows a round halve their rounds of dependent loads.
constexpr int kEvalWindows = 2;

template <int P>
static __device__ bool march_volume_group(const DevVolume& V, const Ray& r, float delta, int kmax, float best_t,
                                          int best_id, float& tstar, int& kstar, int cell[3], int j)
{
    int k0, k1;
    ray_k_range(V, r, delta, kmax, k0, k1);
    if (k0 > k1) return false;
    {
        const float t0 = (float)k0 * delta;
        if (t0 > best_t || (t0 == best_t && V.id > best_id)) return false;
    }
    float dl[3], inv_dl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dl[a] = delta * r.dw[a] * V.inv_s;
        inv_dl[a] = approx_rcp(dl[a]);
    }
    const int gbase = (int)(threadIdx.x & 63u) & ~(P - 1);
    const uint32_t gm = (1u << P) - 1u;
    GPTR(const uint8_t) const distp = gptr((const uint8_t*)V.dist);
    GPTR(const uint64_t) const cmaskp = gptr((const uint64_t*)V.cmask);
    SkipCache sc;
    sc.b = 0xffffffffu;
    sc.D = 0;
    sc.cm = 0;
    int prev_k = -2;
    bool prev_ok = false;
    float Fprev = 0.0f;
    int k = k0;
    while (k <= k1) {
        if ((float)(k - 1) * delta > best_t) break;   // nothing nearer can follow
        const int w0 = (prev_k != k - 1) ? k - 1 : k;
        const int sidx = w0 + j;
        const bool far = sidx >= k && sidx <= k1;       // may be the far end of a crossing
        float l[3];
        sample_coord(V, r, (float)sidx * delta, l);
        const bool dom = in_domain(V, l);
        int i[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) i[a] = (int)floorf(l[a]);
        int reach = sidx + 1;   // end (exclusive) of the run of samples this lane vouches for
        bool must = false;
        if (far && dom) {
            const int jump = skip_run(V, l, i, dl, inv_dl, distp, cmaskp, sc);
            if (jump) reach = sidx + jump;
            else must = true;
        }
        const uint32_t must_g = (uint32_t)(__ballot(must) >> gbase) & gm;
        if (must_g == 0) {
            // the far-end samples of the window lie in overlapping clear runs
            int rmax = far ? reach : k + 1;
#pragma unroll
            for (int o = 1; o < P; o <<= 1) rmax = max(rmax, __shfl_xor(rmax, o));
            prev_ok = false;
            prev_k = -2;
            k = rmax;
            continue;
        }
        // evaluation round: kEvalWindows windows of P consecutive samples
        // from w0, lane j taking sample w0 + w*P + j of window w.  Samples of
        // the later windows are evaluated without a skip test: a sample the
        // test would pass over cannot be the far end of a crossing, so the
        // first crossing found is still the sequential march's.  All gathers
        // are issued before any is used (a sample outside the domain reads
        // cell 0 and is discarded).
        constexpr int S = kEvalWindows;
        float Fs[S], Fns[S];
        int oks[S], ics[S][3];
        uint32_t cross_all = 0, excl_all = 0;
        {
            float cs[S][8], fs[S][3];
            bool doms[S];
#pragma unroll
            for (int w = 0; w < S; ++w) {
                float ls[3];
                if (w == 0) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) ls[a] = l[a];
                    doms[w] = dom;
                } else {
                    sample_coord(V, r, (float)(sidx + w * P) * delta, ls);
                    doms[w] = sidx + w * P <= k1 && in_domain(V, ls);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float fl = floorf(ls[a]);
                    ics[w][a] = doms[w] ? (int)fl : 0;
                    fs[w][a] = ls[a] - fl;
                }
                gather8(V, ics[w], cs[w]);
            }
            float Fc = Fprev;
            int okc = prev_ok;
#pragma unroll
            for (int w = 0; w < S; ++w) {
                const float Fk = trilinear(cs[w], fs[w]);
                const bool ok = doms[w] && !isnan(Fk);
                Fs[w] = Fk;
                oks[w] = ok;
                float Fn = __shfl_up(Fk, 1, P);
                int okn = __shfl_up((int)ok, 1, P);
                if (j == 0) { Fn = Fc; okn = okc; }
                Fns[w] = Fn;
                Fc = __shfl(Fk, gbase + P - 1);
                okc = __shfl((int)ok, gbase + P - 1);
                const int si = sidx + w * P;
                const bool farw = si >= k && si <= k1;
                const bool excl = farw && (float)(si - 1) * delta > best_t;   // the sequential march stops first
                const bool cross = farw && !excl && okn && ok && Fn > 0.0f && Fk <= 0.0f;
                cross_all |= ((uint32_t)(__ballot(cross) >> gbase) & gm) << (w * P);
                excl_all |= ((uint32_t)(__ballot(excl) >> gbase) & gm) << (w * P);
            }
        }
        const int jc = cross_all ? __ffs(cross_all) - 1 : S * P;
        const int je = excl_all ? __ffs(excl_all) - 1 : S * P;
        if (jc < je) {
            const int wc = jc / P, lc = jc - wc * P;
            float Fn = 0.0f, Fk = 0.0f;
            int ic[3] = {0, 0, 0};
#pragma unroll
            for (int w = 0; w < S; ++w)
                if (w == wc) {
                    Fn = Fns[w]; Fk = Fs[w];
                    ic[0] = ics[w][0]; ic[1] = ics[w][1]; ic[2] = ics[w][2];
                }
            float ts = 0.0f;
            int acc = 0;
            if (j == lc) {
                const float ta = (float)(w0 + jc - 1) * delta;
                ts = ta + ((delta * Fn) / (Fn - Fk));
                acc = (ts < best_t || (ts == best_t && V.id < best_id)) ? 1 : 0;
            }
            ts = __shfl(ts, gbase + lc);
            acc = __shfl(acc, gbase + lc);
            if (!acc) return false;
            tstar = ts;
            kstar = w0 + jc;
#pragma unroll
            for (int a = 0; a < 3; ++a) cell[a] = __shfl(ic[a], gbase + lc);
            return true;
        }
        if (je < S * P) return false;
        // no crossing: the last far-end sample becomes the previous one
        const int last = min(w0 + S * P - 1, k1);
        const int jl = last - w0, wl = jl / P, ll = jl - wl * P;
        float Fl = 0.0f;
        int okl = 0;
#pragma unroll
        for (int w = 0; w < S; ++w)
            if (w == wl) { Fl = Fs[w]; okl = oks[w]; }
        prev_ok = __shfl(okl, gbase + ll) != 0;
        Fprev = __shfl(Fl, gbase + ll);
        prev_k = last;
        k = last + 1;
    }
    return false;
}
#endif

// unit normal: the gradient, at world point x, of the trilinear interpolant
// of the given cell (the cell of the crossing's second sample, whose 8
// voxels are all observed)
static __host__ __device__ void surface_normal(const DevVolume& V, const float x[3], const int i[3], float n[3])
{
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float l = (((x[a] - V.o[a]) * V.inv_s) - 0.5f) - (float)V.off[a];
        f[a] = l - (float)i[a];
    }
    float c[8];
    gather8(V, i, c);
    const float gx0 = lerp32(c[1] - c[0], c[3] - c[2], f[1]);
    const float gx1 = lerp32(c[5] - c[4], c[7] - c[6], f[1]);
    const float gx = lerp32(gx0, gx1, f[2]);
    const float c00 = lerp32(c[0], c[1], f[0]);
    const float c10 = lerp32(c[2], c[3], f[0]);
    const float c01 = lerp32(c[4], c[5], f[0]);
    const float c11 = lerp32(c[6], c[7], f[0]);
    const float gy = lerp32(c10 - c00, c11 - c01, f[2]);
    const float gz = lerp32(c01, c11, f[1]) - lerp32(c00, c10, f[1]);
    const float nn = sqrtf(gx * gx + gy * gy + gz * gz);
    if (nn > 0.0f) {
        const float inv = 1.0f / nn;
        n[0] = gx * inv; n[1] = gy * inv; n[2] = gz * inv;
    } else {
        n[0] = n[1] = n[2] = qnan();
    }
}

// Pixel (u, v) of stream s; j: lane of the pixel's group (the host build
// marches sequentially with j = 0).
template <int P>
static __host__ __device__ void raycast_pixel(const RaycastLaunch& L, const LaunchHeader& H, int s, int u, int v,
                                              int j = 0);

template <int P>
__global__ __launch_bounds__(64, 5) void mvf_raycast_kernel(RaycastLaunch L)
{
    const LaunchHeader H = *cptr(L.hdr);
    // Tile groups are taken in the launch order (the slowest groups of the
    // last launch first, when an order is given); each block records how
    // long its tile took.
    const int ngroups = ray_groups(H.total_tiles);
    const int slots = ray_blocks(H.total_tiles);
    for (int idx = blockIdx.x; idx < slots; idx += gridDim.x) {
        const int win = idx / (kXcds * kRayGroup), r = idx - win * (kXcds * kRayGroup);
        const int k = win * kXcds + r % kXcds;   // position in the order
        if (k >= ngroups) continue;
        const int g = L.tile_order ? cptr(L.tile_order)[k] : k;
        const int tile = g * kRayGroup + r / kXcds;
        if (tile >= H.total_tiles) continue;
        const unsigned long long t_tile = wall_clock64();
        CPTR(int32_t) const tile_base = cptr(L.tile_base);
        int s = 0;
        while (s + 1 < H.nstreams && tile_base[s + 1] <= tile) ++s;
        s = wave_uniform(s);
        const int out_w = cptr(L.frames)[s].out_w, out_h = cptr(L.frames)[s].out_h;
        const int local = tile - tile_base[s];
        const int tiles_x = (out_w + L.tile_w - 1) / L.tile_w;
        const int ty = local / tiles_x, tx = local - ty * tiles_x;
        const int pix = (int)threadIdx.x / P;   // P lanes per pixel
        const int u = tx * L.tile_w + pix % L.tile_w;
        const int v = ty * L.tile_h + pix / L.tile_w;
        if (u < out_w && v < out_h) raycast_pixel<P>(L, H, s, u, v, (int)threadIdx.x % P);
        if (L.tile_cost && threadIdx.x == 0) {
            const unsigned long long d = wall_clock64() - t_tile;
            L.tile_cost[tile] = d < 0xffffffffull ? (uint32_t)d : 0xffffffffu;
        }
    }
}

__global__ __launch_bounds__(1024) void mvf_tile_order_kernel(const uint32_t* cost, int32_t* order, int ntiles)
{
    __shared__ int hist[kOrderBins];
    tile_order_block(cost, order, ntiles, hist);
}

int launch_tile_order(const uint32_t* cost, int32_t* order, int n, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(mvf_tile_order_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, cost, order, n);
    return (int)hipGetLastError();
}

template <int P>
static __host__ __device__ void raycast_pixel(const RaycastLaunch& L, const LaunchHeader& H, int s, int u, int v,
                                              int j)
{
    const DevFrame Fr = cptr(L.frames)[s];
    const size_t p = (size_t)v * Fr.out_w + u;

    // ray (binary32 contract)
    Ray r;
    float dh[3];
    {
        const float dc0 = ((float)u - Fr.cx) / Fr.fx;
        const float dc1 = ((float)v - Fr.cy) / Fr.fy;
        const float n = sqrtf(((dc0 * dc0) + (dc1 * dc1)) + (1.0f * 1.0f));
        const float inv_n = 1.0f / n;
        dh[0] = dc0 * inv_n;
        dh[1] = dc1 * inv_n;
        dh[2] = 1.0f * inv_n;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.dw[a] = ((Fr.T[4 * a + 0] * dh[0]) + (Fr.T[4 * a + 1] * dh[1])) + (Fr.T[4 * a + 2] * dh[2]);
            r.C[a] = Fr.T[4 * a + 3];
            r.inv_dw[a] = approx_rcp(r.dw[a]);
        }
        r.inv_delta = approx_rcp(H.rp.delta);
        // the range bounds of the pixel's cell and of the whole image
        r.t_lo = 0.0f;
        r.t_hi = pinf();
        if (Fr.rb_lo) {
            const int cell = (v / kBoundCell) * Fr.cells_x + u / kBoundCell;
            r.t_lo = Fr.rb_lo[cell];
            r.t_hi = Fr.rb_hi[cell];
        }
    }
    float best_t = pinf();
    int best_id = 0x7fffffff;
    int best_vol = -1;
    int best_k = -1;
    int best_cell[3] = {0, 0, 0};
    if (!H.first_wave) {
        const int prev = Fr.best_id[p];
        if (prev >= 0) { best_t = Fr.best_t[p]; best_id = prev; }
    }
    const int l0 = cptr(L.list_base)[s], l1 = cptr(L.list_base)[s + 1];
    for (int li = l0; li < l1; ++li) {
        const DevVolume V = cptr(L.vols)[cptr(L.lists)[li]];
        float ts;
        int ks, cell[3];
#if defined(__HIP_DEVICE_COMPILE__)
        const bool found = march_volume_group<P>(V, r, H.rp.delta, H.rp.kmax, best_t, best_id, ts, ks, cell, j);
#else
        const bool found = march_volume(V, r, H.rp.delta, H.rp.kmax, best_t, best_id, ts, ks, cell);
#endif
        if (found) {
            best_t = ts;
            best_id = V.id;
            best_k = ks;
            best_vol = cptr(L.lists)[li];
            best_cell[0] = cell[0]; best_cell[1] = cell[1]; best_cell[2] = cell[2];
        }
    }
    if (j != 0) return;   // the group's first lane writes the pixel
    if (best_vol >= 0) {
        const DevVolume V = cptr(L.vols)[best_vol];
        float x[3], n[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = r.C[a] + (best_t * r.dw[a]);
        surface_normal(V, x, best_cell, n);
        Fr.depth[p] = best_t * dh[2];
        if (Fr.vertex) { Fr.vertex[3 * p] = x[0]; Fr.vertex[3 * p + 1] = x[1]; Fr.vertex[3 * p + 2] = x[2]; }
        if (Fr.normal) { Fr.normal[3 * p] = n[0]; Fr.normal[3 * p + 1] = n[1]; Fr.normal[3 * p + 2] = n[2]; }
        if (Fr.hit) Fr.hit[p] = V.id;
        if (Fr.record) Fr.record[p] = best_k;
        if (Fr.best_t) { Fr.best_t[p] = best_t; Fr.best_id[p] = best_id; }
    } else if (H.first_wave) {
        const float qn = qnan();
        Fr.depth[p] = 0.0f;
        if (Fr.vertex) { Fr.vertex[3 * p] = qn; Fr.vertex[3 * p + 1] = qn; Fr.vertex[3 * p + 2] = qn; }
        if (Fr.normal) { Fr.normal[3 * p] = qn; Fr.normal[3 * p + 1] = qn; Fr.normal[3 * p + 2] = qn; }
        if (Fr.hit) Fr.hit[p] = -1;
        if (Fr.record) Fr.record[p] = -1;
        if (Fr.best_t) { Fr.best_t[p] = pinf(); Fr.best_id[p] = -1; }
    }
}

template <int P>
static void launch_raycast_p(const RaycastLaunch& L, int blocks, hipStream_t stream, hipEvent_t a, hipEvent_t b)
{
    if (a)
        hipExtLaunchKernelGGL(mvf_raycast_kernel<P>, dim3(blocks), dim3(64), 0, stream, a, b, 0, L);
    else
        hipLaunchKernelGGL(mvf_raycast_kernel<P>, dim3(blocks), dim3(64), 0, stream, L);
}

int launch_raycast(const RaycastLaunch& L, int blocks, void* stream, void* ev_start, void* ev_stop)
{
    if (blocks <= 0) return 0;
    if (ray_tile_w(L.lanes) != L.tile_w || ray_tile_h(L.lanes) != L.tile_h) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = (hipEvent_t)ev_start, b = (hipEvent_t)ev_stop;
    switch (L.lanes) {
    case 2: launch_raycast_p<2>(L, blocks, s, a, b); break;
    case 4: launch_raycast_p<4>(L, blocks, s, a, b); break;
    case 8: launch_raycast_p<8>(L, blocks, s, a, b); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Brick summary: exact recompute of the per-brick "may hold F <= 0" flags
// and sub-block masks (after a volume is written from the host).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mvf_brick_summary_kernel(DevVolume v, size_t nbricks)
{
    const int lane = threadIdx.x & 63;
    const size_t brick = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (brick >= nbricks) return;
    const float* F = v.F + brick * kBrickVox + lane;
    uint64_t fm = 0;
    for (int zp = 0; zp < kBrick / 2; ++zp) {
        const bool a = F[(2 * zp) * 64] <= kFlagThreshold;
        const bool b = F[(2 * zp + 1) * 64] <= kFlagThreshold;
        fm |= (uint64_t)subblock_bits(__ballot(a | b)) << (16 * zp);
    }
    if (lane == 0) {
        v.flag[brick] = fm ? 1 : 0;
        v.fmask[brick] = fm;
    }
}

// Column flag words after a full flag recompute: one wavefront per word,
// lane l taking the flag of brick 64 w + l of the column.
__global__ __launch_bounds__(256) void mvf_column_flags_kernel(DevVolume v, int ncolw)
{
    const int lane = threadIdx.x & 63;
    const int nw = col_words(v.bd[2]);
    const int step = (int)(gridDim.x * (blockDim.x >> 6));
    for (int cw = wave_uniform((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6))); cw < ncolw; cw += step) {
        const int col = cw / nw, w = cw - col * nw;
        const int bz = 64 * w + lane;
        const bool f = bz < v.bd[2] && v.flag[(size_t)col * v.bd[2] + bz] != 0;
        const unsigned long long m = __ballot(f);
        if (lane == 0) v.colm[cw] = m;
    }
}

int launch_brick_summary(DevVolume v, void* stream)
{
    const size_t nb = (size_t)v.bd[0] * v.bd[1] * v.bd[2];
    hipLaunchKernelGGL(mvf_brick_summary_kernel, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0,
                       (hipStream_t)stream, v, nb);
    const int ncolw = v.bd[0] * v.bd[1] * col_words(v.bd[2]);
    hipLaunchKernelGGL(mvf_column_flags_kernel, dim3((unsigned)std::min((ncolw + 3) / 4, 65535)), dim3(256), 0,
                       (hipStream_t)stream, v, ncolw);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Brick distance transform and cell masks: one launch for every volume of
// the table, two kinds of wavefronts.
//
// Distance lines (the first kDistWaves wavefronts): one per (bx, chunk of
// kDistRows columns along y, 64-brick word w of the columns).  Lane l holds
// the row y = y0 - kDistCap + l and ORs that row's column words along x
// outwards, X_k = OR over |dx| <= k; C_k, the OR of X_k over the lanes
// within k, covers the columns within Chebyshev distance k in (x, y); a
// brick of the word is within distance k of a flagged brick iff its bit is
// set in the z-dilation of C_k by k.  The capped distances of the word's 64
// bricks are kept as four bit planes (bit z of plane i = bit i of brick z's
// distance) and written by the middle kDistRows lanes.  Columns of more than
// 64 bricks also take the words below and above (the dilation reaches
// kDistCap < 64 bits into them).
//
// Bricks (the other wavefronts): one thread per brick, 64 consecutive
// bricks of one volume per wavefront (brick_base): the cell mask from the
// sub-block flags of the brick and its +x, +y, +z neighbours and, with range
// bounds, the brick's footprint.
// ---------------------------------------------------------------------------
constexpr int kDistSide = 2 * kDistCap + 1;
constexpr int kDistRows = 64 - 2 * kDistCap;  // output columns of a distance line
constexpr int kDistWaves = 256;               // wavefronts of the distance lines

// Dilation by r (r < 16) in shift steps of 1, 2, 4 and the rest: a step s
// with s <= c + 1 widens the covered offsets [-c, c] to [-(c + s), c + s]
// without a gap (shifts of 8 and 2 alone would cover only 0, 2, 6, 8, 10).
template <class Step>
static __device__ __forceinline__ void covering_steps(int r, Step step)
{
    int c = 0;
#pragma unroll
    for (int s = 1; s <= 8; s <<= 1) {
        if (c < r) {
            const int st = min(s, r - c);
            step(st);
            c += st;
        }
    }
}

// OR of x over the lanes within r; lanes beyond the wavefront add nothing.
static __device__ __forceinline__ uint64_t lane_dilate(uint64_t x, int r)
{
    covering_steps(r, [&](int st) { x |= __shfl_up(x, st) | __shfl_down(x, st); });
    return x;
}

// The bits of the window prev | cur | next within r (r <= kDistCap) of a set
// bit; prev and next keep the bits that can still reach cur.
static __device__ __forceinline__ void z_dilate(uint64_t& prev, uint64_t& cur, uint64_t& next, int r)
{
    covering_steps(r, [&](int st) {
        const uint64_t p = prev, c = cur, n = next;
        cur = c | (c << st) | (c >> st) | (p >> (64 - st)) | (n << (64 - st));
        prev = p | (p << st) | (p >> st) | (c << (64 - st));
        next = n | (n << st) | (n >> st) | (c >> (64 - st));
    });
}

// Bits 0..3 of x to the low bit of each byte.
static __device__ __forceinline__ uint32_t spread4(uint32_t x)
{
    x &= 0xfu;
    return (x | (x << 7) | (x << 14) | (x << 21)) & 0x01010101u;
}

template <bool Multi>
static __device__ void distance_line(const DevVolume& V, int bx, int y0, int w, int lane)
{
    const int nw = col_words(V.bd[2]);
    const int ncw = V.bd[0] * V.bd[1] * nw;
    GPTR(const uint64_t) const colm = gptr((const uint64_t*)V.colm);
    const int y = y0 - kDistCap + lane;
    const bool row_in = y >= 0 && y < V.bd[1];
    const uint32_t row = (uint32_t)(row_in ? y : 0);
    // word ncw of colm is always zero: out-of-range neighbours read it
    auto word = [&](int x, int ww) -> uint64_t {
        const bool in = row_in && x >= 0 && x < V.bd[0] && ww >= 0 && ww < nw;
        return ld_elem(colm, in ? ((uint32_t)x * (uint32_t)V.bd[1] + row) * (uint32_t)nw + (uint32_t)ww
                                : (uint32_t)ncw);
    };
    uint64_t Xp = 0, X = 0, Xn = 0;
    uint64_t p0 = 0, p1 = 0, p2 = ~0ull, p3 = ~0ull, found = 0;  // kDistCap = 12 = 0b1100 until found
    static_assert(kDistCap == 12, "bit planes start at the cap");
    // distance k: C_k dilated along z, the bricks it reaches first get k
    auto ring = [&](int k) {
        uint64_t c = lane_dilate(X, k);
        uint64_t cp = Multi ? lane_dilate(Xp, k) : 0ull;
        uint64_t cn = Multi ? lane_dilate(Xn, k) : 0ull;
        z_dilate(cp, c, cn, k);
        const uint64_t fresh = c & ~found;
        found |= c;
        p0 = (k & 1) ? (p0 | fresh) : (p0 & ~fresh);
        p1 = (k & 2) ? (p1 | fresh) : (p1 & ~fresh);
        p2 = (k & 4) ? (p2 | fresh) : (p2 & ~fresh);
        p3 = (k & 8) ? (p3 | fresh) : (p3 & ~fresh);
    };
    if (Multi) {
        // three words a row: loaded as the rings grow (a rare shape)
#pragma unroll 1
        for (int k = 0; k <= kDistCap; ++k) {
            X |= word(bx - k, w) | word(bx + k, w);
            Xp |= word(bx - k, w - 1) | word(bx + k, w - 1);
            Xn |= word(bx - k, w + 1) | word(bx + k, w + 1);
            ring(k);
        }
    } else {
        uint64_t m[kDistSide];
#pragma unroll
        for (int i = 0; i < kDistSide; ++i) m[i] = word(bx + i - kDistCap, w);
#pragma unroll
        for (int k = 0; k <= kDistCap; ++k) {
            X |= m[kDistCap - k] | m[kDistCap + k];
            ring(k);
        }
    }
    if (lane < kDistCap || lane >= kDistCap + kDistRows || !row_in) return;
    const int nz = min(64, V.bd[2] - 64 * w);
    const uint32_t b0 = ((uint32_t)bx * (uint32_t)V.bd[1] + row) * (uint32_t)V.bd[2] + 64u * (uint32_t)w;
    const bool aligned = (V.bd[2] & 3) == 0;
#pragma unroll
    for (int j = 0; j < 64; j += 4) {
        if (j >= nz) break;
        const uint32_t v = spread4((uint32_t)(p0 >> j)) | (spread4((uint32_t)(p1 >> j)) << 1) |
                           (spread4((uint32_t)(p2 >> j)) << 2) | (spread4((uint32_t)(p3 >> j)) << 3);
        if (aligned) {
            *(uint32_t*)(V.dist + b0 + j) = v;  // nz is a multiple of 4 here
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j + q < nz) V.dist[b0 + j + q] = (uint8_t)(v >> (8 * q));
        }
    }
}

// at most 96 VGPRs: five wavefronts per SIMD still hold every brick wavefront of
// a 512^3 volume at once
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void mvf_brick_distance_kernel(
    const LaunchHeader* hdr, const DevVolume* vols, const int32_t* brick_base, const DevFrame* frames, RayBounds rb)
{
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int nvol = cptr(hdr)->nvol;
    if (wave < kDistWaves) {
        // the lines of all volumes, numbered volume by volume, are dealt to
        // the distance wavefronts in turn; acc = lines before volume v,
        // modulo kDistWaves
        int acc = 0;
        for (int v = 0; v < nvol; ++v) {
            CPTR(DevVolume) const Vp = cptr(vols) + v;
            const int nw = col_words(Vp->bd[2]);
            const int nyc = (Vp->bd[1] + kDistRows - 1) / kDistRows;
            const int nl = Vp->bd[0] * nyc * nw;
            int first = (wave - acc) % kDistWaves;
            if (first < 0) first += kDistWaves;
            acc = (int)(((long long)acc + nl) % kDistWaves);
            if (first >= nl) continue;
            const DevVolume V = *Vp;
            for (int t = first; t < nl; t += kDistWaves) {
                const int w = t % nw, r = t / nw;
                const int yc = r % nyc, bx = r / nyc;
                if (nw == 1) distance_line<false>(V, bx, yc * kDistRows, w, lane);
                else distance_line<true>(V, bx, yc * kDistRows, w, lane);
            }
        }
        return;
    }
    const int total = cptr(hdr)->total_bricks;
    const int bwaves = (int)(gridDim.x * (blockDim.x >> 6)) - kDistWaves;
    CPTR(int32_t) const bbase = cptr(brick_base);
    for (int g = wave - kDistWaves; g * 64 < total; g += bwaves) {
        const int gw = g * 64;
        int lo = 0, hi = nvol - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (bbase[mid] <= gw) lo = mid; else hi = mid - 1;
        }
        lo = wave_uniform(lo);
        const DevVolume V = cptr(vols)[lo];
        const int nb = V.bd[0] * V.bd[1] * V.bd[2];
        const int b = gw + lane - bbase[lo];
        const bool valid = b < nb;
        const int bc = valid ? b : 0;
        const int bz = bc % V.bd[2];
        const int t = bc / V.bd[2];
        const int by = t % V.bd[1];
        const int bx = t / V.bd[1];
        uint64_t cm = 0;
        if (valid) {
            GPTR(const uint64_t) const fm = gptr((const uint64_t*)V.fmask);
            uint64_t M[2][2][2];
#pragma unroll
            for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        const bool in = bx + dx < V.bd[0] && by + dy < V.bd[1] && bz + dz < V.bd[2];
                        M[dz][dy][dx] = ld_elem(fm, in ? brick_index32(V, bx + dx, by + dy, bz + dz) : (uint32_t)b);
                        M[dz][dy][dx] = in ? M[dz][dy][dx] : 0ull;
                    }
            cm = cell_mask(M);
            V.cmask[b] = cm;
        }
        if (frames && rb.entries) collect_footprint(V, frames[V.frame], lo, cm, bx, by, bz, brick_base, hdr, rb);
    }
}

// blocks: wavefront groups of four for the bricks; the distance lines get
// kDistWaves more wavefronts
int launch_brick_distance(const LaunchHeader* hdr, const DevVolume* vols, const int32_t* brick_base, int blocks,
                          void* stream, const DevFrame* frames, RayBounds rb)
{
    if (blocks <= 0) return 0;
    hipLaunchKernelGGL(mvf_brick_distance_kernel, dim3(blocks + kDistWaves / 4), dim3(256), 0, (hipStream_t)stream,
                       hdr, vols, brick_base, frames, rb);
    return (int)hipGetLastError();
}

// Range-bound footprints of every brick of the table (one thread per brick,
// a wavefront within one volume as in the distance transform).
__global__ __launch_bounds__(256) void mvf_ray_bounds_collect_kernel(const LaunchHeader* hdr, const DevVolume* vols,
                                                                     const int32_t* brick_base,
                                                                     const DevFrame* frames, RayBounds rb)
{
    const int total = hdr->total_bricks;
    const int nvol = hdr->nvol;
    for (int g0 = blockIdx.x * blockDim.x; g0 < total; g0 += gridDim.x * blockDim.x) {
        const int gw = wave_uniform(g0 + (int)(threadIdx.x & ~63u));
        int lo = 0, hi = nvol - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (brick_base[mid] <= gw) lo = mid; else hi = mid - 1;
        }
        lo = wave_uniform(lo);
        const DevVolume& V = vols[lo];
        const int b = g0 + (int)threadIdx.x - brick_base[lo];
        const int nb = V.bd[0] * V.bd[1] * V.bd[2];
        if (b >= nb) continue;
        const int bz = b % V.bd[2];
        const int t = b / V.bd[2];
        collect_footprint(V, frames[V.frame], lo, V.cmask[b], t / V.bd[1], t % V.bd[1], bz, brick_base, hdr, rb);
    }
}

int launch_ray_bounds_collect(const LaunchHeader* hdr, const DevVolume* vols, const int32_t* brick_base,
                              const DevFrame* frames, RayBounds rb, int blocks, void* stream)
{
    if (blocks <= 0) return 0;
    hipLaunchKernelGGL(mvf_ray_bounds_collect_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, hdr, vols,
                       brick_base, frames, rb);
    return (int)hipGetLastError();
}

// Block (x, y, s): cells [8x, 8x + 8) x [8y, 8y + 8) of stream s, folded in
// LDS from every footprint of the stream's volumes.  Block (0, 0, 0) also
// clears the other half of the counts.
__global__ __launch_bounds__(1024) void mvf_ray_bounds_merge_kernel(const LaunchHeader* hdr, const DevFrame* frames,
                                                                   const int32_t* lists, const int32_t* list_base,
                                                                   const int32_t* brick_base, RayBounds rb)
{
    const int par = hdr->rb_parity;
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0)
        for (int i = threadIdx.x; i < rb.cap; i += blockDim.x) rb.counts[(1 - par) * rb.cap + i] = 0;
    const int s = blockIdx.z;
    if (s >= hdr->nstreams) return;
    const DevFrame& Fr = frames[s];
    const int cx0 = blockIdx.x * 8, cy0 = blockIdx.y * 8;
    if (!Fr.rb_lo || cx0 >= Fr.cells_x || cy0 >= Fr.cells_y) return;
    __shared__ uint32_t lo[64], hi[64];
    if (threadIdx.x < 64) {
        lo[threadIdx.x] = 0x7f800000u;   // +inf
        hi[threadIdx.x] = 0u;
    }
    __syncthreads();
    for (int li = list_base[s]; li < list_base[s + 1]; ++li) {
        const int v = lists[li];
        const uint32_t n = rb.counts[par * rb.cap + v];
        const RayBoundEntry* E = rb.entries + brick_base[v];
        // four entries per thread per round, their loads in flight together
        for (uint32_t i0 = 0; i0 < n; i0 += 4 * blockDim.x) {
            RayBoundEntry e[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t i = i0 + q * blockDim.x + threadIdx.x;
                if (i < n) e[q] = E[i];
                else e[q].x0 = 1, e[q].x1 = 0;   // empty
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x0 = max((int)e[q].x0, cx0), x1 = min((int)e[q].x1, cx0 + 7);
                const int y0 = max((int)e[q].y0, cy0), y1 = min((int)e[q].y1, cy0 + 7);
                if (x0 > x1) continue;
                for (int y = y0; y <= y1; ++y)
                    for (int x = x0; x <= x1; ++x) {
                        const int k = (y - cy0) * 8 + (x - cx0);
                        atomicMin(&lo[k], __float_as_uint(e[q].dn));   // distances are >= 0: bit order is value order
                        atomicMax(&hi[k], __float_as_uint(e[q].df));
                    }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int x = cx0 + (threadIdx.x & 7), y = cy0 + (threadIdx.x >> 3);
        if (x < Fr.cells_x && y < Fr.cells_y) {
            Fr.rb_lo[y * Fr.cells_x + x] = __uint_as_float(lo[threadIdx.x]);
            Fr.rb_hi[y * Fr.cells_x + x] = __uint_as_float(hi[threadIdx.x]);
        }
    }
}

int launch_ray_bounds_merge(const LaunchHeader* hdr, const DevFrame* frames, const int32_t* lists,
                            const int32_t* list_base, const int32_t* brick_base, RayBounds rb, int nstreams,
                            int max_cells_x, int max_cells_y, void* stream)
{
    if (nstreams <= 0) return 0;
    const dim3 grid((max_cells_x + 7) / 8, (max_cells_y + 7) / 8, nstreams);
    hipLaunchKernelGGL(mvf_ray_bounds_merge_kernel, grid, dim3(1024), 0, (hipStream_t)stream, hdr, frames, lists,
                       list_base, brick_base, rb);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversion between brick-linear device planes and canonical
// x-fastest planes.  One thread per canonical voxel.
// ---------------------------------------------------------------------------
static __device__ __forceinline__ size_t brick_offset(const DevVolume& v, int x, int y, int z)
{
    return brick_index(v.bd, x >> 3, y >> 3, z >> 3) * kBrickVox +
           (size_t)(((z & 7) << 6) | ((y & 7) << 3) | (x & 7));
}

__global__ __launch_bounds__(256) void mvf_to_canonical_kernel(DevVolume v, float* F, uint16_t* W, uint32_t* C)
{
    const size_t n = (size_t)v.dims[0] * v.dims[1] * v.dims[2];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int x = (int)(i % v.dims[0]);
        const int y = (int)((i / v.dims[0]) % v.dims[1]);
        const int z = (int)(i / ((size_t)v.dims[0] * v.dims[1]));
        const size_t b = brick_offset(v, x, y, z);
        const uint16_t w = v.W[b];
        if (F) F[i] = w ? v.F[b] : 0.0f;
        if (W) W[i] = w;
        if (C) C[i] = v.C[b];
    }
}

__global__ __launch_bounds__(256) void mvf_from_canonical_kernel(DevVolume v, const float* F, const uint16_t* W,
                                                                 const uint32_t* C)
{
    const size_t n = (size_t)v.dims[0] * v.dims[1] * v.dims[2];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int x = (int)(i % v.dims[0]);
        const int y = (int)((i / v.dims[0]) % v.dims[1]);
        const int z = (int)(i / ((size_t)v.dims[0] * v.dims[1]));
        const size_t b = brick_offset(v, x, y, z);
        const uint16_t w = W ? W[i] : 0;
        v.W[b] = w;
        v.F[b] = (w && F) ? F[i] : (w ? 0.0f : __uint_as_float(0x7fc00000u));
        v.C[b] = C ? C[i] : 0u;
    }
}

static int conv_blocks(const DevVolume& v)
{
    const size_t n = (size_t)v.dims[0] * v.dims[1] * v.dims[2];
    size_t b = (n + 255) / 256;
    return (int)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
}

int launch_to_canonical(DevVolume v, float* F, uint16_t* W, uint32_t* C, void* stream)
{
    hipLaunchKernelGGL(mvf_to_canonical_kernel, dim3(conv_blocks(v)), dim3(256), 0, (hipStream_t)stream,
                       v, F, W, C);
    return (int)hipGetLastError();
}

int launch_from_canonical(DevVolume v, const float* F, const uint16_t* W, const uint32_t* C, void* stream)
{
    hipLaunchKernelGGL(mvf_from_canonical_kernel, dim3(conv_blocks(v)), dim3(256), 0, (hipStream_t)stream,
                       v, F, W, C);
    return (int)hipGetLastError();
}

__global__ void mvf_fill_u64_kernel(unsigned long long* p, int n, unsigned long long value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

int launch_fill_u64(unsigned long long* p, int n, unsigned long long value, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(mvf_fill_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, p, n,
                       value);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Placement counting (Dynamic Mapping for SLAM section): per valid pixel,
// endpoint e = R (D K^-1 [u v 1]) + t, cell k = floor((e - o) / cell), then
// an open-addressing hash count.  Slot h holds the packed cell key in
// table[2h] (all ones = empty) and its count in table[2h + 1].
// ---------------------------------------------------------------------------
static __device__ __forceinline__ unsigned long long pack_cell(int kx, int ky, int kz)
{
    return ((unsigned long long)(uint32_t)(kx + (1 << 20)) << 42) |
           ((unsigned long long)(uint32_t)(ky + (1 << 20)) << 21) |
           (unsigned long long)(uint32_t)(kz + (1 << 20));
}

__global__ __launch_bounds__(256) void mvf_placement_count_kernel(
    const float* __restrict__ depth, int depth_pitch, int width, int height, float fx, float fy,
    float cx, float cy, const float* __restrict__ Tp, float o0, float o1, float o2, float cell,
    unsigned long long* table, int table_size, int* overflow, const int32_t* __restrict__ boxes,
    int n_boxes, float voxel)
{
    const int u = blockIdx.x * 32 + (threadIdx.x & 31);
    const int v = blockIdx.y * 8 + (threadIdx.x >> 5);
    if (u >= width || v >= height) return;
    const float Dz = depth[(size_t)v * depth_pitch + u];
    if (!(Dz > 0.0f && Dz < INFINITY)) return;
    float T[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) T[i] = Tp[i];
    const float ra = ((float)u - cx) / fx;
    const float rb = ((float)v - cy) / fy;
    const float q0 = Dz * ra, q1 = Dz * rb, q2 = Dz;
    const float o[3] = { o0, o1, o2 };
    int k[3];
    float e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        e[r] = (((T[4 * r + 0] * q0) + (T[4 * r + 1] * q1)) + (T[4 * r + 2] * q2)) + T[4 * r + 3];
        const float kf = floorf((e[r] - o[r]) / cell);
        if (!(kf >= -1048576.0f && kf < 1048576.0f)) { atomicOr(overflow, 2); return; }
        k[r] = (int)kf;
    }
    if (n_boxes > 0) {
        // endpoints inside a listed volume (global voxels [h_t, h_t + dims))
        // are not counted; the voxel is the cell of the side-one lattice
        int g[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float gf = floorf((e[r] - o[r]) / voxel);
            if (!(gf >= -1073741824.0f && gf < 1073741824.0f)) { atomicOr(overflow, 2); return; }
            g[r] = (int)gf;
        }
        for (int b = 0; b < n_boxes; ++b) {
            const int32_t* B = boxes + 6 * b;
            bool in = true;
#pragma unroll
            for (int r = 0; r < 3; ++r) in = in && g[r] >= B[r] && (int64_t)g[r] < (int64_t)B[r] + B[3 + r];
            if (in) return;
        }
    }
    const unsigned long long key = pack_cell(k[0], k[1], k[2]);
    unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 40) & (unsigned)(table_size - 1);
    for (int probe = 0; probe < table_size; ++probe) {
        unsigned long long* slot = table + 2 * (size_t)h;
        const unsigned long long prev = atomicCAS(slot, ~0ull, key);
        if (prev == ~0ull || prev == key) {
            atomicAdd(slot + 1, 1ull);
            return;
        }
        h = (h + 1) & (unsigned)(table_size - 1);
    }
    atomicOr(overflow, 1);
}

__global__ void mvf_placement_clear_kernel(unsigned long long* table, int table_size)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < table_size) {
        table[2 * (size_t)i] = ~0ull;
        table[2 * (size_t)i + 1] = 0ull;
    }
}

int launch_placement_clear(unsigned long long* table, int table_size, void* stream)
{
    hipLaunchKernelGGL(mvf_placement_clear_kernel, dim3((table_size + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, table, table_size);
    return (int)hipGetLastError();
}

int launch_placement_count(const float* depth, int depth_pitch, int width, int height, float fx, float fy,
                           float cx, float cy, const float* T, float o0, float o1, float o2, float cell,
                           unsigned long long* table, int table_size, int* overflow, const int32_t* boxes,
                           int n_boxes, float voxel, void* stream)
{
    dim3 grid((width + 31) / 32, (height + 7) / 8);
    hipLaunchKernelGGL(mvf_placement_count_kernel, grid, dim3(256), 0, (hipStream_t)stream, depth, depth_pitch,
                       width, height, fx, fy, cx, cy, T, o0, o1, o2, cell, table, table_size, overflow, boxes,
                       n_boxes, voxel);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Surface points (Input and Output: the vertex set V with normals N, at most
// one vertex per voxel; Metrics: a voxel the surface crosses gets a vertex).
// Voxel g emits a vertex when its cell [g, g + 1]^3 lies in the volume, all
// 8 corners are observed (not NaN), and F changes sign (one end > 0, the
// other <= 0) inside the band (|F| < 1) along one of the edges +x, +y, +z
// leaving g; the first such edge in that order holds the vertex, at the
// linear zero crossing, and the normal is the normalised gradient of the
// cell's trilinear interpolant there.  A cell whose base voxel lies in a
// sub-block with a clear cell-mask bit has no corner F <= 2^-100, hence no
// sign change: such z-slice pairs and bricks are skipped.
//
// Three launches: per-brick counts (one wavefront per brick), an exclusive
// prefix sum over the bricks, and the emission, which writes brick by brick
// (inside a brick z-slice by z-slice, x fastest), so the order is fixed.
// ---------------------------------------------------------------------------
struct SurfVoxel {
    bool emit;
    int axis;
    float c[8];   // corner (x + (k & 1), y + (k >> 1 & 1), z + (k >> 2))
};

static __device__ __forceinline__ void surf_voxel(const DevVolume& v, GPTR(const float) F, int gx, int gy, int gz,
                                                  SurfVoxel& S)
{
    S.emit = false;
    S.axis = -1;
    if (gx + 1 >= v.dims[0] || gy + 1 >= v.dims[1] || gz + 1 >= v.dims[2]) return;
    bool observed = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int x = gx + (k & 1), y = gy + ((k >> 1) & 1), z = gz + (k >> 2);
        const size_t o = brick_index(v.bd, x >> 3, y >> 3, z >> 3) * kBrickVox +
                         (size_t)(((z & 7) << 6) | ((y & 7) << 3) | (x & 7));
        S.c[k] = F[o];
        observed &= !__builtin_isnan(S.c[k]);
    }
    if (!observed) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float f0 = S.c[0], f1 = S.c[1 << a];
        const bool in_band = fabsf(f0) < 1.0f && fabsf(f1) < 1.0f;
        const bool change = (f0 > 0.0f && f1 <= 0.0f) || (f0 <= 0.0f && f1 > 0.0f);
        if (S.axis < 0 && in_band && change) S.axis = a;
    }
    S.emit = S.axis >= 0;
}

// Bits of the cell mask for the two z-slices 2 zp and 2 zp + 1 of a brick.
static __device__ __forceinline__ uint32_t cmask_pair(uint64_t cm, int zp)
{
    return (uint32_t)((cm >> (16 * zp)) & 0xffffu);
}

__global__ __launch_bounds__(256) void mvf_extract_count_kernel(DevVolume v, size_t nbricks, uint32_t* counts)
{
    const int lane = threadIdx.x & 63;
    const int lx = lane & 7, ly = lane >> 3;
    GPTR(const float) F = gptr((const float*)v.F);
    const size_t waves = (size_t)gridDim.x * (blockDim.x >> 6);
    for (size_t b = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nbricks; b += waves) {
        const uint64_t cm = v.cmask[b];
        uint32_t n = 0;
        if (cm) {
            const int bz = (int)(b % v.bd[2]);
            const size_t t = b / v.bd[2];
            const int by = (int)(t % v.bd[1]), bx = (int)(t / v.bd[1]);
            for (int zp = 0; zp < 4; ++zp) {
                if (!cmask_pair(cm, zp)) continue;
                for (int dz = 0; dz < 2; ++dz) {
                    SurfVoxel S;
                    surf_voxel(v, F, 8 * bx + lx, 8 * by + ly, 8 * bz + 2 * zp + dz, S);
                    n += (uint32_t)__popcll(__ballot(S.emit));
                }
            }
        }
        if (lane == 0) counts[b] = n;
    }
}

// Exclusive prefix sum of n counts by one block of 1024 threads (each takes
// a contiguous run); total[0] = the sum.
__global__ __launch_bounds__(1024) void mvf_extract_scan_kernel(const uint32_t* counts, size_t n,
                                                                unsigned long long* offsets,
                                                                long long* total)
{
    __shared__ unsigned long long part[1024];
    const size_t per = (n + 1023) / 1024;
    const size_t lo = min(n, (size_t)threadIdx.x * per), hi = min(n, lo + per);
    unsigned long long s = 0;
    for (size_t i = lo; i < hi; ++i) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned long long add = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0ull;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = part[threadIdx.x] - s;
    for (size_t i = lo; i < hi; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == 1023) total[0] = (long long)part[1023];
}

__global__ __launch_bounds__(256) void mvf_extract_emit_kernel(DevVolume v, size_t nbricks,
                                                               const unsigned long long* offsets, float* V, float* N,
                                                               int32_t* G, long long cap)
{
    const int lane = threadIdx.x & 63;
    const int lx = lane & 7, ly = lane >> 3;
    GPTR(const float) F = gptr((const float*)v.F);
    const unsigned long long below = (1ull << lane) - 1ull;
    const size_t waves = (size_t)gridDim.x * (blockDim.x >> 6);
    for (size_t b = (size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nbricks; b += waves) {
        const uint64_t cm = v.cmask[b];
        if (!cm) continue;
        unsigned long long base = offsets[b];
        if ((long long)base >= cap) continue;
        const int bz = (int)(b % v.bd[2]);
        const size_t t = b / v.bd[2];
        const int by = (int)(t % v.bd[1]), bx = (int)(t / v.bd[1]);
        for (int zp = 0; zp < 4; ++zp) {
            if (!cmask_pair(cm, zp)) continue;
            for (int dz = 0; dz < 2; ++dz) {
                const int gx = 8 * bx + lx, gy = 8 * by + ly, gz = 8 * bz + 2 * zp + dz;
                SurfVoxel S;
                surf_voxel(v, F, gx, gy, gz, S);
                const unsigned long long m = __ballot(S.emit);
                const unsigned long long idx = base + (unsigned long long)__popcll(m & below);
                base += (unsigned long long)__popcll(m);
                if (!S.emit || (long long)idx >= cap) continue;
                const float* c = S.c;
                const int a = S.axis;
                const float f0 = c[0], f1 = c[1 << a];
                float fr[3] = { 0.0f, 0.0f, 0.0f };
                fr[a] = f0 / (f0 - f1);
                // gradient of the trilinear interpolant at fr (local units)
                const float c00 = lerp32(c[0], c[1], fr[0]), c10 = lerp32(c[2], c[3], fr[0]);
                const float c01 = lerp32(c[4], c[5], fr[0]), c11 = lerp32(c[6], c[7], fr[0]);
                const float g0 = lerp32(lerp32(c[1] - c[0], c[3] - c[2], fr[1]),
                                        lerp32(c[5] - c[4], c[7] - c[6], fr[1]), fr[2]);
                const float g1 = lerp32(c10 - c00, c11 - c01, fr[2]);
                const float g2 = lerp32(c01, c11, fr[1]) - lerp32(c00, c10, fr[1]);
                const float len = sqrtf((g0 * g0 + g1 * g1) + g2 * g2);
                const float inv = len > 0.0f ? 1.0f / len : qnan();
                const int g[3] = { v.off[0] + gx, v.off[1] + gy, v.off[2] + gz };
                const float gr[3] = { g0, g1, g2 };
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    V[3 * idx + q] = v.o[q] + v.s * (((float)g[q] + 0.5f) + fr[q]);
                    N[3 * idx + q] = gr[q] * inv;
                    if (G) G[3 * idx + q] = g[q];
                }
            }
        }
    }
}

int launch_extract(DevVolume v, uint32_t* counts, unsigned long long* offsets, long long* total, float* V,
                   float* N, int32_t* G, long long cap, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)v.bd[0] * v.bd[1] * v.bd[2];
    const unsigned blocks = (unsigned)std::min<size_t>(65536, (nb + 3) / 4);
    hipLaunchKernelGGL(mvf_extract_count_kernel, dim3(blocks), dim3(256), 0, s, v, nb, counts);
    hipLaunchKernelGGL(mvf_extract_scan_kernel, dim3(1), dim3(1024), 0, s, counts, nb, offsets, total);
    if (cap > 0)
        hipLaunchKernelGGL(mvf_extract_emit_kernel, dim3(blocks), dim3(256), 0, s, v, nb, offsets, V, N, G, cap);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Differentiable raycast on one dense x-fastest volume (F, W).  The forward
// is the same march (binary32 contract; validity from W), skipping bricks by
// a summary computed for the call; it records k of the crossing's second
// sample.  The backward
// recomputes the two bracketing samples from k, and with the structure held
// fixed scatters dL/dF (16 voxels per pixel, float atomics) and reduces
// dL/dxi per block into binary64 partials, summed by a second kernel in a
// fixed order (deterministic).
// ---------------------------------------------------------------------------
static __device__ __forceinline__ double lerp64(double a, double b, double t)
{
    return a * (1.0 - t) + b * t;
}

struct DSample {
    int i[3];
    float f[3];
    float c[8];
    float F;
    bool ok;
};

static __device__ __forceinline__ size_t dense_idx(const DiffVolume& v, int x, int y, int z)
{
    return ((size_t)z * v.dims[1] + y) * v.dims[0] + x;
}

static __device__ __forceinline__ void dense_sample(const DiffVolume& v, const Ray& r, float tk, DSample& S)
{
    S.ok = false;
    float l[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = r.C[a] + (tk * r.dw[a]);
        const float c = ((x - v.o[a]) * v.inv_s) - 0.5f;
        l[a] = c - (float)v.off[a];
        if (!(l[a] >= 0.0f && l[a] < (float)(v.dims[a] - 1))) return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float fl = floorf(l[a]);
        S.i[a] = (int)fl;
        S.f[a] = l[a] - fl;
    }
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const size_t id = dense_idx(v, S.i[0] + dx, S.i[1] + dy, S.i[2] + dz);
                if (v.W[id] == 0) return;
                S.c[dz * 4 + dy * 2 + dx] = v.F[id];
            }
    S.F = trilinear(S.c, S.f);
    S.ok = true;
}

static __device__ __forceinline__ void make_ray(int u, int v, float fx, float fy, float cx, float cy,
                                                const float* T, Ray& r, float dh[3])
{
    const float dc0 = ((float)u - cx) / fx;
    const float dc1 = ((float)v - cy) / fy;
    const float n = sqrtf(((dc0 * dc0) + (dc1 * dc1)) + (1.0f * 1.0f));
    const float inv_n = 1.0f / n;
    dh[0] = dc0 * inv_n;
    dh[1] = dc1 * inv_n;
    dh[2] = 1.0f * inv_n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.dw[a] = ((T[4 * a + 0] * dh[0]) + (T[4 * a + 1] * dh[1])) + (T[4 * a + 2] * dh[2]);
        r.C[a] = T[4 * a + 3];
    }
    r.t_lo = 0.0f;
    r.t_hi = INFINITY;
}

struct PoseArgs {
    float T[12];
};

__global__ __launch_bounds__(256) void mvf_diffray_backward_kernel(
    DiffVolume v, PoseArgs P, float fx, float fy, float cx, float cy, int width, int height, RayParams rp,
    const float* __restrict__ grad_depth, const int32_t* __restrict__ record, float* grad_F, double* partials)
{
    const int u = blockIdx.x * 16 + (threadIdx.x & 15);
    const int vv = blockIdx.y * 16 + (threadIdx.x >> 4);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (u < width && vv < height) {
        const size_t p = (size_t)vv * width + u;
        const int k = record[p];
        const float gd = grad_depth[p];
        if (k >= 1 && gd != 0.0f) {
            Ray r;
            float dh[3];
            make_ray(u, vv, fx, fy, cx, cy, P.T, r, dh);
            DSample S[2];
            dense_sample(v, r, (float)(k - 1) * rp.delta, S[0]);
            dense_sample(v, r, (float)k * rp.delta, S[1]);
            if (S[0].ok && S[1].ok) {
                // The binary32 march fixed the structure (k and the two
                // cells); the values are re-evaluated in binary64 at the
                // exact sample positions.  A crossing whose two samples are
                // close in value has dt/dF ~ 1 / (F_a - F_b)^2, so binary32
                // positions (an ulp of a local coordinate near 512 is 6e-5
                // voxel) would dominate the gradient of such pixels.
                double dh64[3], dw64[3];
                {
                    const double dc0 = ((double)u - (double)cx) / (double)fx;
                    const double dc1 = ((double)vv - (double)cy) / (double)fy;
                    const double n = sqrt(dc0 * dc0 + dc1 * dc1 + 1.0);
                    dh64[0] = dc0 / n;
                    dh64[1] = dc1 / n;
                    dh64[2] = 1.0 / n;
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        dw64[a] = (double)P.T[4 * a + 0] * dh64[0] + (double)P.T[4 * a + 1] * dh64[1] +
                                  (double)P.T[4 * a + 2] * dh64[2];
                }
                const double delta = (double)rp.delta;
                const double s64 = (double)v.s;
                double Fs[2], fr[2][3], gl[2][3];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double t = (double)(k - 1 + j) * delta;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const double x = (double)P.T[4 * a + 3] + t * dw64[a];
                        fr[j][a] = (x - (double)v.o[a]) / s64 - 0.5 - (double)v.off[a] - (double)S[j].i[a];
                    }
                    const float* c = S[j].c;
                    const double f0 = fr[j][0], f1 = fr[j][1], f2 = fr[j][2];
                    const double c00 = lerp64(c[0], c[1], f0), c10 = lerp64(c[2], c[3], f0);
                    const double c01 = lerp64(c[4], c[5], f0), c11 = lerp64(c[6], c[7], f0);
                    const double c0 = lerp64(c00, c10, f1), c1 = lerp64(c01, c11, f1);
                    gl[j][0] = lerp64(lerp64((double)c[1] - c[0], (double)c[3] - c[2], f1),
                                      lerp64((double)c[5] - c[4], (double)c[7] - c[6], f1), f2);
                    gl[j][1] = lerp64(c10 - c00, c11 - c01, f2);
                    gl[j][2] = c1 - c0;
                    Fs[j] = lerp64(c0, c1, f2);
                }
                const double den = Fs[0] - Fs[1];
                const double dt[2] = { -delta * Fs[1] / (den * den), delta * Fs[0] / (den * den) };
                const double gz = (double)gd * dh64[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double kk = gz * dt[j];
                    const double t = (double)(k - 1 + j) * delta;
                    double gc[3], q[3];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        gc[cc] = ((double)P.T[cc] * gl[j][0] + (double)P.T[4 + cc] * gl[j][1] +
                                  (double)P.T[8 + cc] * gl[j][2]) / s64;
                        q[cc] = t * dh64[cc];
                    }
                    acc[0] += kk * gc[0];
                    acc[1] += kk * gc[1];
                    acc[2] += kk * gc[2];
                    acc[3] += kk * (q[1] * gc[2] - q[2] * gc[1]);
                    acc[4] += kk * (q[2] * gc[0] - q[0] * gc[2]);
                    acc[5] += kk * (q[0] * gc[1] - q[1] * gc[0]);
                    if (grad_F) {
                        const DSample& sm = S[j];
#pragma unroll
                        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                                for (int dx = 0; dx < 2; ++dx) {
                                    const double w = (dx ? fr[j][0] : 1.0 - fr[j][0]) *
                                                     (dy ? fr[j][1] : 1.0 - fr[j][1]) *
                                                     (dz ? fr[j][2] : 1.0 - fr[j][2]);
                                    atomicAdd(&grad_F[dense_idx(v, sm.i[0] + dx, sm.i[1] + dy, sm.i[2] + dz)],
                                              (float)(kk * w));
                                }
                    }
                }
            }
        }
    }
    // deterministic block reduction of the 6 pose terms
    __shared__ double red[6][256];
#pragma unroll
    for (int i = 0; i < 6; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int stride = 128; stride >= 1; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
#pragma unroll
            for (int i = 0; i < 6; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + stride];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) {
        const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        partials[blk * 6 + threadIdx.x] = red[threadIdx.x][0];
    }
}

__global__ void mvf_reduce_partials_kernel(const double* partials, int nblocks, double* out)
{
    __shared__ double red[256];
    const int comp = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)b * 6 + comp];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int stride = 128; stride >= 1; stride >>= 1) {
        if ((int)threadIdx.x < stride) red[threadIdx.x] += red[threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[comp] = red[0];
}

int diffray_partials_needed(int width, int height)
{
    return ((width + 15) / 16) * ((height + 15) / 16);
}

// Static scratch of the allocation-free backward: the binary64 pose partials
// of up to kDiffScratchBlocks 16x16-pixel blocks.  Every block of a launch
// writes its own 6 entries before the reduction reads them, so nothing needs
// clearing between calls.  Each GPU holds its own copy, at its own address.
static __device__ __align__(256) double scratch[6 * kDiffScratchBlocks];

// Device addresses of `scratch`, one per device, taken once with that device
// current.  In host code the array's name is only a stand-in for the symbol.
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

int diffray_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[device] = static_cast<double*>(p);
    return 0;
}

double* diffray_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

int launch_diffray_backward(DiffVolume v, const float* T, float fx, float fy, float cx, float cy, int width,
                            int height, RayParams rp, const float* grad_depth, const int32_t* record,
                            float* grad_F, double* partials, int n_partials, double* grad_xi, void* stream)
{
    PoseArgs P;
    for (int i = 0; i < 12; ++i) P.T[i] = T[i];
    dim3 grid((width + 15) / 16, (height + 15) / 16);
    if ((int)(grid.x * grid.y) > n_partials) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(mvf_diffray_backward_kernel, grid, dim3(256), 0, (hipStream_t)stream, v, P, fx, fy, cx,
                       cy, width, height, rp, grad_depth, record, grad_F, partials);
    hipLaunchKernelGGL(mvf_reduce_partials_kernel, dim3(6), dim3(256), 0, (hipStream_t)stream, partials,
                       (int)(grid.x * grid.y), grad_xi);
    return (int)hipGetLastError();
}

}  // namespace mvf
