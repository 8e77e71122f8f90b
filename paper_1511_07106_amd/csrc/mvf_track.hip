// Camera tracking kernels for gfx950 (Depth Map Conversion and Camera
// Tracking sections of Salvato, Finman, Leonard, arXiv 1511.07106; the
// tracker is KinectFusion's projective point-to-plane ICP, which the paper
// cites).  Built with -ffp-contract=off and IEEE division/sqrt: every
// decision (pixel validity, the model pixel a vertex projects to, the
// distance and normal tests) is the binary32 contract of the CPU reference;
// residuals, Jacobians and the normal-equation sums are binary64.
//
// One Gauss-Newton step is two launches: the association kernel, whose
// blocks reduce their pairs' 6x6 system to binary64 partials, and a
// one-wavefront kernel that sums the partials in a fixed order, solves the
// system by Cholesky and moves the pose estimate, which stays in device
// memory.  A whole coarse-to-fine run is enqueued without a host round trip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mvf_internal.h"

namespace mvf {

static __device__ __forceinline__ bool depth_valid(float d) { return d > 0.0f && d <= 3.4e38f; }

static __device__ __forceinline__ float qnanf() { return __builtin_nanf(""); }

// Edge-preserving smoothing before the pyramid: for a valid pixel the
// binomial-weighted (C(6, dx + 3) C(6, dy + 3)) mean of the valid depths of
// its 7x7 window inside the image within delta of its own depth; invalid
// pixels give 0.  Binary32, the window row by row (the weights and their
// sums are small integers, exact).  A 16x16 tile of pixels reads its
// 22x22 neighbourhood from LDS.
__global__ __launch_bounds__(256) void mvf_track_smooth_kernel(const float* __restrict__ D, int pitch, int w, int h,
                                                               float delta, float* __restrict__ out)
{
    __shared__ float tile[22][23];
    const int x0 = blockIdx.x * 16 - 3, y0 = blockIdx.y * 16 - 3;
    for (int i = threadIdx.x; i < 22 * 22; i += 256) {
        const int ty = i / 22, tx = i - ty * 22;
        const int xx = x0 + tx, yy = y0 + ty;
        tile[ty][tx] = (xx >= 0 && xx < w && yy >= 0 && yy < h) ? D[(size_t)yy * pitch + xx] : 0.0f;
    }
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = blockIdx.x * 16 + lx, y = blockIdx.y * 16 + ly;
    if (x >= w || y >= h) return;
    const float d0 = tile[ly + 3][lx + 3];
    float r = 0.0f;
    if (depth_valid(d0)) {
        const float c6[7] = { 1.0f, 6.0f, 15.0f, 20.0f, 15.0f, 6.0f, 1.0f };
        float num = 0.0f, den = 0.0f;
        for (int dy = -3; dy <= 3; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= h) continue;
            for (int dx = -3; dx <= 3; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= w) continue;
                const float d = tile[ly + 3 + dy][lx + 3 + dx];
                if (!depth_valid(d) || !(fabsf(d - d0) <= delta)) continue;
                const float wt = c6[dx + 3] * c6[dy + 3];
                num = num + wt * d;
                den = den + wt;
            }
        }
        r = num / den;
    }
    out[(size_t)y * w + x] = r;
}

// Level l+1 depth (floor(w/2) x floor(h/2)): mean of the valid depths of the
// 2x2 block within tau of the block's first valid one (order (0,0), (1,0),
// (0,1), (1,1)), 0 when the block has none.
__global__ __launch_bounds__(256) void mvf_track_down_kernel(const float* __restrict__ D, int pitch, int w, int h,
                                                             float tau, float* __restrict__ D2)
{
    const int w2 = w / 2, h2 = h / 2;
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= w2 || y >= h2) return;
    const float q[4] = { D[(size_t)(2 * y) * pitch + 2 * x], D[(size_t)(2 * y) * pitch + 2 * x + 1],
                         D[(size_t)(2 * y + 1) * pitch + 2 * x], D[(size_t)(2 * y + 1) * pitch + 2 * x + 1] };
    bool have = false;
    float ref = 0.0f, sum = 0.0f;
    int n = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!depth_valid(q[k])) continue;
        if (!have) { ref = q[k]; have = true; }
        if (fabsf(q[k] - ref) <= tau) { sum = sum + q[k]; ++n; }
    }
    D2[(size_t)y * w2 + x] = n ? sum / (float)n : 0.0f;
}

static __device__ __forceinline__ void vertex_at(const float* D, int pitch, int x, int y, float fx, float fy,
                                                 float cx, float cy, float v[3])
{
    const float d = D[(size_t)y * pitch + x];
    if (!depth_valid(d)) { v[0] = v[1] = v[2] = qnanf(); return; }
    v[0] = (((float)x - cx) / fx) * d;
    v[1] = (((float)y - cy) / fy) * d;
    v[2] = d;
}

// Vertex map v = K^-1 [x y 1]^T D and normal map n = (v(x+1,y) - v(x,y)) x
// (v(x,y+1) - v(x,y)), normalised (camera frame, NaN where undefined).
__global__ __launch_bounds__(256) void mvf_track_vn_kernel(const float* __restrict__ D, int pitch, int w, int h,
                                                           float fx, float fy, float cx, float cy,
                                                           float* __restrict__ V, float* __restrict__ N)
{
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= w || y >= h) return;
    const size_t p = (size_t)y * w + x;
    float v00[3];
    vertex_at(D, pitch, x, y, fx, fy, cx, cy, v00);
    float n[3] = { qnanf(), qnanf(), qnanf() };
    if (!__builtin_isnan(v00[2]) && x + 1 < w && y + 1 < h) {
        float v10[3], v01[3];
        vertex_at(D, pitch, x + 1, y, fx, fy, cx, cy, v10);
        vertex_at(D, pitch, x, y + 1, fx, fy, cx, cy, v01);
        if (!__builtin_isnan(v10[2]) && !__builtin_isnan(v01[2])) {
            const float a[3] = { v10[0] - v00[0], v10[1] - v00[1], v10[2] - v00[2] };
            const float b[3] = { v01[0] - v00[0], v01[1] - v00[1], v01[2] - v00[2] };
            const float c[3] = { (a[1] * b[2]) - (a[2] * b[1]), (a[2] * b[0]) - (a[0] * b[2]),
                                 (a[0] * b[1]) - (a[1] * b[0]) };
            const float len = sqrtf(((c[0] * c[0]) + (c[1] * c[1])) + (c[2] * c[2]));
            if (len > 0.0f) {
                n[0] = c[0] / len;
                n[1] = c[1] / len;
                n[2] = c[2] / len;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        V[3 * p + a] = v00[a];
        N[3 * p + a] = n[a];
    }
}

// Model maps of level l+1: the sample (2x, 2y) of level l.
__global__ __launch_bounds__(256) void mvf_track_model_down_kernel(const float* __restrict__ V,
                                                                   const float* __restrict__ N, int w, int h,
                                                                   float* __restrict__ V2, float* __restrict__ N2)
{
    const int w2 = w / 2, h2 = h / 2;
    const int x = blockIdx.x * 16 + (threadIdx.x & 15);
    const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (x >= w2 || y >= h2) return;
    const size_t s = (size_t)(2 * y) * w + 2 * x, d = (size_t)y * w2 + x;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        V2[3 * d + a] = V[3 * s + a];
        N2[3 * d + a] = N[3 * s + a];
    }
}

// One association pass over the current maps (w x h): per block the sums
// of its pairs (A upper triangle 21, b 6, pairs, sum r^2) into
// partials[block * kTrackSums ...], in a fixed order.
__global__ __launch_bounds__(kTrackThreads) void mvf_icp_reduce_kernel(TrackLaunch L)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    double acc[kTrackSums];
#pragma unroll
    for (int i = 0; i < kTrackSums; ++i) acc[i] = 0.0;
    const float* T = L.state->T32;
    const float* Tm = L.Tm;
    const float e2 = L.eps_d * L.eps_d;
    const int npix = L.w * L.h;
    const int base = blockIdx.x * kTrackThreads * kTrackPixPerThread;
    for (int k = 0; k < kTrackPixPerThread; ++k) {
        const int p = base + k * kTrackThreads + (int)threadIdx.x;
        if (p >= npix) break;
        if (L.inlier) L.inlier[p] = 0;
        const float v[3] = { L.V[3 * p], L.V[3 * p + 1], L.V[3 * p + 2] };
        const float n[3] = { L.N[3 * p], L.N[3 * p + 1], L.N[3 * p + 2] };
        if (__builtin_isnan(v[0]) || __builtin_isnan(v[1]) || __builtin_isnan(v[2]) || __builtin_isnan(n[0]) ||
            __builtin_isnan(n[1]) || __builtin_isnan(n[2]))
            continue;
        float vg[3], ng[3], d[3], q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            vg[a] = (((T[4 * a] * v[0]) + (T[4 * a + 1] * v[1])) + (T[4 * a + 2] * v[2])) + T[4 * a + 3];
            ng[a] = ((T[4 * a] * n[0]) + (T[4 * a + 1] * n[1])) + (T[4 * a + 2] * n[2]);
            d[a] = vg[a] - Tm[4 * a + 3];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = ((Tm[a] * d[0]) + (Tm[4 + a] * d[1])) + (Tm[8 + a] * d[2]);
        if (!(q[2] > 0.0f)) continue;
        const float iz = 1.0f / q[2];
        const float ur = floorf((((L.fx * q[0]) * iz) + L.cx) + 0.5f);
        const float vr = floorf((((L.fy * q[1]) * iz) + L.cy) + 0.5f);
        if (!(ur >= 0.0f && ur <= (float)(L.w - 1) && vr >= 0.0f && vr <= (float)(L.h - 1))) continue;
        const size_t m = (size_t)vr * L.w + (size_t)ur;
        const float vm[3] = { L.Vm[3 * m], L.Vm[3 * m + 1], L.Vm[3 * m + 2] };
        const float nm[3] = { L.Nm[3 * m], L.Nm[3 * m + 1], L.Nm[3 * m + 2] };
        if (__builtin_isnan(vm[0]) || __builtin_isnan(vm[1]) || __builtin_isnan(vm[2]) || __builtin_isnan(nm[0]) ||
            __builtin_isnan(nm[1]) || __builtin_isnan(nm[2]))
            continue;
        const float dv[3] = { vg[0] - vm[0], vg[1] - vm[1], vg[2] - vm[2] };
        const float dist2 = ((dv[0] * dv[0]) + (dv[1] * dv[1])) + (dv[2] * dv[2]);
        if (!(dist2 <= e2)) continue;
        const float dot = ((ng[0] * nm[0]) + (ng[1] * nm[1])) + (ng[2] * nm[2]);
        if (!(fabsf(dot) >= L.cos_theta)) continue;
        if (L.inlier) L.inlier[p] = 1;
        const double g[3] = { vg[0], vg[1], vg[2] };
        const double nn[3] = { nm[0], nm[1], nm[2] };
        const double r = nn[0] * (g[0] - (double)vm[0]) + nn[1] * (g[1] - (double)vm[1]) +
                         nn[2] * (g[2] - (double)vm[2]);
        const double J[6] = { nn[0], nn[1], nn[2], g[1] * nn[2] - g[2] * nn[1], g[2] * nn[0] - g[0] * nn[2],
                              g[0] * nn[1] - g[1] * nn[0] };
        int kk = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) acc[kk++] += J[i] * J[j];
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * r;
        acc[27] += 1.0;
        acc[28] += r * r;
    }
    // wavefront tree (fixed pairing), then the block's waves in order
#pragma unroll
    for (int i = 0; i < kTrackSums; ++i) {
        double x = acc[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_down(x, o, 64);
        acc[i] = x;
    }
    __shared__ double part[kTrackThreads / 64][kTrackSums];
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kTrackSums; ++i) part[wave][i] = acc[i];
    }
    __syncthreads();
    if (threadIdx.x < kTrackSums) {
        double s = 0.0;
#pragma unroll
        for (int wv = 0; wv < kTrackThreads / 64; ++wv) s += part[wv][threadIdx.x];
        L.partials[(size_t)blockIdx.x * kTrackSums + threadIdx.x] = s;
    }
}

// Left-multiplied SE(3) exponential Exp(xi) T, xi = (rho, omega), binary64.
static __device__ void se3_left_update(const double xi[6], double T[12])
{
    const double w0 = xi[3], w1 = xi[4], w2 = xi[5];
    const double th = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    const double W[9] = { 0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0 };
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
    double a, b, c;
    if (th < 1e-10) {
        a = 1.0;
        b = 0.5;
        c = 1.0 / 6.0;
    } else {
        const double s = sin(th), co = cos(th);
        a = s / th;
        b = (1.0 - co) / (th * th);
        c = (th - s) / (th * th * th);
    }
    double R[9], Vm[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + a * W[i] + b * W2[i];
        Vm[i] = I + b * W[i] + c * W2[i];
    }
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = Vm[3 * i] * xi[0] + Vm[3 * i + 1] * xi[1] + Vm[3 * i + 2] * xi[2];
    double out[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            out[4 * i + j] = R[3 * i] * T[j] + R[3 * i + 1] * T[4 + j] + R[3 * i + 2] * T[8 + j];
        out[4 * i + 3] = R[3 * i] * T[3] + R[3 * i + 1] * T[7] + R[3 * i + 2] * T[11] + t[i];
    }
    for (int i = 0; i < 12; ++i) T[i] = out[i];
}

// Sum of the partials (fixed order), the step's statistics, and the
// Gauss-Newton update: solve A xi = -b by Cholesky, T <- Exp(xi) T.  Fewer
// than 6 pairs, or an A that is not positive definite, leave T as it is.
// One wavefront.
__global__ __launch_bounds__(64) void mvf_icp_solve_kernel(const double* __restrict__ partials, int nblocks,
                                                           TrackState* state, int step)
{
    __shared__ double tot[kTrackSums];
    const int lane = threadIdx.x;
    if (lane < kTrackSums) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[(size_t)b * kTrackSums + lane];
        tot[lane] = s;
    }
    __syncthreads();
    if (lane != 0) return;
    const int pairs = (int)tot[27];
    state->pairs[step] = pairs;
    state->sq_err[step] = tot[28];
    state->steps = step + 1;
    if (pairs < 6) return;
    double A[6][6], L[6][6], y[6], xi[6];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) { A[i][j] = tot[k]; A[j][i] = tot[k]; ++k; }
    for (int j = 0; j < 6; ++j) {
        double s = A[j][j];
        for (int q = 0; q < j; ++q) s -= L[j][q] * L[j][q];
        if (!(s > 0.0)) return;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = A[i][j];
            for (int q = 0; q < j; ++q) t -= L[i][q] * L[j][q];
            L[i][j] = t / L[j][j];
        }
    }
    for (int i = 0; i < 6; ++i) {
        double s = -tot[21 + i];
        for (int q = 0; q < i; ++q) s -= L[i][q] * y[q];
        y[i] = s / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int q = i + 1; q < 6; ++q) s -= L[q][i] * xi[q];
        xi[i] = s / L[i][i];
    }
    se3_left_update(xi, state->T);
    for (int i = 0; i < 12; ++i) state->T32[i] = (float)state->T[i];
}

// The estimate's binary32 copy from its binary64 value (first step).
__global__ void mvf_track_init_kernel(TrackState* state)
{
    if (threadIdx.x < 12) state->T32[threadIdx.x] = (float)state->T[threadIdx.x];
    if (threadIdx.x == 0) state->steps = 0;
}

int launch_track_smooth(const float* D, int pitch, int w, int h, float delta, float* out, void* stream)
{
    dim3 grid((w + 15) / 16, (h + 15) / 16);
    hipLaunchKernelGGL(mvf_track_smooth_kernel, grid, dim3(256), 0, (hipStream_t)stream, D, pitch, w, h, delta, out);
    return (int)hipGetLastError();
}

int launch_track_down(const float* D, int pitch, int w, int h, float tau, float* D2, void* stream)
{
    dim3 grid((w / 2 + 15) / 16, (h / 2 + 15) / 16);
    if (grid.x == 0 || grid.y == 0) return 0;
    hipLaunchKernelGGL(mvf_track_down_kernel, grid, dim3(256), 0, (hipStream_t)stream, D, pitch, w, h, tau, D2);
    return (int)hipGetLastError();
}

int launch_track_vn(const float* D, int pitch, int w, int h, const float K[4], float* V, float* N, void* stream)
{
    dim3 grid((w + 15) / 16, (h + 15) / 16);
    hipLaunchKernelGGL(mvf_track_vn_kernel, grid, dim3(256), 0, (hipStream_t)stream, D, pitch, w, h, K[0], K[1],
                       K[2], K[3], V, N);
    return (int)hipGetLastError();
}

int launch_track_model_down(const float* V, const float* N, int w, int h, float* V2, float* N2, void* stream)
{
    dim3 grid((w / 2 + 15) / 16, (h / 2 + 15) / 16);
    if (grid.x == 0 || grid.y == 0) return 0;
    hipLaunchKernelGGL(mvf_track_model_down_kernel, grid, dim3(256), 0, (hipStream_t)stream, V, N, w, h, V2, N2);
    return (int)hipGetLastError();
}

int track_blocks(int w, int h)
{
    return (w * h + kTrackThreads * kTrackPixPerThread - 1) / (kTrackThreads * kTrackPixPerThread);
}

int launch_icp_step(const TrackLaunch& L, TrackState* state, int step, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    const int nb = track_blocks(L.w, L.h);
    if (nb > 0) hipLaunchKernelGGL(mvf_icp_reduce_kernel, dim3(nb), dim3(kTrackThreads), 0, s, L);
    hipLaunchKernelGGL(mvf_icp_solve_kernel, dim3(1), dim3(64), 0, s, (const double*)L.partials, nb, state, step);
    return (int)hipGetLastError();
}

int launch_track_init(TrackState* state, void* stream)
{
    hipLaunchKernelGGL(mvf_track_init_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, state);
    return (int)hipGetLastError();
}

}  // namespace mvf
