/*
 * mvf_oracle.c -- CPU oracle for multi-volume TSDF mapping.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or helper with the HIP library; the two are compared on the
 * same seeded inputs.
 *
 * Paper: Salvato, Finman, Leonard, "Multi-Volume High Resolution RGB-D
 * Mapping with Dynamic Volume Placement" (arXiv 1511.07106).
 *
 * Precision.  The paper fixes no precision.  Every step whose floating-point
 * result decides an integer (which voxel is touched, which pixel it projects
 * to, whether the weight grows, which ray sample holds the zero crossing,
 * which placement cell a ray endpoint falls in) is evaluated in IEEE binary32
 * with one rounding per written operation, in the written order, with no
 * fused multiply-add (build with -ffp-contract=off, never -ffast-math).
 * Values that are not decisions (the stored TSDF, raycast depth, vertex,
 * normal, gradients) are carried in binary64.
 *
 * Layouts.  A volume of dims (nx, ny, nz) is stored x-fastest:
 * index(x, y, z) = (z * ny + y) * nx + x.  Colour is RGBA8 per voxel with A
 * the colour weight.  Poses are row-major 3x4 camera-to-world [R | t]
 * (OpenCV camera axes).  Intrinsics are (fx, fy, cx, cy); pixel (u, v) has
 * its centre at integer coordinates.  The world grid has origin o and voxel
 * size s; global voxel g has its centre at o + s (g + 1/2); a volume covers
 * the global voxels [h_t, h_t + dims).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_AMBIG_F 1e-5f       /* |F| below this makes a sign test ambiguous */
#define ORC_AMBIG_DF 1e-3f      /* F_a - F_b below this makes t* ill conditioned */

/* Cell whose trilinear patch gives the raycast normal.  1 (the reading
 * taken): the cell of the crossing's second sample, evaluated at the
 * vertex.  0 (the first sample's cell) and 2 (the vertex's own cell, clamped
 * into the volume) are alternative readings, compiled only by the test that
 * shows its pin tells the three apart. */
#ifndef ORC_NORMAL_CELL
#define ORC_NORMAL_CELL 1
#endif

static inline int64_t vidx(const int32_t* dims, int x, int y, int z) {
    return ((int64_t)z * dims[1] + y) * dims[0] + x;
}

/* ------------------------------------------------------------------------
 * Volumetric integration (Volumetric Integration section; Algorithm 1, the
 * per-voxel loop).  Every voxel is visited; each is independent of all
 * others (Comparison to KinectFusion section).
 *
 * Readings of the paper taken here:
 *  - the voxel coordinate used is the global index t_s = t_l + h_t;
 *  - dist compares ranges: the measured depth along the pixel ray (z-depth
 *    times the ray length factor lambda) minus the distance from the current
 *    camera centre to the voxel centre;
 *  - the pixel is the nearest one, floor(x + 1/2); invalid depths (<= 0,
 *    NaN, inf) and pixels outside the image give no update;
 *  - truncation mu = trunc_voxels * s: voxels more than mu behind the
 *    measured surface are not updated, the stored value is min(1, dist/mu);
 *  - the per-observation weight is 1 and the running weight is capped at
 *    w_max ("linearly increasing up to some maximum");
 *  - colour (not described in the paper) is a rounded running mean in the
 *    band |dist| <= mu, with its own weight capped at 255.
 * ------------------------------------------------------------------------ */
int orc_integrate(const int32_t dims[3], const int32_t off[3],
                  const float grid[5], /* ox, oy, oz, s, trunc_voxels */
                  int w_max, double* F, uint16_t* W, uint8_t* C,
                  const float* depth, const uint8_t* rgb, int width, int height,
                  const float K[4], const float T[12], int64_t stats[3])
{
    const float s = grid[3];
    const float mu = grid[4] * s;
    const float fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    int64_t n_in_image = 0, n_updated = 0, n_band = 0;
    if (w_max < 1 || w_max > 65535) return 1;

#pragma omp parallel for schedule(dynamic, 1) reduction(+:n_in_image, n_updated, n_band)
    for (int z = 0; z < dims[2]; ++z) {
        for (int y = 0; y < dims[1]; ++y) {
            for (int x = 0; x < dims[0]; ++x) {
                /* global voxel index and its centre in the world */
                const int32_t g[3] = { off[0] + x, off[1] + y, off[2] + z };
                float xw[3], d[3], p[3];
                for (int a = 0; a < 3; ++a) xw[a] = grid[a] + (s * ((float)g[a] + 0.5f));
                /* camera-frame position p = R^T (xw - t) */
                for (int a = 0; a < 3; ++a) d[a] = xw[a] - T[4 * a + 3];
                for (int c = 0; c < 3; ++c)
                    p[c] = ((T[0 * 4 + c] * d[0]) + (T[1 * 4 + c] * d[1])) + (T[2 * 4 + c] * d[2]);
                if (!(p[2] > 0.0f)) continue;
                /* back-projection to the nearest pixel */
                const float iz = 1.0f / p[2];
                const float uf = ((fx * p[0]) * iz) + cx;
                const float vf = ((fy * p[1]) * iz) + cy;
                const float ur = floorf(uf + 0.5f);
                const float vr = floorf(vf + 0.5f);
                if (!(ur >= 0.0f && ur < (float)width && vr >= 0.0f && vr < (float)height)) continue;
                const int u = (int)ur, v = (int)vr;
                const float Dz = depth[(int64_t)v * width + u];
                if (!(Dz > 0.0f && Dz < INFINITY)) continue;
                ++n_in_image;
                /* measured range along the pixel ray minus the voxel's range */
                const float ra = ((float)u - cx) / fx;
                const float rb = ((float)v - cy) / fy;
                const float lam = sqrtf(((ra * ra) + (rb * rb)) + 1.0f);
                const float rho = sqrtf(((p[0] * p[0]) + (p[1] * p[1])) + (p[2] * p[2]));
                const float sdf = (Dz * lam) - rho;
                if (sdf < -mu) continue;
                ++n_updated;
                /* running weighted average, per-observation weight 1 */
                const int64_t i = vidx(dims, x, y, z);
                const double phi = fmin(1.0, (double)sdf / (double)mu);
                const double Wf = (double)W[i];
                F[i] = (F[i] * Wf + phi) / (Wf + 1.0);
                W[i] = (uint16_t)((int)W[i] + 1 < w_max ? (int)W[i] + 1 : w_max);
                if (sdf <= mu) {
                    ++n_band;
                    if (rgb) {
                        uint8_t* c4 = C + 4 * i;
                        const uint32_t A = c4[3];
                        const uint8_t* obs = rgb + 3 * ((int64_t)v * width + u);
                        for (int ch = 0; ch < 3; ++ch)
                            c4[ch] = (uint8_t)(((uint32_t)c4[ch] * A + obs[ch] + ((A + 1u) >> 1)) / (A + 1u));
                        c4[3] = (uint8_t)(A + 1u < 255u ? A + 1u : 255u);
                    }
                }
            }
        }
    }
    if (stats) { stats[0] = n_in_image; stats[1] = n_updated; stats[2] = n_band; }
    return 0;
}

/* ------------------------------------------------------------------------
 * Raycasting (Raycasting section; Algorithm 1, the per-pixel loop).
 *
 * Readings taken here: rays sample a global lattice t_k = k * delta from the
 * camera centre, delta = step * s with step < 1; a sample is in a volume's
 * domain when its local continuous voxel coordinate l satisfies
 * 0 <= l < dims - 1 on every axis, and valid when all 8 voxels of its cell
 * have weight > 0; the value is the trilinear interpolant (x, then y, then
 * z, with lerp(a, b, t) = a (1 - t) + b t); a surface is the first pair of
 * consecutive valid samples going from F > 0 to F <= 0 (front faces only);
 * its distance is the linear interpolation between the two samples; the
 * normal is the gradient, at the vertex, of the trilinear interpolant of the
 * cell holding the crossing's second sample (a cell whose 8 voxels are all
 * observed, so the normal never reads an unobserved voxel); across volumes
 * the smallest distance wins (ties: lower volume index), as the shared-map
 * rule of the Raycasting section requires.
 * ------------------------------------------------------------------------ */

typedef struct {
    const int32_t* dims;
    const int32_t* off;
    const float* F;
    const uint16_t* W;
} orc_vol;

/* binary32 lerp in the stated form */
static inline float lerp32(float a, float b, float t) { return (a * (1.0f - t)) + (b * t); }
static inline double lerp64(double a, double b, double t) { return a * (1.0 - t) + b * t; }

/* Trilinear sample in binary32 at local coordinate l (already in domain).
 * Returns 0 if some corner has W == 0, else 1 with *out and the cell. */
static int sample32(const orc_vol* v, const float l[3], float* out, int cell[3])
{
    float f[3];
    for (int a = 0; a < 3; ++a) {
        const float fl = floorf(l[a]);
        cell[a] = (int)fl;
        f[a] = l[a] - fl;
    }
    float c[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int64_t i = vidx(v->dims, cell[0] + dx, cell[1] + dy, cell[2] + dz);
                if (v->W[i] == 0) return 0;
                c[dz][dy][dx] = v->F[i];
            }
    const float c00 = lerp32(c[0][0][0], c[0][0][1], f[0]);
    const float c10 = lerp32(c[0][1][0], c[0][1][1], f[0]);
    const float c01 = lerp32(c[1][0][0], c[1][0][1], f[0]);
    const float c11 = lerp32(c[1][1][0], c[1][1][1], f[0]);
    const float c0 = lerp32(c00, c10, f[1]);
    const float c1 = lerp32(c01, c11, f[1]);
    *out = lerp32(c0, c1, f[2]);
    return 1;
}

/* Trilinear value and gradient (w.r.t. the local voxel coordinate) in
 * binary64 at fraction f inside the given cell; optional corner weights
 * wts[dz][dy][dx]. */
static double sample64(const orc_vol* v, const int cell[3], const double f[3],
                       double grad[3], double wts[8])
{
    double c[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                c[dz][dy][dx] = (double)v->F[vidx(v->dims, cell[0] + dx, cell[1] + dy, cell[2] + dz)];
    const double c00 = lerp64(c[0][0][0], c[0][0][1], f[0]);
    const double c10 = lerp64(c[0][1][0], c[0][1][1], f[0]);
    const double c01 = lerp64(c[1][0][0], c[1][0][1], f[0]);
    const double c11 = lerp64(c[1][1][0], c[1][1][1], f[0]);
    const double c0 = lerp64(c00, c10, f[1]);
    const double c1 = lerp64(c01, c11, f[1]);
    if (grad) {
        /* d/dfx: differences along x, interpolated in y then z */
        const double gx0 = lerp64(c[0][0][1] - c[0][0][0], c[0][1][1] - c[0][1][0], f[1]);
        const double gx1 = lerp64(c[1][0][1] - c[1][0][0], c[1][1][1] - c[1][1][0], f[1]);
        grad[0] = lerp64(gx0, gx1, f[2]);
        grad[1] = lerp64(c10 - c00, c11 - c01, f[2]);
        grad[2] = c1 - c0;
    }
    if (wts) {
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    wts[dz * 4 + dy * 2 + dx] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1])
                                              * (dz ? f[2] : 1.0 - f[2]);
    }
    return lerp64(c0, c1, f[2]);
}

/* Per-pixel camera ray in binary32: unit direction in the camera frame and
 * in the world frame. */
static void pixel_ray32(int u, int v, const float K[4], const float T[12],
                        float dhat[3], float dw[3])
{
    const float dc[3] = { ((float)u - K[2]) / K[0], ((float)v - K[3]) / K[1], 1.0f };
    const float n = sqrtf(((dc[0] * dc[0]) + (dc[1] * dc[1])) + (dc[2] * dc[2]));
    const float inv_n = 1.0f / n;
    for (int a = 0; a < 3; ++a) dhat[a] = dc[a] * inv_n;
    for (int r = 0; r < 3; ++r)
        dw[r] = ((T[4 * r + 0] * dhat[0]) + (T[4 * r + 1] * dhat[1])) + (T[4 * r + 2] * dhat[2]);
}

static void pixel_ray64(int u, int v, const float K[4], const double T[12],
                        double dhat[3], double dw[3])
{
    const double dc[3] = { ((double)u - K[2]) / K[0], ((double)v - K[3]) / K[1], 1.0 };
    const double n = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    for (int a = 0; a < 3; ++a) dhat[a] = dc[a] / n;
    for (int r = 0; r < 3; ++r)
        dw[r] = T[4 * r + 0] * dhat[0] + T[4 * r + 1] * dhat[1] + T[4 * r + 2] * dhat[2];
}

/* Conservative sample-index range for the ray inside a volume's domain box
 * (grown by one voxel, plus two samples each side).  Only limits the walk;
 * the exact domain test is made per sample. */
static void k_range(const orc_vol* v, const float grid[4], const float C[3],
                    const float dw[3], double delta, int kmax, int* k0, int* k1)
{
    double t0 = 0.0, t1 = (double)kmax * delta;
    for (int a = 0; a < 3; ++a) {
        const double s = grid[3];
        const double lo = grid[a] + s * ((double)v->off[a] + 0.5) - s;
        const double hi = grid[a] + s * ((double)v->off[a] + (double)v->dims[a] - 0.5) + s;
        if (dw[a] == 0.0f) {
            if ((double)C[a] < lo || (double)C[a] > hi) { *k0 = 1; *k1 = 0; return; }
            continue;
        }
        double ta = (lo - C[a]) / dw[a], tb = (hi - C[a]) / dw[a];
        if (ta > tb) { const double t = ta; ta = tb; tb = t; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (t0 > t1) { *k0 = 1; *k1 = 0; return; }
    int a0 = (int)floor(t0 / delta) - 2, a1 = (int)ceil(t1 / delta) + 2;
    *k0 = a0 < 1 ? 1 : a0;
    *k1 = a1 > kmax ? kmax : a1;
}

/* Result of the binary32 march in one volume. */
typedef struct {
    int found, k;          /* crossing between samples k-1 and k */
    float tstar;           /* binary32 crossing distance */
    int cell_a[3], cell_b[3];
    int ambiguous;
} orc_hit;

static void march_volume(const orc_vol* v, const float grid[4], const float C[3],
                         const float dw[3], float delta, int kmax, orc_hit* h)
{
    const float inv_s = 1.0f / grid[3];
    int k0, k1;
    memset(h, 0, sizeof(*h));
    k_range(v, grid, C, dw, (double)delta, kmax, &k0, &k1);
    int prev_ok = 0;
    float Fprev = 0.0f;
    int cprev[3] = {0, 0, 0};
    for (int k = k0; k <= k1; ++k) {
        const float tk = (float)k * delta;
        float l[3];
        int in = 1;
        for (int a = 0; a < 3; ++a) {
            const float x = C[a] + (tk * dw[a]);
            const float c = ((x - grid[a]) * inv_s) - 0.5f;
            l[a] = c - (float)v->off[a];
            if (!(l[a] >= 0.0f && l[a] < (float)(v->dims[a] - 1))) in = 0;
        }
        float Fk;
        int cell[3];
        if (!in || !sample32(v, l, &Fk, cell)) { prev_ok = 0; continue; }
        if (fabsf(Fk) < ORC_AMBIG_F) h->ambiguous = 1;
        if (prev_ok && Fprev > 0.0f && Fk <= 0.0f) {
            const float ta = (float)(k - 1) * delta;
            h->found = 1;
            h->k = k;
            h->tstar = ta + ((delta * Fprev) / (Fprev - Fk));
            if (Fprev - Fk < ORC_AMBIG_DF) h->ambiguous = 1;
            memcpy(h->cell_a, cprev, sizeof(cprev));
            memcpy(h->cell_b, cell, sizeof(cell));
            return;
        }
        prev_ok = 1;
        Fprev = Fk;
        memcpy(cprev, cell, sizeof(cell));
    }
}

/* Binary64 evaluation of a pixel's crossing in volume v between samples
 * k-1 and k with the cells fixed; pose given in binary64. */
static double eval_crossing64(const orc_vol* v, const float grid[4], double delta,
                              const double C[3], const double dw[3], int k,
                              const int cell_a[3], const int cell_b[3],
                              double* Fa_out, double* Fb_out)
{
    double Fab[2];
    for (int j = 0; j < 2; ++j) {
        const double t = (double)(k - 1 + j) * delta;
        const int* cell = j ? cell_b : cell_a;
        double f[3];
        for (int a = 0; a < 3; ++a) {
            const double x = C[a] + t * dw[a];
            const double l = (x - grid[a]) / (double)grid[3] - 0.5 - (double)v->off[a];
            f[a] = l - (double)cell[a];
        }
        Fab[j] = sample64(v, cell, f, NULL, NULL);
    }
    if (Fa_out) *Fa_out = Fab[0];
    if (Fb_out) *Fb_out = Fab[1];
    return (double)(k - 1) * delta + delta * Fab[0] / (Fab[0] - Fab[1]);
}

/*
 * orc_raycast: multi-volume raycast of one view.
 *  vols: nvol volumes; dims/offs are nvol x 3; F (binary32, the stored TSDF
 *  rounded to the storage type) and W are concatenated, volume j starting at
 *  element base[j].
 *  Outputs per pixel (row-major H x W): depth (camera z, 0 when no hit),
 *  vertex and normal (world, x3, NaN when no hit), hit volume index (-1),
 *  k of the crossing's second sample (-1), the binary32 crossing distance,
 *  the cells of the two samples (6 ints) and of the normal (3 ints), and an
 *  ambiguity flag (a sign test with |F| < 1e-5 or F_a - F_b < 1e-3 on the
 *  winning ray).
 */
int orc_raycast(int nvol, const int32_t* dims, const int32_t* offs,
                const float* Fcat, const uint16_t* Wcat, const int64_t* base,
                const float grid[4], float step, float t_far,
                const float K[4], const float T[12], int width, int height,
                double* depth, double* vertex, double* normal,
                int32_t* hit_vol, int32_t* hit_k, float* tstar32,
                int32_t* cells, uint8_t* ambiguous)
{
    if (!(step > 0.0f && step < 1.0f)) return 1;
    const float delta = step * grid[3];
    const int kmax = (int)floorf(t_far / delta);
    double T64[12];
    for (int i = 0; i < 12; ++i) T64[i] = (double)T[i];

#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < height; ++v) {
        for (int u = 0; u < width; ++u) {
            const int64_t p = (int64_t)v * width + u;
            float dhat[3], dw[3];
            pixel_ray32(u, v, K, T, dhat, dw);
            const float C[3] = { T[3], T[7], T[11] };
            int best = -1;
            orc_hit hb;
            int amb = 0;
            for (int j = 0; j < nvol; ++j) {
                const orc_vol vol = { dims + 3 * j, offs + 3 * j, Fcat + base[j], Wcat + base[j] };
                orc_hit h;
                march_volume(&vol, grid, C, dw, delta, kmax, &h);
                if (h.ambiguous) amb = 1;
                if (h.found && (best < 0 || h.tstar < hb.tstar)) { best = j; hb = h; }
            }
            hit_vol[p] = best;
            ambiguous[p] = (uint8_t)amb;
            if (best < 0) {
                depth[p] = 0.0;
                for (int a = 0; a < 3; ++a) vertex[3 * p + a] = normal[3 * p + a] = NAN;
                hit_k[p] = -1;
                tstar32[p] = 0.0f;
                for (int a = 0; a < 9; ++a) cells[9 * p + a] = -1;
                continue;
            }
            const orc_vol vol = { dims + 3 * best, offs + 3 * best, Fcat + base[best], Wcat + base[best] };
            hit_k[p] = hb.k;
            tstar32[p] = hb.tstar;
            /* binary64 outputs with the structure fixed */
            double dh64[3], dw64[3];
            pixel_ray64(u, v, K, T64, dh64, dw64);
            const double C64[3] = { T64[3], T64[7], T64[11] };
            const double ts = eval_crossing64(&vol, grid, (double)delta, C64, dw64, hb.k,
                                              hb.cell_a, hb.cell_b, NULL, NULL);
            depth[p] = ts * dh64[2];
            double lv[3];
            for (int a = 0; a < 3; ++a) {
                const double x = C64[a] + ts * dw64[a];
                vertex[3 * p + a] = x;
                lv[a] = (x - grid[a]) / (double)grid[3] - 0.5 - (double)vol.off[a];
            }
            /* the normal is the gradient of the trilinear patch of the cell of
             * the crossing's second sample, whose 8 voxels are all observed,
             * evaluated at the vertex (which may lie just outside that cell:
             * the patch is then extended linearly in each coordinate) */
            int cv[3];
            for (int a = 0; a < 3; ++a) {
#if ORC_NORMAL_CELL == 0
                cv[a] = hb.cell_a[a];
#elif ORC_NORMAL_CELL == 2
                int c = (int)floor(lv[a]);
                cv[a] = c < 0 ? 0 : (c > vol.dims[a] - 2 ? vol.dims[a] - 2 : c);
#else
                cv[a] = hb.cell_b[a];
#endif
                cells[9 * p + a] = hb.cell_a[a];
                cells[9 * p + 3 + a] = hb.cell_b[a];
                cells[9 * p + 6 + a] = cv[a];
            }
            double f[3], g[3];
            for (int a = 0; a < 3; ++a) f[a] = lv[a] - (double)cv[a];
            sample64(&vol, cv, f, g, NULL);
            const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            for (int a = 0; a < 3; ++a) normal[3 * p + a] = gn > 0.0 ? g[a] / gn : NAN;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Depth of a pixel as a function of the pose with the discrete structure
 * (crossing index, sample cells) held fixed: the binary64 forward whose
 * derivative the differentiable raycast computes.  One volume.
 *   T64: pose (binary64).  k_cells: per pixel k then cell_a, cell_b (7 ints),
 *   k < 0 for no hit.  depth_out: per pixel (0 for no hit).
 * ------------------------------------------------------------------------ */
int orc_depth_fixed(const int32_t dims[3], const int32_t off[3], const float* F,
                    const uint16_t* W, const float grid[4], float step,
                    const float K[4], const double T64[12], int width, int height,
                    const int32_t* k_cells, double* depth_out)
{
    const orc_vol vol = { dims, off, F, W };
    const double delta = (double)(step * grid[3]);
    const double C[3] = { T64[3], T64[7], T64[11] };
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < height; ++v) {
        for (int u = 0; u < width; ++u) {
            const int64_t p = (int64_t)v * width + u;
            const int32_t* kc = k_cells + 7 * p;
            if (kc[0] < 0) { depth_out[p] = 0.0; continue; }
            double dh[3], dw[3];
            pixel_ray64(u, v, K, T64, dh, dw);
            const double ts = eval_crossing64(&vol, grid, delta, C, dw, kc[0], kc + 1, kc + 4, NULL, NULL);
            depth_out[p] = ts * dh[2];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Analytic gradient of L = sum_p gd[p] * z_p (gd = dL/dz per pixel) with
 * respect to a right perturbation xi = (rho, omega) of the pose,
 * T(xi) = T Exp(xi), at xi = 0, and with respect to the voxel values.
 * Structure fixed as in orc_depth_fixed.  grad_F (dense, x-fastest) is
 * accumulated; it may be NULL.
 *
 * For a sample at camera-frame point q = t dhat: x = R q + C, so
 * dx/drho = R and dx/domega = -R [q]x; with g the world gradient of F at x
 * and g_c = R^T g: dF/drho = g_c and dF/domega = q x g_c.  With
 * t* = t_a + delta F_a / (F_a - F_b): d(t*)/d(F_a) = -delta F_b / (F_a - F_b)^2,
 * d(t*)/d(F_b) = delta F_a / (F_a - F_b)^2, and z = t* dhat_z.
 * ------------------------------------------------------------------------ */
int orc_depth_grad(const int32_t dims[3], const int32_t off[3], const float* F,
                   const uint16_t* W, const float grid[4], float step,
                   const float K[4], const double T64[12], int width, int height,
                   const int32_t* k_cells, const double* gd,
                   double grad_xi[6], double* grad_F)
{
    const orc_vol vol = { dims, off, F, W };
    const double delta = (double)(step * grid[3]);
    const double s = grid[3];
    const double C[3] = { T64[3], T64[7], T64[11] };
    double acc[6] = {0, 0, 0, 0, 0, 0};
    /* serial: the voxel-gradient scatter stays simple and deterministic */
    for (int v = 0; v < height; ++v) {
        for (int u = 0; u < width; ++u) {
            const int64_t p = (int64_t)v * width + u;
            const int32_t* kc = k_cells + 7 * p;
            if (kc[0] < 0 || gd[p] == 0.0) continue;
            double dh[3], dw[3];
            pixel_ray64(u, v, K, T64, dh, dw);
            double Fs[2], gc[2][3], q[2][3], wts[2][8];
            for (int j = 0; j < 2; ++j) {
                const int* cell = kc + 1 + 3 * j;
                const double t = (double)(kc[0] - 1 + j) * delta;
                double f[3], gl[3], gw[3];
                for (int a = 0; a < 3; ++a) {
                    q[j][a] = t * dh[a];
                    const double x = C[a] + t * dw[a];
                    f[a] = (x - grid[a]) / s - 0.5 - (double)off[a] - (double)cell[a];
                }
                Fs[j] = sample64(&vol, cell, f, gl, wts[j]);
                for (int a = 0; a < 3; ++a) gw[a] = gl[a] / s;
                for (int c = 0; c < 3; ++c)
                    gc[j][c] = T64[0 * 4 + c] * gw[0] + T64[1 * 4 + c] * gw[1] + T64[2 * 4 + c] * gw[2];
            }
            const double den = Fs[0] - Fs[1];
            const double dt_dF[2] = { -delta * Fs[1] / (den * den), delta * Fs[0] / (den * den) };
            const double gz = gd[p] * dh[2];
            for (int j = 0; j < 2; ++j) {
                const double k = gz * dt_dF[j];
                const double* g = gc[j];
                const double* qq = q[j];
                acc[0] += k * g[0];
                acc[1] += k * g[1];
                acc[2] += k * g[2];
                acc[3] += k * (qq[1] * g[2] - qq[2] * g[1]);
                acc[4] += k * (qq[2] * g[0] - qq[0] * g[2]);
                acc[5] += k * (qq[0] * g[1] - qq[1] * g[0]);
                if (grad_F) {
                    const int* cell = kc + 1 + 3 * j;
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx)
                                grad_F[vidx(dims, cell[0] + dx, cell[1] + dy, cell[2] + dz)]
                                    += k * wts[j][dz * 4 + dy * 2 + dx];
                }
            }
        }
    }
    for (int i = 0; i < 6; ++i) grad_xi[i] = acc[i];
    return 0;
}

/* ------------------------------------------------------------------------
 * Placement cells (Dynamic Mapping for SLAM section).  For every pixel with
 * a valid depth, the ray endpoint e = R (D K^-1 [u, v, 1]^T) + t (the
 * global vertex of the Depth Map Conversion section) is mapped to the cell
 * k = floor((e - o) / (s (d_v - 2))) of the placement lattice whose volumes
 * have translations h_t = k (d_v - 2).  Output: per pixel the cell (3 ints)
 * and a validity byte.  Counting and the insertion/removal policy are done
 * by the caller.
 * ------------------------------------------------------------------------ */
int orc_placement_cells(const float* depth, int width, int height,
                        const float K[4], const float T[12],
                        const float grid[4], int d_v,
                        int32_t* cells, uint8_t* valid)
{
    if (d_v < 3) return 1;
    const float cell = grid[3] * (float)(d_v - 2);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < height; ++v) {
        for (int u = 0; u < width; ++u) {
            const int64_t p = (int64_t)v * width + u;
            const float Dz = depth[p];
            if (!(Dz > 0.0f && Dz < INFINITY)) { valid[p] = 0; cells[3 * p] = cells[3 * p + 1] = cells[3 * p + 2] = 0; continue; }
            const float ra = ((float)u - K[2]) / K[0];
            const float rb = ((float)v - K[3]) / K[1];
            const float q[3] = { Dz * ra, Dz * rb, Dz };
            int ok = 1;
            for (int r = 0; r < 3; ++r) {
                const float e = (((T[4 * r + 0] * q[0]) + (T[4 * r + 1] * q[1])) + (T[4 * r + 2] * q[2])) + T[4 * r + 3];
                const float kf = floorf((e - grid[r]) / cell);
                if (!(kf >= -1073741824.0f && kf < 1073741824.0f)) ok = 0;
                cells[3 * p + r] = ok ? (int32_t)kf : 0;
            }
            valid[p] = (uint8_t)ok;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Surface points (Input and Output: the vertex set V with normals N, at most
 * one vertex per voxel; Metrics: a voxel that the surface crosses gets a
 * vertex).  Readings of the paper taken here:
 *  - voxel g emits a vertex when its cell [g, g + 1]^3 lies in the volume
 *    and is observed at all 8 corners (W > 0), and the TSDF changes sign
 *    along one of the three edges leaving g (one end > 0, the other <= 0)
 *    with both ends inside the truncation band (|F| < 1);
 *  - the first such edge in the order x, y, z gives the vertex: the linear
 *    zero crossing c(g) + s t e_a with t = F(g) / (F(g) - F(g + e_a)) and
 *    c(g) = o + s (g + 1/2) the voxel centre;
 *  - the normal is the gradient of the cell's trilinear interpolant at the
 *    vertex, normalised (it points to F > 0, the observed free space).
 * The sign and band tests read the binary32 F; positions and normals are
 * binary64.  Points come in global voxel order (z, then y, then x), with
 * their global voxel index in G.  At most max_points are written; *n_out
 * is the total.
 * ------------------------------------------------------------------------ */
int orc_extract(const int32_t dims[3], const int32_t off[3], const float* F,
                const uint16_t* W, const float grid[4], int64_t max_points,
                double* V, double* N, int32_t* G, int64_t* n_out)
{
    const double o[3] = { grid[0], grid[1], grid[2] };
    const double s = grid[3];
    int64_t n = 0;
    if (dims[0] < 2 || dims[1] < 2 || dims[2] < 2) { *n_out = 0; return 0; }
    for (int z = 0; z + 1 < dims[2]; ++z)
        for (int y = 0; y + 1 < dims[1]; ++y)
            for (int x = 0; x + 1 < dims[0]; ++x) {
                /* the cell's corners, c[k] at (x + (k & 1), y + (k >> 1 & 1), z + (k >> 2)) */
                float c[8];
                int observed = 1;
                for (int k = 0; k < 8 && observed; ++k) {
                    const int64_t i = vidx(dims, x + (k & 1), y + ((k >> 1) & 1), z + (k >> 2));
                    observed = W[i] > 0;
                    c[k] = F[i];
                }
                if (!observed) continue;
                /* edges leaving g: +x is corner 1, +y corner 2, +z corner 4 */
                int axis = -1;
                for (int a = 0; a < 3 && axis < 0; ++a) {
                    const float f0 = c[0], f1 = c[1 << a];
                    const int in_band = fabsf(f0) < 1.0f && fabsf(f1) < 1.0f;
                    const int change = (f0 > 0.0f && f1 <= 0.0f) || (f0 <= 0.0f && f1 > 0.0f);
                    if (in_band && change) axis = a;
                }
                if (axis < 0) continue;
                const double f0 = c[0], f1 = c[1 << axis];
                const double t = f0 / (f0 - f1);
                double fr[3] = { 0.0, 0.0, 0.0 };
                fr[axis] = t;
                const int g[3] = { off[0] + x, off[1] + y, off[2] + z };
                double gr[3] = { 0.0, 0.0, 0.0 };
                for (int k = 0; k < 8; ++k) {
                    const int b[3] = { k & 1, (k >> 1) & 1, k >> 2 };
                    for (int a = 0; a < 3; ++a) {
                        double w = b[a] ? 1.0 : -1.0;
                        for (int q = 0; q < 3; ++q)
                            if (q != a) w *= b[q] ? fr[q] : 1.0 - fr[q];
                        gr[a] += w * (double)c[k];
                    }
                }
                const double len = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
                if (n < max_points) {
                    for (int a = 0; a < 3; ++a) {
                        V[3 * n + a] = o[a] + s * ((double)g[a] + 0.5 + fr[a]);
                        N[3 * n + a] = len > 0.0 ? gr[a] / len : NAN;
                        G[3 * n + a] = g[a];
                    }
                }
                ++n;
            }
    *n_out = n;
    return 0;
}

/* ------------------------------------------------------------------------
 * Camera tracking (Depth Map Conversion and Camera Tracking sections; the
 * tracker itself is the projective point-to-plane ICP of KinectFusion that
 * the paper cites).  Readings of the paper taken here:
 *  - vertex v(x, y) = K^-1 [x, y, 1]^T D(x, y) for a valid depth (> 0 and
 *    finite), in camera coordinates; NaN otherwise;
 *  - normal n(x, y) = (v(x+1, y) - v(x, y)) x (v(x, y+1) - v(x, y)),
 *    normalised; NaN when one of the three vertices is missing, outside the
 *    image, or the cross product is zero.  Its sign is not used: the
 *    compatibility test compares |n . n_model|;
 *  - a pyramid of depth maps: level l+1 (floor(w/2) x floor(h/2)) holds the
 *    mean of the valid depths of the 2x2 block whose difference from the
 *    block's first valid depth (order (0,0), (1,0), (0,1), (1,1)) is at
 *    most `tau` metres, 0 when none is valid; intrinsics of level l are
 *    f / 2^l and (c + 1/2) / 2^l - 1/2;
 *  - the model (the raycast vertex and normal maps of the previous pose,
 *    world coordinates) at level l+1 takes the sample (2x, 2y) of level l;
 *  - projective association: the current vertex moved by the estimate,
 *    v_g = R v + t, is projected into the model's camera with the level's
 *    intrinsics to the nearest pixel; the pair is used when that pixel is
 *    in the image and holds a model vertex, |v_g - v_m| <= eps_d and
 *    |R n . n_m| >= cos_theta;
 *  - point-to-plane error sum ((v_g - v_m) . n_m)^2, linearised for a left
 *    perturbation Exp(xi) T, xi = (rho, omega): residual r = n_m . (v_g -
 *    v_m), Jacobian J = [n_m, v_g x n_m]; the normal equations are
 *    A = sum J J^T, b = sum J r and the update solves A xi = -b.
 * Decisions (validity, the pixel, both tests) are binary32 with one rounding
 * per written operation; J, r and the sums are binary64.
 * ------------------------------------------------------------------------ */
static inline int depth_ok(float d) { return d > 0.0f && d <= 3.4e38f; }

/* Edge-preserving smoothing of the depth map before tracking (the
 * KinectFusion tracker the paper cites smooths its input with a bilateral
 * filter; here its range kernel is a window): for a valid pixel p,
 * D_s(p) = sum_q w(q - p) D(q) / sum_q w(q - p) over the valid q of the 7x7
 * window around p inside the image with |D(q) - D(p)| <= delta, with the
 * binomial weights w(dx, dy) = C(6, dx + 3) C(6, dy + 3); invalid pixels
 * give 0.  Products and sums in binary32, the window row by row. */
int orc_depth_smooth(const float* D, int w, int h, float delta, float* out)
{
    static const float c6[7] = { 1.0f, 6.0f, 15.0f, 20.0f, 15.0f, 6.0f, 1.0f };
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const float d0 = D[(int64_t)y * w + x];
            if (!depth_ok(d0)) { out[(int64_t)y * w + x] = 0.0f; continue; }
            float num = 0.0f, den = 0.0f;
            for (int dy = -3; dy <= 3; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= h) continue;
                for (int dx = -3; dx <= 3; ++dx) {
                    const int xx = x + dx;
                    if (xx < 0 || xx >= w) continue;
                    const float d = D[(int64_t)yy * w + xx];
                    if (!depth_ok(d) || !(fabsf(d - d0) <= delta)) continue;
                    const float wt = c6[dx + 3] * c6[dy + 3];
                    num = num + wt * d;
                    den = den + wt;
                }
            }
            out[(int64_t)y * w + x] = num / den;
        }
    return 0;
}

/* Level l+1 depth (w2 = w / 2, h2 = h / 2) from level l. */
int orc_depth_down(const float* D, int w, int h, float tau, float* D2)
{
    const int w2 = w / 2, h2 = h / 2;
    for (int y = 0; y < h2; ++y)
        for (int x = 0; x < w2; ++x) {
            const float q[4] = { D[(2 * y) * w + 2 * x], D[(2 * y) * w + 2 * x + 1],
                                 D[(2 * y + 1) * w + 2 * x], D[(2 * y + 1) * w + 2 * x + 1] };
            int have = 0;
            float ref = 0.0f, sum = 0.0f;
            int n = 0;
            for (int k = 0; k < 4; ++k) {
                if (!depth_ok(q[k])) continue;
                if (!have) { ref = q[k]; have = 1; }
                if (fabsf(q[k] - ref) <= tau) { sum = sum + q[k]; ++n; }
            }
            D2[y * w2 + x] = n ? sum / (float)n : 0.0f;
        }
    return 0;
}

static void vertex32(const float* D, int w, int x, int y, const float K[4], float v[3])
{
    const float d = D[y * w + x];
    if (!depth_ok(d)) { v[0] = v[1] = v[2] = NAN; return; }
    v[0] = (((float)x - K[2]) / K[0]) * d;
    v[1] = (((float)y - K[3]) / K[1]) * d;
    v[2] = d;
}

/* Vertex and normal maps (w x h x 3, camera frame) of a depth map. */
int orc_vertex_normal(const float* D, int w, int h, const float K[4], float* V, float* N)
{
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            float v00[3], v10[3], v01[3];
            vertex32(D, w, x, y, K, v00);
            float* vo = V + 3 * ((int64_t)y * w + x);
            float* no = N + 3 * ((int64_t)y * w + x);
            vo[0] = v00[0]; vo[1] = v00[1]; vo[2] = v00[2];
            no[0] = no[1] = no[2] = NAN;
            if (isnan(v00[2]) || x + 1 >= w || y + 1 >= h) continue;
            vertex32(D, w, x + 1, y, K, v10);
            vertex32(D, w, x, y + 1, K, v01);
            if (isnan(v10[2]) || isnan(v01[2])) continue;
            const float a[3] = { v10[0] - v00[0], v10[1] - v00[1], v10[2] - v00[2] };
            const float b[3] = { v01[0] - v00[0], v01[1] - v00[1], v01[2] - v00[2] };
            const float c[3] = { (a[1] * b[2]) - (a[2] * b[1]), (a[2] * b[0]) - (a[0] * b[2]),
                                 (a[0] * b[1]) - (a[1] * b[0]) };
            const float len = sqrtf(((c[0] * c[0]) + (c[1] * c[1])) + (c[2] * c[2]));
            if (!(len > 0.0f)) continue;
            no[0] = c[0] / len; no[1] = c[1] / len; no[2] = c[2] / len;
        }
    return 0;
}

/* Model maps of level l+1 from level l: sample (2x, 2y). */
int orc_model_down(const float* V, const float* N, int w, int h, float* V2, float* N2)
{
    const int w2 = w / 2, h2 = h / 2;
    for (int y = 0; y < h2; ++y)
        for (int x = 0; x < w2; ++x)
            for (int a = 0; a < 3; ++a) {
                V2[3 * ((int64_t)y * w2 + x) + a] = V[3 * ((int64_t)(2 * y) * w + 2 * x) + a];
                N2[3 * ((int64_t)y * w2 + x) + a] = N[3 * ((int64_t)(2 * y) * w + 2 * x) + a];
            }
    return 0;
}

/* One association + normal-equation pass.  V, N: current maps (w x h,
 * camera frame); Vm, Nm: model maps (wm x hm, world); Km: the level's
 * intrinsics (model and current images share them); T: the estimate;
 * Tm: the model's camera-to-world pose.  sums: A (upper triangle, row by
 * row, 21), b (6), inlier count, sum r^2.  inlier: per current pixel. */
int orc_icp_reduce(const float* V, const float* N, int w, int h, const float* Vm, const float* Nm, int wm,
                   int hm, const float Km[4], const float T[12], const float Tm[12], float eps_d,
                   float cos_theta, double sums[29], uint8_t* inlier)
{
    double acc[29];
    for (int i = 0; i < 29; ++i) acc[i] = 0.0;
    const float e2 = eps_d * eps_d;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            const int64_t p = (int64_t)y * w + x;
            if (inlier) inlier[p] = 0;
            const float* v = V + 3 * p;
            const float* n = N + 3 * p;
            if (isnan(v[0]) || isnan(v[1]) || isnan(v[2]) || isnan(n[0]) || isnan(n[1]) || isnan(n[2])) continue;
            float vg[3], ng[3], d[3], q[3];
            for (int a = 0; a < 3; ++a) {
                vg[a] = (((T[4 * a] * v[0]) + (T[4 * a + 1] * v[1])) + (T[4 * a + 2] * v[2])) + T[4 * a + 3];
                ng[a] = ((T[4 * a] * n[0]) + (T[4 * a + 1] * n[1])) + (T[4 * a + 2] * n[2]);
                d[a] = vg[a] - Tm[4 * a + 3];
            }
            for (int a = 0; a < 3; ++a) q[a] = ((Tm[a] * d[0]) + (Tm[4 + a] * d[1])) + (Tm[8 + a] * d[2]);
            if (!(q[2] > 0.0f)) continue;
            const float iz = 1.0f / q[2];
            const float ur = floorf((((Km[0] * q[0]) * iz) + Km[2]) + 0.5f);
            const float vr = floorf((((Km[1] * q[1]) * iz) + Km[3]) + 0.5f);
            if (!(ur >= 0.0f && ur <= (float)(wm - 1) && vr >= 0.0f && vr <= (float)(hm - 1))) continue;
            const int64_t m = (int64_t)vr * wm + (int64_t)ur;
            const float* vm = Vm + 3 * m;
            const float* nm = Nm + 3 * m;
            if (isnan(vm[0]) || isnan(vm[1]) || isnan(vm[2]) || isnan(nm[0]) || isnan(nm[1]) || isnan(nm[2]))
                continue;
            const float dv[3] = { vg[0] - vm[0], vg[1] - vm[1], vg[2] - vm[2] };
            const float dist2 = ((dv[0] * dv[0]) + (dv[1] * dv[1])) + (dv[2] * dv[2]);
            if (!(dist2 <= e2)) continue;
            const float dot = ((ng[0] * nm[0]) + (ng[1] * nm[1])) + (ng[2] * nm[2]);
            if (!(fabsf(dot) >= cos_theta)) continue;
            if (inlier) inlier[p] = 1;
            /* binary64 from here */
            const double g[3] = { vg[0], vg[1], vg[2] };
            const double nn[3] = { nm[0], nm[1], nm[2] };
            const double r = nn[0] * (g[0] - (double)vm[0]) + nn[1] * (g[1] - (double)vm[1]) +
                             nn[2] * (g[2] - (double)vm[2]);
            const double J[6] = { nn[0], nn[1], nn[2], g[1] * nn[2] - g[2] * nn[1], g[2] * nn[0] - g[0] * nn[2],
                                  g[0] * nn[1] - g[1] * nn[0] };
            int k = 0;
            for (int i = 0; i < 6; ++i)
                for (int j = i; j < 6; ++j) acc[k++] += J[i] * J[j];
            for (int i = 0; i < 6; ++i) acc[21 + i] += J[i] * r;
            acc[27] += 1.0;
            acc[28] += r * r;
        }
    for (int i = 0; i < 29; ++i) sums[i] = acc[i];
    return 0;
}

/* Threads the oracle's parallel loops use (for reporting CPU timings). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
/* Threads the parallel loops use from now on (n >= 1). */
void orc_set_threads(int n) { omp_set_num_threads(n < 1 ? 1 : n); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
