/*
 * CPU ORACLE for the Disentangled 4D Gaussian Splatting render path.
 *
 * TEST INFRASTRUCTURE ONLY: this library is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  No product code
 * links, loads or calls it.  It shares no source with the GPU library.
 *
 * What it computes (paper: "Disentangled 4D Gaussian Splatting", Sec. 3.1-3.2):
 *   camera stage  -- Alg. 1 camera branch; Eq. 9-10 (camera-space mean), Eq. 11
 *                    (camera-space velocity), Eq. 12-13 (ray-space mean/velocity),
 *                    Sigma = R S S^T R^T from scale and quaternion;
 *   time stage    -- Alg. 1 per-timestamp steps; temporal weight of the sliced
 *                    Gaussian (Eq. 6-7 with lambda = 1/s_t^2), motion of the mean,
 *                    Jacobian at the time-moved mean (Eq. 14), Eq. 15;
 *   binning       -- 16x16 tiles, lists ordered by (tile, depth, index), the tiled
 *                    rasteriser the paper adopts from 3D Gaussian Splatting;
 *   blending      -- Eq. 4 front to back with alpha_i = o_i w_i G'_i;
 *   adjoint       -- the exact derivative of the blend with discrete decisions
 *                    held fixed (reverse accumulation over stored per-pixel lists),
 *                    and of the projection by the complex-step method
 *                    (Squire & Trapp, SIAM Rev. 1998), which is exact to rounding.
 *
 * Readings of passages the paper leaves open are fixed in the design notes; each
 * is marked below where it is used.  Precision: quantities that decide integers
 * (culls, tile rectangles, depth keys) are computed in FP32 in a fixed operation
 * order; everything else in FP64.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_VERSION 2

/* fp32(2 ln 255): tau^2 > KT * s_t^2  <=>  w < 1/255 (up to rounding) */
#define OC_KT 11.0825272f
/* Relative margins inside which an FP32 evaluation may legitimately decide a threshold
 * differently from this FP64 blend (flag bookkeeping only: no result depends on them).
 * Defaults; oc_set_flag_margins changes them for measurements of the FP32 error. */
static double OC_FLAG_ALPHA_REL = 3e-5;
static double OC_FLAG_T_REL = 1e-5;  /* |T' - 1e-4| < 1e-9 */
static double OC_FLAG_POWER_REL = 1e-5;
void oc_set_flag_margins(double alpha_rel, double t_rel, double power_rel)
{
    OC_FLAG_ALPHA_REL = alpha_rel;
    OC_FLAG_T_REL = t_rel;
    OC_FLAG_POWER_REL = power_rel;
}

/* Motion / covariance model of the time stage (the readings of Eq. 13-14 made
 * switchable): 0 = the 2D mean moves linearly (Eq. 13 as printed), Jacobian at the
 * moved mean; 1 = the 2D mean is the exact projection of the moved mean; 2 = linear
 * motion, Jacobian frozen at the camera stage's mean (fully deferred covariance). */
#define OC_MOTION_LINEAR 0
#define OC_MOTION_EXACT 1
#define OC_MOTION_FROZEN_J 2
static int oc_motion = OC_MOTION_LINEAR;
void oc_set_motion(int m) { oc_motion = m; }
int oc_get_motion(void) { return oc_motion; }

typedef struct {
    int32_t n, sh_degree;
    const double *mean;     /* [3][n] */
    const double *scale;    /* [3][n] activated (positive) */
    const double *quat;     /* [4][n] scalar first, not necessarily normalised */
    const double *opacity;  /* [n] activated, in (0,1) */
    const double *t_mean;   /* [n] */
    const double *t_scale;  /* [n] activated (positive) */
    const double *velocity; /* [3][n] */
    const double *sh;       /* [K][3][n], K = (deg+1)^2 */
} oc_scene;

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy, tan_fovx, tan_fovy, znear;
    float R[9];      /* world -> camera rotation, row major; camera looks along +z */
    float T[3];
    float campos[3]; /* camera centre in world coordinates */
} oc_camera;

/* ---------------- spherical-harmonic tables from their definition ---------------- */
struct sh_tab {
    double dpoly[4][4][4]; /* [l][m][j]: coefficient of z^j in the m-th derivative of P_l */
    double norm[4][4];     /* [l][m]: normalisation including (-1)^m */
};

static double fact(int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; }
static double binom(int a, int b) { return fact(a) / (fact(b) * fact(a - b)); }

static struct sh_tab g_sh_tab;

static const struct sh_tab *sh_tables(void) { return &g_sh_tab; }

/* Built once when the library is loaded, before any (OpenMP) caller can read it. */
__attribute__((constructor)) static void sh_tables_init(void)
{
    struct sh_tab tb;
    memset(&tb, 0, sizeof(tb));
    for (int l = 0; l <= 3; ++l) {
        /* Legendre: P_l(z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) z^(l-2k) */
        double c[4] = {0, 0, 0, 0};
        for (int k = 0; 2 * k <= l; ++k)
            c[l - 2 * k] = pow(2.0, -l) * ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l);
        for (int m = 0; m <= l; ++m) {
            double d[4] = {0, 0, 0, 0};
            memcpy(d, c, sizeof(d));
            for (int r = 0; r < m; ++r) { /* differentiate once */
                for (int j = 0; j < 3; ++j) d[j] = (j + 1) * d[j + 1];
                d[3] = 0;
            }
            memcpy(tb.dpoly[l][m], d, sizeof(d));
            double k2 = (2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - m) / fact(l + m);
            tb.norm[l][m] = (m == 0) ? sqrt(k2) : sqrt(2.0) * sqrt(k2) * ((m & 1) ? -1.0 : 1.0);
        }
    }
    g_sh_tab = tb;
}

/* Thread count of the OpenMP regions (0 = the OpenMP default). */
void oc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

int oc_num_threads(void) { return omp_get_max_threads(); }

/* ---------------- three instantiations of the body ---------------- */
#define REAL float
#define DEC float
#define SFX(x) x##_f32
#define RE(x) (x)
#define LIT(x) x##f
#define SQRT sqrtf
#define EXP expf
#define FLOORD floorf
#define CEILD ceilf
#define SQRTD sqrtf
#include "oracle_body.inc"
#undef REAL
#undef DEC
#undef SFX
#undef RE
#undef LIT
#undef SQRT
#undef EXP
#undef FLOORD
#undef CEILD
#undef SQRTD

#define REAL double
#define DEC double
#define SFX(x) x##_f64
#define RE(x) (x)
#define LIT(x) x
#define SQRT sqrt
#define EXP exp
#define FLOORD floor
#define CEILD ceil
#define SQRTD sqrt
#include "oracle_body.inc"
#undef REAL
#undef DEC
#undef SFX
#undef RE
#undef LIT
#undef SQRT
#undef EXP
#undef FLOORD
#undef CEILD
#undef SQRTD

#define REAL double complex
#define DEC double
#define SFX(x) x##_c128
#define RE(x) creal(x)
#define LIT(x) x
#define SQRT csqrt
#define EXP cexp
#define FLOORD floor
#define CEILD ceil
#define SQRTD sqrt
#include "oracle_body.inc"
#undef REAL
#undef DEC
#undef SFX
#undef RE
#undef LIT
#undef SQRT
#undef EXP
#undef FLOORD
#undef CEILD
#undef SQRTD

/* ---------------- helpers ---------------- */
static int n_params(int deg) { return 16 + 3 * (deg + 1) * (deg + 1); }

static void gather_params(const oc_scene *s, int g, double *prm)
{
    int n = s->n, K = (s->sh_degree + 1) * (s->sh_degree + 1);
    for (int i = 0; i < 3; ++i) prm[i] = s->mean[i * n + g];
    for (int i = 0; i < 3; ++i) prm[3 + i] = s->scale[i * n + g];
    for (int i = 0; i < 4; ++i) prm[6 + i] = s->quat[i * n + g];
    prm[10] = s->opacity[g];
    prm[11] = s->t_mean[g];
    prm[12] = s->t_scale[g];
    for (int i = 0; i < 3; ++i) prm[13 + i] = s->velocity[i * n + g];
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < 3; ++c) prm[16 + k * 3 + c] = s->sh[(k * 3 + c) * n + g];
}

int oc_version(void) { return OC_VERSION; }

/* ---------------- projection (camera stage + time stage) ----------------
 * Outputs are planar: p[3n], u[3n], covc[6n], m0[2n], md[2n], rgb[3n], m[2n],
 * conic[3n], amax[n], w[n], depth[n] (FP32 bits of the camera-space z at t),
 * rect[4n] (x0,y0,x1,y1), count[n], mdt[2n] (the 2D mean's velocity at t, the flow),
 * margin[n] (the smallest relative margin of the Gaussian's time-stage decisions, a
 * diagnostic).  Any output pointer may be NULL.                                             */
#define DEFINE_PROJECT(SUF, T)                                                                       \
    void oc_project_##SUF(const oc_scene *s, const oc_camera *cam, double t, T *p, T *u, T *covc,   \
                          T *m0, T *md, T *rgb, T *m, T *conic, T *amax, T *w, float *depth,         \
                          int32_t *rect, int32_t *count, T *mdt, T *margin)                          \
    {                                                                                                \
        int n = s->n, P = n_params(s->sh_degree);                                                    \
        _Pragma("omp parallel for schedule(static)") for (int g = 0; g < n; ++g)                     \
        {                                                                                            \
            double prmd[64];                                                                         \
            T prm[64];                                                                               \
            rec_##SUF r;                                                                             \
            gather_params(s, g, prmd);                                                               \
            for (int j = 0; j < P; ++j) prm[j] = (T)prmd[j];                                         \
            project_one_##SUF(prm, s->sh_degree, cam, (T)t, &r);                                     \
            for (int i = 0; i < 3; ++i) {                                                            \
                if (p) p[i * n + g] = r.p[i];                                                        \
                if (u) u[i * n + g] = r.u[i];                                                        \
                if (rgb) rgb[i * n + g] = r.rgb[i];                                                  \
                if (conic) conic[i * n + g] = r.conic[i];                                            \
            }                                                                                        \
            for (int i = 0; i < 6; ++i)                                                              \
                if (covc) covc[i * n + g] = r.covc[i];                                               \
            for (int i = 0; i < 2; ++i) {                                                            \
                if (m0) m0[i * n + g] = r.m0[i];                                                     \
                if (md) md[i * n + g] = r.md[i];                                                     \
                if (m) m[i * n + g] = r.m[i];                                                        \
                if (mdt) mdt[i * n + g] = r.mdt[i];                                                  \
            }                                                                                        \
            if (amax) amax[g] = r.amax;                                                              \
            if (w) w[g] = r.w;                                                                       \
            if (depth) depth[g] = (float)r.depth;                                                    \
            for (int i = 0; i < 4; ++i)                                                              \
                if (rect) rect[i * n + g] = r.count > 0 ? r.rect[i] : 0;                             \
            if (count) count[g] = r.count;                                                           \
            if (margin) margin[g] = (T)r.margin;                                                     \
        }                                                                                            \
    }
DEFINE_PROJECT(f32, float)
DEFINE_PROJECT(f64, double)

/* ---------------- binning: per-tile lists ordered by (depth bits, index) ---------------- */
typedef struct { uint32_t dbits, g; } oc_item;

static int cmp_item(const void *a, const void *b)
{
    const oc_item *x = a, *y = b;
    if (x->dbits != y->dbits) return x->dbits < y->dbits ? -1 : 1;
    return x->g < y->g ? -1 : (x->g > y->g);
}

/* keys[I] = (tile << 32) | bits(depth), values[I] = Gaussian index, ranges[2*tiles] = [start, end).
 * Returns the number of instances.  keys/values/ranges may be NULL to only count. */
int64_t oc_bin(int n, int W, int H, const int32_t *rect, const int32_t *count, const float *depth,
               uint64_t *keys, uint32_t *values, uint32_t *ranges)
{
    int TX = (W + 15) / 16, TY = (H + 15) / 16, tiles = TX * TY;
    int64_t *len = calloc(tiles + 1, sizeof(int64_t));
    int64_t ninst = 0;
    for (int g = 0; g < n; ++g) {
        if (count[g] <= 0) continue;
        for (int y = rect[n + g]; y < rect[3 * n + g]; ++y)
            for (int x = rect[g]; x < rect[2 * n + g]; ++x) len[y * TX + x]++;
        ninst += count[g];
    }
    if (!keys) { free(len); return ninst; }
    int64_t *start = calloc(tiles + 1, sizeof(int64_t)), *fill = calloc(tiles, sizeof(int64_t));
    for (int i = 0; i < tiles; ++i) start[i + 1] = start[i] + len[i];
    oc_item *items = malloc(sizeof(oc_item) * (ninst > 0 ? ninst : 1));
    for (int g = 0; g < n; ++g) {
        if (count[g] <= 0) continue;
        uint32_t db;
        memcpy(&db, &depth[g], 4);
        for (int y = rect[n + g]; y < rect[3 * n + g]; ++y)
            for (int x = rect[g]; x < rect[2 * n + g]; ++x) {
                int tile = y * TX + x;
                oc_item it = {db, (uint32_t)g};
                items[start[tile] + fill[tile]++] = it;
            }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int tile = 0; tile < tiles; ++tile)
        qsort(items + start[tile], (size_t)len[tile], sizeof(oc_item), cmp_item);
    for (int tile = 0; tile < tiles; ++tile) {
        for (int64_t j = start[tile]; j < start[tile + 1]; ++j) {
            keys[j] = ((uint64_t)tile << 32) | items[j].dbits;
            values[j] = items[j].g;
        }
        if (ranges) {
            ranges[2 * tile] = (uint32_t)start[tile];
            ranges[2 * tile + 1] = (uint32_t)start[tile + 1];
        }
    }
    free(items); free(start); free(fill); free(len);
    return ninst;
}

/* ---------------- blending (O1: tiled) ---------------- */
static int64_t blend_tiled(int n, int W, int H, const double *m, const double *conic, const double *amax,
                           const double *rgb, const double *md, const uint32_t *values, const uint32_t *ranges,
                           const double *bg, double *img, double *flow, double *final_T, int32_t *n_contrib,
                           int32_t *flags, uint64_t *dhash)
{
    int TX = (W + 15) / 16, TY = (H + 15) / 16;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
    for (int tile = 0; tile < TX * TY; ++tile) {
        int tx = tile % TX, ty = tile / TX;
        uint32_t s0 = ranges[2 * tile], s1 = ranges[2 * tile + 1];
        for (int py = ty * 16; py < ty * 16 + 16 && py < H; ++py)
            for (int px = tx * 16; px < tx * 16 + 16 && px < W; ++px) {
                double out[3], fo[2], T;
                int nc, fl;
                int64_t ne = 0;
                size_t pi = (size_t)py * W + px;
                blend_pixel_f64(n, m, conic, amax, rgb, md, values + s0, (int)(s1 - s0), px + 0.5, py + 0.5, bg,
                                out, fo, &T, &nc, &fl, &ne, dhash ? dhash + pi : NULL);
                total += ne;
                for (int c = 0; c < 3; ++c) img[(size_t)c * W * H + pi] = out[c];
                if (md)
                    for (int c = 0; c < 2; ++c) flow[(size_t)c * W * H + pi] = fo[c];
                if (final_T) final_T[pi] = T;
                if (n_contrib) n_contrib[pi] = nc;
                if (flags) flags[pi] = fl;
            }
    }
    return total;
}

int64_t oc_blend(int n, int W, int H, const double *m, const double *conic, const double *amax,
                 const double *rgb, const uint32_t *values, const uint32_t *ranges, const double *bg,
                 double *img, double *final_T, int32_t *n_contrib, int32_t *flags, uint64_t *dhash)
{
    return blend_tiled(n, W, H, m, conic, amax, rgb, NULL, values, ranges, bg, img, NULL, final_T, n_contrib,
                       flags, dhash);
}

/* The blend with the optical flow of Sec. 3.3 (md planar [2][n]; flow [2][H][W]). */
int64_t oc_blend_flow(int n, int W, int H, const double *m, const double *conic, const double *amax,
                      const double *rgb, const double *md, const uint32_t *values, const uint32_t *ranges,
                      const double *bg, double *img, double *flow, double *final_T, int32_t *n_contrib,
                      int32_t *flags)
{
    return blend_tiled(n, W, H, m, conic, amax, rgb, md, values, ranges, bg, img, flow, final_T, n_contrib,
                       flags, NULL);
}

/* ---------------- blending (O0: brute force per pixel, tiny scenes) ----------------
 * For each pixel: every non-culled Gaussian whose tile rectangle contains the
 * pixel's tile, sorted by (depth bits, index), then the same per-pixel blend.  */
void oc_blend_bruteforce(int n, int W, int H, const double *m, const double *conic, const double *amax,
                         const double *rgb, const int32_t *rect, const int32_t *count, const float *depth,
                         const double *bg, double *img, double *final_T, int32_t *n_contrib, int32_t *flags)
{
    oc_item *items = malloc(sizeof(oc_item) * (n > 0 ? n : 1));
    uint32_t *list = malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int tx = px / 16, ty = py / 16, len = 0;
            for (int g = 0; g < n; ++g) {
                if (count[g] <= 0) continue;
                if (tx < rect[g] || tx >= rect[2 * n + g] || ty < rect[n + g] || ty >= rect[3 * n + g]) continue;
                oc_item it;
                memcpy(&it.dbits, &depth[g], 4);
                it.g = (uint32_t)g;
                items[len++] = it;
            }
            qsort(items, (size_t)len, sizeof(oc_item), cmp_item);
            for (int k = 0; k < len; ++k) list[k] = items[k].g;
            double out[3], T;
            int nc, fl;
            int64_t ne = 0;
            blend_pixel_f64(n, m, conic, amax, rgb, NULL, list, len, px + 0.5, py + 0.5, bg, out, NULL, &T, &nc,
                            &fl, &ne, NULL);
            size_t pi = (size_t)py * W + px;
            for (int c = 0; c < 3; ++c) img[(size_t)c * W * H + pi] = out[c];
            if (final_T) final_T[pi] = T;
            if (n_contrib) n_contrib[pi] = nc;
            if (flags) flags[pi] = fl;
        }
    free(items);
    free(list);
}

/* ---------------- blend adjoint ----------------
 * For pixel colour C = sum_i c_i a_i T_i + T_N bg with T_i = prod_{j<i} (1 - a_j)
 * (and, with md / dL_dflow given, the flow F = sum_i md_i a_i T_i as two more channels
 * of "colour" md_i and background 0):
 *   dC/dc_i = a_i T_i,
 *   dC/da_i = c_i T_i - (sum_{j>i} c_j a_j T_j + T_N bg) / (1 - a_i),
 *   a_i = amax_i exp(power_i) unless clamped to 0.99 (then constant),
 *   power = -1/2 (A dx^2 + C dy^2) - B dx dy,  dx = sx - m_x,  dy = sy - m_y.
 * The per-pixel forward values are stored (no replay) and the sums are formed
 * directly.  Gradients are accumulated per Gaussian over all pixels.
 * Optionally reports the largest relative gap between the stored transmittance
 * and one recovered backwards by division, T_i = T_{i+1} / (1 - a_i).          */
void oc_blend_bwd_flow(int n, int W, int H, const double *m, const double *conic, const double *amax,
                       const double *rgb, const double *md, const uint32_t *values, const uint32_t *ranges,
                       const double *bg, const double *dL_dimg, const double *dL_dflow, double *g_m,
                       double *g_conic, double *g_amax, double *g_rgb, double *g_md, double *replay_rel_err)
{
    int TX = (W + 15) / 16, TY = (H + 15) / 16;
    int nth = omp_get_max_threads();
    const int flow = md != NULL && dL_dflow != NULL;
    double *acc = calloc((size_t)nth * 11 * (n > 0 ? n : 1), sizeof(double));
    double *errs = calloc((size_t)nth, sizeof(double));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        double *a9 = acc + (size_t)tid * 11 * n;  /* m(2) conic(3) amax rgb(3) md(2) */
        size_t cap = 1024;
        uint32_t *gl = malloc(cap * sizeof(uint32_t));
        double *al = malloc(cap * sizeof(double)), *Tl = malloc(cap * sizeof(double));
        double *Gl = malloc(cap * sizeof(double));
        int *cl = malloc(cap * sizeof(int));
        double *dxl = malloc(cap * sizeof(double)), *dyl = malloc(cap * sizeof(double));
#pragma omp for schedule(static)
        for (int tile = 0; tile < TX * TY; ++tile) {
            int tx = tile % TX, ty = tile / TX;
            uint32_t s0 = ranges[2 * tile], s1 = ranges[2 * tile + 1];
            if ((size_t)(s1 - s0) > cap) {
                cap = (size_t)(s1 - s0);
                gl = realloc(gl, cap * sizeof(uint32_t)); al = realloc(al, cap * sizeof(double));
                Tl = realloc(Tl, cap * sizeof(double)); Gl = realloc(Gl, cap * sizeof(double));
                cl = realloc(cl, cap * sizeof(int)); dxl = realloc(dxl, cap * sizeof(double));
                dyl = realloc(dyl, cap * sizeof(double));
            }
            for (int py = ty * 16; py < ty * 16 + 16 && py < H; ++py)
                for (int px = tx * 16; px < tx * 16 + 16 && px < W; ++px) {
                    size_t pi = (size_t)py * W + px;
                    double gC[3], gF[2] = {0.0, 0.0};
                    for (int c = 0; c < 3; ++c) gC[c] = dL_dimg[(size_t)c * W * H + pi];
                    if (flow)
                        for (int c = 0; c < 2; ++c) gF[c] = dL_dflow[(size_t)c * W * H + pi];
                    /* forward, storing every blended entry */
                    double T = 1.0, sx = px + 0.5, sy = py + 0.5;
                    int cnt = 0;
                    for (uint32_t j = s0; j < s1; ++j) {
                        uint32_t g = values[j];
                        double dx = sx - m[g], dy = sy - m[n + g];
                        double A = conic[g], B = conic[n + g], Cc = conic[2 * n + g];
                        double power = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
                        if (power > 0) continue;
                        double G = exp(power);
                        double alpha = amax[g] * G;
                        int clamped = 0;
                        if (alpha > 0.99) { alpha = 0.99; clamped = 1; }
                        if (alpha < 1.0 / 255.0) continue;
                        double Tn = T * (1.0 - alpha);
                        if (Tn < 1e-4) break;
                        gl[cnt] = g; al[cnt] = alpha; Tl[cnt] = T; Gl[cnt] = G; cl[cnt] = clamped;
                        dxl[cnt] = dx; dyl[cnt] = dy;
                        ++cnt;
                        T = Tn;
                    }
                    double TN = T;
                    /* suffix sums S_i = sum_{j>i} c_j a_j T_j + T_N bg, per channel */
                    double S[3], SF[2] = {0.0, 0.0};
                    for (int c = 0; c < 3; ++c) S[c] = TN * bg[c];
                    double Trec = TN;
                    for (int i = cnt - 1; i >= 0; --i) {
                        uint32_t g = gl[i];
                        double alpha = al[i], Ti = Tl[i];
                        /* replay check: T_i recovered from T_{i+1} */
                        Trec = Trec / (1.0 - alpha);
                        double re = fabs(Trec - Ti) / Ti;
                        if (re > errs[tid]) errs[tid] = re;
                        double dC_da = 0.0;
                        for (int c = 0; c < 3; ++c) {
                            double cc = rgb[c * n + g];
                            a9[(6 + c) * n + g] += gC[c] * alpha * Ti;
                            dC_da += gC[c] * (cc * Ti - S[c] / (1.0 - alpha));
                        }
                        for (int c = 0; c < 3; ++c) S[c] += rgb[c * n + g] * alpha * Ti;
                        if (flow) {
                            for (int c = 0; c < 2; ++c) {
                                double f = md[c * n + g];
                                a9[(9 + c) * n + g] += gF[c] * alpha * Ti;
                                dC_da += gF[c] * (f * Ti - SF[c] / (1.0 - alpha));
                            }
                            for (int c = 0; c < 2; ++c) SF[c] += md[c * n + g] * alpha * Ti;
                        }
                        if (cl[i]) continue;
                        double dpower = dC_da * alpha;
                        a9[5 * n + g] += dC_da * Gl[i];
                        double dx = dxl[i], dy = dyl[i];
                        double A = conic[g], B = conic[n + g], Cc = conic[2 * n + g];
                        a9[0 * n + g] += dpower * (A * dx + B * dy);
                        a9[1 * n + g] += dpower * (Cc * dy + B * dx);
                        a9[2 * n + g] += dpower * (-0.5 * dx * dx);
                        a9[3 * n + g] += dpower * (-dx * dy);
                        a9[4 * n + g] += dpower * (-0.5 * dy * dy);
                    }
                }
        }
        free(gl); free(al); free(Tl); free(Gl); free(cl); free(dxl); free(dyl);
    }
    for (int t = 0; t < nth; ++t) {
        const double *a9 = acc + (size_t)t * 11 * n;
        for (int g = 0; g < n; ++g) {
            if (g_md)
                for (int c = 0; c < 2; ++c) g_md[c * n + g] += a9[(9 + c) * n + g];
            g_m[g] += a9[g];
            g_m[n + g] += a9[n + g];
            g_conic[g] += a9[2 * n + g];
            g_conic[n + g] += a9[3 * n + g];
            g_conic[2 * n + g] += a9[4 * n + g];
            g_amax[g] += a9[5 * n + g];
            for (int c = 0; c < 3; ++c) g_rgb[c * n + g] += a9[(6 + c) * n + g];
        }
        if (replay_rel_err && errs[t] > *replay_rel_err) *replay_rel_err = errs[t];
    }
    free(acc);
    free(errs);
}

void oc_blend_bwd(int n, int W, int H, const double *m, const double *conic, const double *amax,
                  const double *rgb, const uint32_t *values, const uint32_t *ranges, const double *bg,
                  const double *dL_dimg, double *g_m, double *g_conic, double *g_amax, double *g_rgb,
                  double *replay_rel_err)
{
    oc_blend_bwd_flow(n, W, H, m, conic, amax, rgb, NULL, values, ranges, bg, dL_dimg, NULL, g_m, g_conic, g_amax,
                      g_rgb, NULL, replay_rel_err);
}

/* ---------------- projection adjoint by the complex-step method ----------------
 * For every Gaussian with active[g] != 0 and every parameter j, the projection is
 * evaluated with parameter j displaced by i*h; Im(output)/h is the exact partial
 * derivative of each output (discrete decisions -- clamps, culls -- follow the real
 * part, i.e. are held fixed).  The splat-level gradients (m, conic, amax, rgb) are
 * contracted with these partials.  g_prm is planar [16+3K][n] in the parameter
 * order mu(3), s(3), q(4), o, mu_t, s_t, v(3), sh(k-major, rgb-minor).          */
void oc_project_bwd_flow(const oc_scene *s, const oc_camera *cam, double t, const int32_t *active,
                         const double *g_m, const double *g_conic, const double *g_amax, const double *g_rgb,
                         const double *g_md, double *g_prm)
{
    int n = s->n, P = n_params(s->sh_degree);
    const double h = 1e-30;
#pragma omp parallel for schedule(dynamic, 64)
    for (int g = 0; g < n; ++g) {
        if (!active[g]) {
            for (int j = 0; j < P; ++j) g_prm[(size_t)j * n + g] = 0.0;
            continue;
        }
        double prmd[64];
        double complex prm[64];
        rec_c128 r;
        gather_params(s, g, prmd);
        for (int j = 0; j < P; ++j) {
            for (int k = 0; k < P; ++k) prm[k] = prmd[k];
            prm[j] = prmd[j] + _Complex_I * h;
            project_one_c128(prm, s->sh_degree, cam, (double complex)t, &r);
            double d = 0.0;
            d += g_m[g] * cimag(r.m[0]) / h + g_m[n + g] * cimag(r.m[1]) / h;
            for (int i = 0; i < 3; ++i) d += g_conic[i * n + g] * cimag(r.conic[i]) / h;
            d += g_amax[g] * cimag(r.amax) / h;
            for (int c = 0; c < 3; ++c) d += g_rgb[c * n + g] * cimag(r.rgb[c]) / h;
            if (g_md) d += g_md[g] * cimag(r.mdt[0]) / h + g_md[n + g] * cimag(r.mdt[1]) / h;
            g_prm[(size_t)j * n + g] = d;
        }
    }
}

void oc_project_bwd(const oc_scene *s, const oc_camera *cam, double t, const int32_t *active,
                    const double *g_m, const double *g_conic, const double *g_amax, const double *g_rgb,
                    double *g_prm)
{
    oc_project_bwd_flow(s, cam, t, active, g_m, g_conic, g_amax, g_rgb, NULL, g_prm);
}

/* Spherical-harmonic basis at given unit directions (pins of the basis). */
void oc_sh_basis(int deg, int count, const double *dirs, double *Y)
{
    for (int i = 0; i < count; ++i) {
        double d[3] = {dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2]}, y[16];
        sh_basis_f64(deg, d, y);
        for (int k = 0; k < (deg + 1) * (deg + 1); ++k) Y[i * (deg + 1) * (deg + 1) + k] = y[k];
    }
}
