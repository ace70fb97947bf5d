// Internal declarations shared by the HIP translation units of libd4dgs (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "d4dgs.h"

namespace d4 {

constexpr int kWave = 64;
constexpr int kTile = D4DGS_TILE;
constexpr int kBlock = 256;             // threads per block of the per-Gaussian kernels
constexpr int kRadix = 256;             // buckets of the 8-bit radix digits

// fp32(2 ln 255): a Gaussian with tau^2 > kTemporalCull * s_t^2 has w < 1/255 and is culled.
constexpr float kTemporalCull = 11.0825272f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kDilation = 0.3f;
constexpr float kGuard = 1.3f;
constexpr float kLog2e = 1.44269504088896340736f;

// Camera as passed to kernels (by value).
struct CamK {
    float R[9], T[3], campos[3];
    float fx, fy, cx, cy;
    float limx, limy, znear;
    int W, H, TX, TY;
    uint32_t txm;  // div_magic(TX): tile rows and columns without a vector division
};

CamK make_camk(const d4dgs_camera &c);
// width and height the kernels handle
bool image_size_ok(int32_t w, int32_t h);
// NULL if the camera is usable, else what is wrong with it
const char *camera_problem(const d4dgs_camera &c);

// --- wave64 helpers ---------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;  // lane 0 -> 0
}

// DPP move of a 32-bit value (row_mask selects the 16-lane rows that are written; the
// others get 0).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the wave with DPP (no LDS): Hillis-Steele inside each row of
// 16 lanes (shifts by 1, 2, 4, 8; lanes shifted in from outside the row add 0), then
// row 0's total is added to row 1 and row 2's to row 3 (row_bcast:15), then the total of
// rows 0-1 to rows 2-3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_u32<0x111>(v);       // row_shr:1
    v += dpp_u32<0x112>(v);       // row_shr:2
    v += dpp_u32<0x114>(v);       // row_shr:4
    v += dpp_u32<0x118>(v);       // row_shr:8
    v += dpp_u32<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_u32<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Inclusive max-scan over the wavefront, by the same moves (lanes shifted in from outside
// a row give 0, the identity of an unsigned max).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    v = max(v, dpp_u32<0x111>(v));
    v = max(v, dpp_u32<0x112>(v));
    v = max(v, dpp_u32<0x114>(v));
    v = max(v, dpp_u32<0x118>(v));
    v = max(v, dpp_u32<0x142, 0xa>(v));
    v = max(v, dpp_u32<0x143, 0xc>(v));
    return v;
}

// Orders a wavefront's LDS accesses before the ones after it.  The accesses of one
// wavefront complete in order, so this costs no instruction; it keeps the compiler from
// moving accesses across it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same on 64-bit values (both halves moved by DPP).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)v), hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    v += dpp_u64<0x111>(v);
    v += dpp_u64<0x112>(v);
    v += dpp_u64<0x114>(v);
    v += dpp_u64<0x118>(v);
    v += dpp_u64<0x142, 0xa>(v);
    v += dpp_u64<0x143, 0xc>(v);
    return v;
}

// Wave sums, uniform: DPP inside each row (partners l ^ 1, l ^ 2, rotations by 4 and 8),
// then the four rows' values through scalar registers.
__device__ __forceinline__ uint32_t wave_sum_u32_uniform(uint32_t v) {
    v += dpp_u32<0xB1>(v);
    v += dpp_u32<0x4E>(v);
    v += dpp_u32<0x124>(v);
    v += dpp_u32<0x128>(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}
__device__ __forceinline__ uint64_t wave_sum_u64_uniform(uint64_t v) {
    v += dpp_u64<0xB1>(v);
    v += dpp_u64<0x4E>(v);
    v += dpp_u64<0x124>(v);
    v += dpp_u64<0x128>(v);
    uint64_t t = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        t += ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), 16 * r) << 32) |
             __builtin_amdgcn_readlane((uint32_t)v, 16 * r);
    return t;
}

// Wave minimum / maximum, uniform: DPP inside each row (partners l ^ 1, l ^ 2, rotations
// by 4 and 8), then the four rows' values through scalar registers.
__device__ __forceinline__ uint32_t wave_min_u32_uniform(uint32_t v) {
    v = min(v, dpp_u32<0xB1>(v));
    v = min(v, dpp_u32<0x4E>(v));
    v = min(v, dpp_u32<0x124>(v));
    v = min(v, dpp_u32<0x128>(v));
    const uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return min(min(a, b), min(c, d));
}
__device__ __forceinline__ uint32_t wave_max_u32_uniform(uint32_t v) {
    v = max(v, dpp_u32<0xB1>(v));
    v = max(v, dpp_u32<0x4E>(v));
    v = max(v, dpp_u32<0x124>(v));
    v = max(v, dpp_u32<0x128>(v));
    const uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return max(max(a, b), max(c, d));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
    return v;
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }

// The blend's per-(pixel, splat) opacity, shared instruction for instruction by the
// forward and the backward so that both take the same skip/stop decisions.
//
// Folded splat (3 x float4, staged in LDS):
//   f0 = {m.x, m.y, qa, qb},  f1 = {qc, la, r, g},  f2 = {b, amax, -, -}
// with qa = -log2(e)/2 a, qb = -log2(e) b, qc = -log2(e)/2 c (conic a, b, c) and
// la = log2(amax), so that for d = sample - m
//   q = qa dx^2 + qb dx dy + qc dy^2 + la = log2(amax) + log2(e) * power,
//   alpha = min(0.99, 2^q),  and "power > 0" is "q > la".
// Over a wavefront's pixel region q is evaluated as a polynomial in the pixel's offset
// from the region's centre (see square_coeffs).
//
__device__ __forceinline__ void fold_raw(const float4 &p, const float4 &q, const float4 &s, float4 &f0, float4 &f1,
                                         float4 &f2) {
    f0 = make_float4(p.x, p.y, (-0.5f * kLog2e) * p.z, (-kLog2e) * p.w);
    f1 = make_float4((-0.5f * kLog2e) * q.x, log2_fast(q.y), q.z, q.w);
    f2 = make_float4(s.x, q.y, 0.0f, 0.0f);
}

// A splat is "plain" when two of the per-pixel tests cannot fire: its conic is positive
// definite with margin (so the exponent is never positive, up to rounding at the very
// centre, where the exact value is 0) and amax < 0.985 (so amax exp(power) stays below
// the 0.99 clamp).  For plain splats the forward and the backward both drop the
// "exponent > 0" skip and the clamp; every other splat takes all tests.  Nearly every
// splat is plain (sigmoid opacities above 0.985 are rare).
__device__ __forceinline__ bool splat_plain(const float4 &p, const float4 &q) {
    const float a = p.z, b = p.w, c = q.x;
    return (a > 0.0f) & (c > 0.0f) & (a * c - b * b > 1e-5f * (a * c)) & (q.y < 0.985f);
}

__device__ __forceinline__ void fold_splat(const float4 *__restrict__ rec, uint32_t gi, float4 &f0, float4 &f1,
                                           float4 &f2) {
    fold_raw(rec[3 * (size_t)gi + 0], rec[3 * (size_t)gi + 1], rec[3 * (size_t)gi + 2], f0, f1, f2);
}

// Whether the splat can reach alpha >= 1/255 at some point of the pixel-centre box
// [x0,x1] x [y0,y1].  With d = point - m, alpha = amax 2^-P(d), P(d) = A dx^2 + 2B dx dy +
// C dy^2 (A = -qa, B = -qb / 2, C = -qc: the conic in log2 units), and alpha >= 1/255
// exactly where P(d) <= log2(255 amax).  For a positive definite P the smallest value over
// the box is 0 if the box holds the mean; otherwise it lies on a side of the box that faces
// the mean (from any other boundary point P decreases along a direction that stays in the
// box), where P is a parabola along the side: the side
// x = Xn (Xn the box's x-range clamped to 0; Xn = 0 when the range holds 0, which leaves a
// point of the box) takes its smallest value at y = -B Xn / C clamped to the side, and
// likewise the side y = Yn.  The smaller of the two values is the minimum.  It is compared
// with the bound inflated by 1% + 0.01 and by 1e-5 of the terms' magnitude -- far beyond
// FP32 rounding, the approximate reciprocals and the exponent's own error (1e-4 in log2
// units) -- so a splat that fails the test is skipped by every pixel of the box without
// changing any decision (P1, P2 and the magnitude are formed with FMAs; the margin covers
// either rounding).  A conic that is not positive definite with margin is never skipped;
// amax clearly below 1/255 always is.
__device__ __forceinline__ bool splat_reaches(const float4 &f0, const float4 &f1, float x0, float x1, float y0,
                                              float y1) {
    const float A = -f0.z, B = -0.5f * f0.w, C = -f1.x;
    const float thr = f1.y + 7.99435344f;  // log2(255 amax)
    const float X0 = x0 - f0.x, X1 = x1 - f0.x, Y0 = y0 - f0.y, Y1 = y1 - f0.y;
    const float Xn = __builtin_amdgcn_fmed3f(0.0f, X0, X1), Yn = __builtin_amdgcn_fmed3f(0.0f, Y0, Y1);
    const float ys = __builtin_amdgcn_fmed3f(-B * Xn * __builtin_amdgcn_rcpf(C), Y0, Y1);
    const float xs = __builtin_amdgcn_fmed3f(-B * Yn * __builtin_amdgcn_rcpf(A), X0, X1);
    const float B2 = 2.0f * B;
    const float P1 = __builtin_fmaf(Xn, __builtin_fmaf(A, Xn, B2 * ys), C * ys * ys);
    const float P2 = __builtin_fmaf(xs, __builtin_fmaf(A, xs, B2 * Yn), C * Yn * Yn);
    const float mag = __builtin_fmaf(A, __builtin_fmaf(Xn, Xn, xs * xs), C * __builtin_fmaf(ys, ys, Yn * Yn));
    // the flags are combined without short-circuit branches (straight-line code); amax
    // clearly below 1/255: no point keeps it
    const bool pd = (A > 0.0f) & (C > 0.0f) & (A * C - B * B > 1e-5f * (A * C));
    const bool near = fminf(P1, P2) <= __builtin_fmaf(thr, 1.01f, __builtin_fmaf(1e-5f, mag, 0.01f));
    return !(thr < -0.02f) & (!pd | near);
}

// The exponent over one wavefront's pixel region, expanded about the region's centre
// (xc, yc): with (dx, dy) = (xc, yc) - m and the pixel's offset (u, v) from the centre,
//   q = K + Lx u + Ly v + qa u^2 + qb u v + qc v^2,
//   K = qa dx^2 + qb dx dy + qc dy^2 + la,  Lx = 2 qa dx + qb dy,  Ly = qb dx + 2 qc dy.
// K, Lx, Ly are formed once per (region, splat) -- by the forward while it stages a
// batch, by the backward for each of its quadrants -- with these same instructions, and
// q per pixel by sq_exponent (five FMAs with the lane's constants u, v, u^2, u v, v^2,
// all exact), so the forward and the backward take every decision on the same FP32
// value.  Offsets from the centre (|u|, |v| <= 3.5 on an 8 x 8 square) keep the terms
// small: against an FP64 evaluation the error of q stays within 1e-4 (log2 units).
__device__ __forceinline__ float4 square_coeffs(const float4 &f0, const float4 &f1, float xc, float yc) {
    const float dx = xc - f0.x, dy = yc - f0.y;
    const float qbdy = f0.w * dy;
    const float Lx = __builtin_fmaf(2.0f * f0.z, dx, qbdy);
    const float Ly = __builtin_fmaf(2.0f * f1.x, dy, f0.w * dx);
    const float K = __builtin_fmaf(__builtin_fmaf(f0.z, dx, qbdy), dx, __builtin_fmaf(f1.x * dy, dy, f1.y));
    return make_float4(K, Lx, Ly, 0.0f);
}

// a lane's pixel as an offset from the region's centre
struct PixUV {
    float u, v, uu, uv, vv;
};

__device__ __forceinline__ PixUV pix_uv(float u, float v) { return {u, v, u * u, u * v, v * v}; }

// q at pixel p of a splat with region coefficients (K, Lx, Ly) and exponent constants
// (qa, qb, qc)
__device__ __forceinline__ float sq_exponent(float K, float Lx, float Ly, float qa, float qb, float qc,
                                             const PixUV &p) {
    return __builtin_fmaf(qc, p.vv, __builtin_fmaf(qb, p.uv, __builtin_fmaf(qa, p.uu,
                          __builtin_fmaf(Ly, p.v, __builtin_fmaf(Lx, p.u, K)))));
}

// --- tile order of the per-tile launches ---------------------------------------------
// The hardware deals a launch's workgroups round-robin to the 8 XCDs: block b runs on
// XCD b % 8, as the k-th (k = b / 8) workgroup that XCD receives.  A launch does upt
// units of work per tile (a unit being one workgroup); a tile's units run consecutively
// on one XCD and share its L2.  XCD x takes the tiles of rows x, x + 8, x + 16, ...: that
// spreads the scene's dense middle evenly (a contiguous band per XCD left the XCDs under
// it with twice the work of the others) and keeps the tiles an XCD renders, and the
// splats they share, within its L2.  Without a tile order an XCD takes its tiles row by
// row; with one (written by the binning: segment x holds XCD x's tiles, longest list
// first) it starts with its long lists, so that they do not run alone at the end.
__host__ __device__ inline int tile_grid(int TX, int TY, int upt) { return 8 * ((TY + 7) / 8) * TX * upt; }

// Division by a divisor d > 0 known on the host: m = div_magic(d) = floor((2^32 - 1) / d)
// gives n / d as mulhi(n, m) or one more (mulhi(n, m) > n / d - 1 for every 32-bit n), so
// one correction makes it exact.  With n, d and m uniform over a wavefront the whole
// division runs on the scalar unit (there is no scalar divide; the compiler's own
// expansion of an integer division uses the vector unit's reciprocal).
__host__ __device__ inline uint32_t div_magic(uint32_t d) { return 0xffffffffu / d; }

__device__ __forceinline__ uint32_t udiv_magic(uint32_t n, uint32_t d, uint32_t m, uint32_t &r) {
    uint32_t q = __umulhi(n, m);
    r = n - q * d;
    if (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

__device__ __forceinline__ int class_rows(int TY, int x) { return TY > x ? (TY - 1 - x) / 8 + 1 : 0; }

// (tx, ty): the tile's column and row; txm = div_magic(TX).
__device__ __forceinline__ bool tile_unit(int b, int TX, int TY, uint32_t txm, int upt,
                                          const uint32_t *__restrict__ order, int &tile, int &tx, int &ty, int &sub) {
    const int x = b & 7, k = b >> 3;
    const int j = k / upt;  // the XCD's j-th tile
    sub = k - j * upt;
    if (j >= TX * class_rows(TY, x)) return false;
    uint32_t r;
    if (order) {
        int off = 0;
        for (int y = 0; y < x; ++y) off += class_rows(TY, y);
        const uint32_t o = order[TX * off + j];
        if (o >= (uint32_t)(TX * TY)) return false;  // an order not written by the binning stays in bounds
        tile = (int)o;
        ty = (int)udiv_magic(o, (uint32_t)TX, txm, r);
        tx = (int)r;
    } else {
        ty = x + 8 * (int)udiv_magic((uint32_t)j, (uint32_t)TX, txm, r);
        tx = (int)r;
        tile = ty * TX + tx;
    }
    return true;
}

// --- launchers (host side) ----------------------------------------------------------
struct SceneK {
    int n, deg;
    const float *mean, *scale, *quat, *opacity, *t_mean, *t_scale, *velocity, *sh;
};

SceneK make_scenek(const d4dgs_scene &s);

// Where a projection that also runs the binning's count pass writes (the counters of a
// workspace; they must be zero when the projection starts).
struct BinK {
    uint32_t *cnt_g, *cnt_n, *grp_off;
    int TX;
};

// mode 0: camera + time stage, no record; 1: camera + time stage, writes record; 2: time stage from record
// bin (optional): also run the binning's count pass (see BinK)
hipError_t launch_project(const SceneK &s, const CamK &c, float t, int mode, float *cam_rec, int cam_cap,
                          float4 *rec, uint32_t *count, uint32_t *block_sums, float2 *mdot, int motion,
                          hipStream_t st, const BinK *bin = nullptr);

// One request of a batched projection (kernel argument, by value).  bin.cnt_g non-null:
// the projection also runs the binning's count pass for this request (see BinK).
struct ReqK {
    CamK cam;
    float t;
    float4 *rec;
    uint32_t *count;
    uint32_t *partial;
    BinK bin;
};
constexpr int kMaxBatch = 16;  // requests per batched-projection launch
struct BatchArgs {
    int nreq;
    ReqK r[kMaxBatch];
};
hipError_t launch_project_batch(const SceneK &s, const BatchArgs &args, hipStream_t st);

// One frame of a fixed-viewpoint multi-timestamp projection (kernel argument, by value).
struct FrameK {
    float t;
    float4 *rec;
    uint32_t *count;
    uint32_t *partial;
};
constexpr int kMaxTimes = 16;  // frames per multi-timestamp projection launch
struct TimesArgs {
    int nt;
    int motion;  // d4dgs_motion of every frame
    FrameK f[kMaxTimes];
};
// mode as launch_project (0: no cache, 1: fill the cache, 2: from the cache)
hipError_t launch_project_times(const SceneK &s, const CamK &c, int mode, float *cam_rec, int cam_cap,
                                const TimesArgs &args, hipStream_t st);

struct SortWs {
    uint64_t *bucket;   // [capacity] per-tile buckets of (depth bits << 32 | gaussian)
    uint64_t *alt;      // [capacity] scratch of the large-bucket radix sort
    uint32_t *grp_off;  // [blocks][kCells] per-(block, tile) bucket reservations
    uint32_t *cnt_g;    // [tiles] grouped instance counters (zero between calls)
    uint32_t *cnt_n;    // [tiles] ungrouped instance counters (zero between calls)
    uint32_t *cur_n;    // [tiles] ungrouped bucket cursors
    uint32_t *misc;     // [64]: [0] instances kept, [1] status
    size_t counter_bytes;  // bytes from cnt_g to the end of cnt_n
};

size_t sort_workspace_bytes(int n, int64_t capacity, int tiles);
SortWs carve_workspace(void *ws, int n, int64_t capacity, int tiles);

// zeroes a workspace's tile counters (which every binning leaves zero)
hipError_t clear_bin_counters(const SortWs &ws, hipStream_t st);

// order (optional, [tiles]): receives the tiles longest list first
hipError_t launch_bin_sort(const float4 *rec, const uint32_t *count, uint32_t *offset, uint32_t *partial, int n,
                           const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                           int64_t *num_inst, int64_t capacity, int32_t *d_status, uint32_t *order,
                           hipStream_t st);

// The binning after a projection that counted (launch_project with a BinK): both scans
// in one launch, the scatter and the sort; leaves the counters zero.
hipError_t launch_bin_counted(const float4 *rec, const uint32_t *count, uint32_t *offset, uint32_t *partial, int n,
                              const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                              int64_t *num_inst, int64_t capacity, int32_t *d_status, uint32_t *order,
                              hipStream_t st);

// order (optional): the binning's tile order; e0/e1 (optional): events set to the blend
// kernel's own start and end
hipError_t launch_blend(const float4 *rec, const uint32_t *vals, const uint32_t *ranges, const uint32_t *order,
                        const CamK &c, const float bg[3], float *img, float *final_T, uint32_t *n_contrib,
                        hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// the blend with the optical flow: mdot [n] per splat, flow [2][H][W]
hipError_t launch_blend_flow(const float4 *rec, const float2 *mdot, const uint32_t *vals, const uint32_t *ranges,
                             const uint32_t *order, const CamK &c, const float bg[3], float *img, float *flow, float *final_T,
                             uint32_t *n_contrib, hipStream_t st);

// mdot / dL_dflow NULL: colour only; e0/e1 (optional): events set to the kernel's own start and end
hipError_t launch_blend_bwd(const float4 *rec, const uint32_t *offset, const uint32_t *vals,
                            const uint32_t *ranges, const uint32_t *order, const CamK &c, const float bg[3], const float *final_T,
                            const uint32_t *n_contrib, const float *dL_dimg, const float2 *mdot,
                            const float *dL_dflow, float4 *inst_grads, int64_t capacity, hipStream_t st,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

size_t flow_loss_workspace_bytes(int W, int H);
hipError_t launch_flow_loss(const float *img, const float *flow, int W, int H, float lambda, float eps, void *ws,
                            float *loss, float *dL_dflow, hipStream_t st);

hipError_t launch_project_bwd(const SceneK &s, const CamK &c, float t, const float4 *rec, const uint32_t *count,
                              const uint32_t *offset, const float4 *inst_grads, int64_t capacity,
                              const d4dgs_grads &g, int motion, hipStream_t st, hipEvent_t e0 = nullptr,
                              hipEvent_t e1 = nullptr);

// spatial order of a scene (a one-time step): perm [n]; workspace of
// spatial_order_workspace_bytes(n)
size_t spatial_order_workspace_bytes(int n);
hipError_t launch_spatial_order(const float *mean, int n, uint32_t *perm, void *ws, hipStream_t st);
// dst[c][j] = src[c][perm[j]], planar [comps][n]
hipError_t launch_permute(const float *src, float *dst, const uint32_t *perm, int n, int comps, hipStream_t st);

void set_error(const std::string &msg);

}  // namespace d4
