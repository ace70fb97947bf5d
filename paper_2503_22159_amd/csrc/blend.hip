// Per-tile front-to-back alpha blending (Eq. 4 with alpha_i = o_i w_i G'_i).
//
// One wavefront renders one 16x16 tile, four pixels per lane (lane l owns column l % 16
// and rows l / 16 + 4k).  The wave walks the tile's depth-sorted list in order; the list
// index, the Gaussian index and its 48-byte splat record are the same for every lane,
// so they are loaded once per wave (scalar loads) and broadcast -- no LDS staging and no
// block barriers.  The wave stops as soon as all of its pixels are saturated
// (transmittance would drop below 1e-4), a wave-wide vote.
//
// Launch order is XCD-aware: the hardware deals consecutive workgroups round-robin to the
// 8 XCDs, so block b renders tile (b % 8) * per_xcd + b / 8 -- each XCD gets a contiguous
// band of tiles, and neighbouring tiles, which share splats, share that XCD's L2.
#include "internal.hpp"

namespace d4 {

namespace {

constexpr int kPx = 4;  // pixels per lane

__global__ __launch_bounds__(kWave) void k_blend(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                 const uint32_t *__restrict__ ranges, CamK c, float bg0, float bg1,
                                                 float bg2, float *__restrict__ img, float *__restrict__ final_T,
                                                 uint32_t *__restrict__ ncontrib, int ntiles, int per_xcd) {
    const int b = blockIdx.x;
    const int tile = (b & 7) * per_xcd + (b >> 3);
    if (tile >= ntiles) return;
    const int tx = tile % c.TX, ty = tile / c.TX;
    const int ln = lane_id();
    const int px = tx * kTile + (ln & 15);
    float sx = (float)px + 0.5f, sy[kPx];
    bool in[kPx], done[kPx];
    float T[kPx], C0[kPx], C1[kPx], C2[kPx];
    uint32_t last[kPx];
#pragma unroll
    for (int k = 0; k < kPx; ++k) {
        const int py = ty * kTile + (ln >> 4) + 4 * k;
        sy[k] = (float)py + 0.5f;
        in[k] = px < c.W && py < c.H;
        done[k] = !in[k];
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = 0.0f;
        last[k] = 0u;
    }
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    for (uint32_t j = start; j < end; ++j) {
        const bool alldone = done[0] && done[1] && done[2] && done[3];
        if (__all(alldone)) break;
        const uint32_t gi = vals[j];
        const SplatK s = load_splat(rec, gi);
#pragma unroll
        for (int k = 0; k < kPx; ++k) {
            const float dx = sx - s.mx, dy = sy[k] - s.my;
            const float q = splat_exponent(s, dx, dy);
            const float alpha = fminf(kAlphaMax, s.amax * exp2_fast(q));
            const bool ok = !done[k] && q <= 0.0f && alpha >= kAlphaMin;
            const float Tn = T[k] * (1.0f - alpha);
            const bool stop = ok && Tn < kTMin;
            const bool blend = ok && !stop;
            const float wgt = blend ? alpha * T[k] : 0.0f;
            C0[k] = __builtin_fmaf(s.r, wgt, C0[k]);
            C1[k] = __builtin_fmaf(s.g, wgt, C1[k]);
            C2[k] = __builtin_fmaf(s.b, wgt, C2[k]);
            T[k] = blend ? Tn : T[k];
            last[k] = blend ? (j - start + 1) : last[k];
            done[k] = done[k] || stop;
        }
    }
    const size_t plane = (size_t)c.W * c.H;
#pragma unroll
    for (int k = 0; k < kPx; ++k) {
        if (!in[k]) continue;
        const int py = ty * kTile + (ln >> 4) + 4 * k;
        const size_t pi = (size_t)py * c.W + px;
        img[pi] = C0[k] + T[k] * bg0;
        img[plane + pi] = C1[k] + T[k] * bg1;
        img[2 * plane + pi] = C2[k] + T[k] * bg2;
        if (final_T) final_T[pi] = T[k];
        if (ncontrib) ncontrib[pi] = last[k];
    }
}

}  // namespace

hipError_t launch_blend(const float4 *rec, const uint32_t *vals, const uint32_t *ranges, const CamK &c,
                        const float bg[3], float *img, float *final_T, uint32_t *n_contrib, hipStream_t st) {
    const int ntiles = c.TX * c.TY;
    if (ntiles == 0) return hipSuccess;
    const int per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL(k_blend, dim3(per_xcd * 8), dim3(kWave), 0, st, rec, vals, ranges, c, bg[0], bg[1], bg[2],
                       img, final_T, n_contrib, ntiles, per_xcd);
    return hipGetLastError();
}

}  // namespace d4
