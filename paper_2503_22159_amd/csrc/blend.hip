// Per-tile front-to-back alpha blending (Eq. 4 with alpha_i = o_i w_i G'_i).
//
// A 16x16 tile is rendered by one workgroup of 4 / PX wavefronts.  Each wavefront owns
// an RW x (64 / RW) PX pixel region of the tile: lane l has column l % RW and rows
// l / RW + (64 / RW) k, k < PX.  Each wavefront walks the tile's depth-sorted list in
// batches of 64: every lane gathers one splat record, folds it (exponent constants, log2
// of the peak opacity), forms the exponent's coefficients about the centre of the
// wavefront's region and parks them in LDS; then the wave steps through the batch reading
// each splat as an LDS broadcast, five FMAs giving a pixel's exponent.  The wavefronts of
// a tile work independently, each on LDS of its own (no workgroup barriers); one
// workgroup per tile rather than per wavefront quarters the workgroups the hardware
// dispatches (measured 3 % faster).  A wave stops as soon as all of its pixels are
// saturated.
//
// Launch order (tile_unit): XCD x takes every eighth row of tiles from row x, in the
// binning's longest-first order when it is given.
#include <hip/hip_ext.h>

#include "internal.hpp"

namespace d4 {

namespace {

// Per pixel row k, "done" (saturated, or outside the image) is a wave-uniform lane mask kept
// in scalar registers; the per-pixel skip / stop / blend decisions are formed as lane masks
// (ballots of the compares) and applied with inverse ballots.  A done pixel neither blends
// nor changes: T keeps the transmittance it had before the splat that stopped it.
//
// Staging culls: each lane tests whether its own splat can reach alpha >= 1/255 anywhere in
// the wavefront's pixel-centre box (splat_reaches: the ellipse against the box, exactly up
// to a margin) and only the splats that can reach one of its pixels are parked, compacted
// in list order (ballot + lane-rank), so the per-splat loop carries no test.
// One splat against the lane's PX pixels: g0 = {K, Lx, Ly, qa}, g1 = {qb, qc, r, g},
// g2 = {b, tag, la, -} (see square_coeffs), md = dm/dt.  PLAIN: the splat passed
// splat_plain, so the "exponent > 0" skip and the 0.99 clamp cannot fire and are not
// evaluated.
template <int PX, bool STATE, bool PLAIN, bool FLOW>
__device__ __forceinline__ void blend_splat(const float4 &g0, const float4 &g1, const float4 &g2, float2 md,
                                            uint32_t pos, const PixUV (&p)[PX], float (&T)[PX], float (&C0)[PX],
                                            float (&C1)[PX], float (&C2)[PX], float (&F0)[PX], float (&F1)[PX],
                                            uint64_t (&done)[PX], uint32_t (&last)[PX]) {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const float q = sq_exponent(g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, p[k]);
        const float e = exp2_fast(q);
        const float alpha = PLAIN ? e : fminf(kAlphaMax, e);
        uint64_t ok = __ballot(alpha >= kAlphaMin) & ~done[k];
        if (!PLAIN) ok &= __ballot(!(q > g2.z));
        const float Tk = T[k];
        const float Tn = __builtin_fmaf(-alpha, Tk, Tk);  // T (1 - alpha)
        const uint64_t stop = ok & __ballot(Tn < kTMin);
        const bool blend = __builtin_amdgcn_inverse_ballot_w64(ok & ~stop);
        done[k] |= stop;
        const float wgt = blend ? alpha * Tk : 0.0f;
        C0[k] = __builtin_fmaf(g1.z, wgt, C0[k]);
        C1[k] = __builtin_fmaf(g1.w, wgt, C1[k]);
        C2[k] = __builtin_fmaf(g2.x, wgt, C2[k]);
        if (FLOW) {
            F0[k] = __builtin_fmaf(md.x, wgt, F0[k]);
            F1[k] = __builtin_fmaf(md.y, wgt, F1[k]);
        }
        T[k] = blend ? Tn : Tk;
        if (STATE) last[k] = blend ? pos : last[k];
    }
}

// Orders a wavefront's LDS writes before its later reads of other lanes' entries (and
// the reads before the next writes): LDS accesses of one wavefront complete in order, so
// this costs no instruction; it keeps the compiler from moving accesses across it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// True when every pixel of the wavefront is done.
template <int PX>
__device__ __forceinline__ bool wave_done(const uint64_t (&done)[PX]) {
    uint64_t all = ~0ull;
#pragma unroll
    for (int k = 0; k < PX; ++k) all &= done[k];
    return all == ~0ull;
}

template <int PX, int RW, bool STATE, bool FLOW>
__global__ __launch_bounds__(4 * kWave) void k_blend(const float4 *__restrict__ rec, const uint32_t *__restrict__ vals,
                                                 const uint32_t *__restrict__ ranges,
                                                 const uint32_t *__restrict__ order, CamK c, float bg0, float bg1,
                                                 float bg2, float *__restrict__ img, float *__restrict__ final_T,
                                                 uint32_t *__restrict__ ncontrib,
                                                 const float2 *__restrict__ mdot, float *__restrict__ flow) {
    constexpr int LR = kWave / RW;      // lane rows
    constexpr int RH = LR * PX;         // rows of the wavefront's pixel region (RW x RH)
    constexpr int NXR = kTile / RW;     // regions across a tile
    constexpr int WPT = 4 / PX;         // waves per tile
    static_assert(RH <= kTile && (RW == 8 || RW == 16), "wavefront region must tile a 16x16 tile");
    // staged splat i of wavefront w: S0[w][i] = {K, Lx, Ly, qa}, S1[w][i] = {qb, qc, r, g},
    // S2[w][i] = {b, bits(plain << 31 | list position + 1), la, -}, S3[w][i] = dm/dt (flow
    // only): arrays of one stride, so that one address register serves every read
    __shared__ float4 S0[WPT][kWave], S1[WPT][kWave], S2[WPT][kWave];
    __shared__ float2 S3[FLOW ? WPT : 1][FLOW ? kWave : 1];
    int tile, tx, ty, unused;
    if (!tile_unit(blockIdx.x, c.TX, c.TY, c.txm, 1, order, tile, tx, ty, unused)) return;  // uniform per workgroup
    const int sub = threadIdx.x / kWave;
    float4 *s0 = S0[sub], *s1 = S1[sub], *s2 = S2[sub];
    float2 *s3 = S3[FLOW ? sub : 0];
    // the wavefront's region, from the wave index in a scalar register (integer work on
    // the scalar unit); the LDS arrays keep the vector form, which the loop addresses best
    const int wsub = __builtin_amdgcn_readfirstlane(sub);
    const int rx0 = tx * kTile + (wsub % NXR) * RW, ry0 = ty * kTile + (wsub / NXR) * RH;
    const int ln = lane_id();
    const int px = rx0 + ln % RW;
    // pixel-centre box of this wavefront (for skipping splats that cannot reach it) and
    // its centre, about which the exponent is expanded
    const float wx0 = (float)rx0 + 0.5f, wx1 = wx0 + (float)(RW - 1);
    const float wy0 = (float)ry0 + 0.5f, wy1 = wy0 + (float)(RH - 1);
    const float xc = (float)rx0 + 0.5f * RW, yc = (float)ry0 + 0.5f * RH;
    PixUV p[PX];
    float T[PX], C0[PX], C1[PX], C2[PX], F0[PX], F1[PX];
    uint64_t done[PX];
    uint32_t last[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int py = ry0 + ln / RW + LR * k;
        p[k] = pix_uv((float)(ln % RW) + 0.5f - 0.5f * RW, (float)(ln / RW + LR * k) + 0.5f - 0.5f * RH);
        T[k] = 1.0f;
        done[k] = __ballot(!(px < c.W && py < c.H));
        C0[k] = C1[k] = C2[k] = F0[k] = F1[k] = 0.0f;
        last[k] = 0u;
    }
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    // software pipeline: list entries two batches ahead, records one batch ahead (a lane
    // reads its record registers only for list entries it has loaded)
    float4 n0, n1, n2;
    float2 nm;
    if (start + ln < end) {
        const uint32_t g = vals[start + ln];
        n0 = rec[3 * (size_t)g];
        n1 = rec[3 * (size_t)g + 1];
        n2 = rec[3 * (size_t)g + 2];
        if (FLOW) nm = mdot[g];
    }
    uint32_t gnext = start + kWave + ln < end ? vals[start + kWave + ln] : 0u;
    for (uint32_t j0 = start; j0 < end; j0 += kWave) {
        if (wave_done(done)) break;
        bool keep = false, plain = false;
        float4 f0, f1, f2;
        if (j0 + ln < end) {
            fold_raw(n0, n1, n2, f0, f1, f2);
            keep = splat_reaches(f0, f1, wx0, wx1, wy0, wy1);
            plain = splat_plain(n0, n1);
        }
        const uint64_t km = __ballot(keep);
        const int nb = __popcll(km);
        if (keep) {
            const int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
            const float4 sc = square_coeffs(f0, f1, xc, yc);
            s0[pos] = make_float4(sc.x, sc.y, sc.z, f0.z);
            s1[pos] = make_float4(f0.w, f1.x, f1.z, f1.w);
            s2[pos] = make_float4(f2.x, __uint_as_float((plain ? 0x80000000u : 0u) | (j0 - start + ln + 1)), f1.y,
                                  0.0f);
            if (FLOW) s3[pos] = nm;
        }
        wave_sync();
        if (j0 + kWave + ln < end) {
            n0 = rec[3 * (size_t)gnext];
            n1 = rec[3 * (size_t)gnext + 1];
            n2 = rec[3 * (size_t)gnext + 2];
            if (FLOW) nm = mdot[gnext];
        }
        if (j0 + 2 * kWave + ln < end) gnext = vals[j0 + 2 * kWave + ln];
        // batches made only of plain splats (nearly all) run the loop without the
        // positive-exponent test and the clamp
        if (__ballot(keep && !plain) == 0) {
            for (int i = 0; i < nb; ++i) {
                const float4 g2 = make_float4(s2[i].x, s2[i].y, 0.f, 0.f);
                const float2 md = FLOW ? s3[i] : make_float2(0.f, 0.f);
                const uint32_t pos = __float_as_uint(g2.y) & 0x7fffffffu;
                blend_splat<PX, STATE, true, FLOW>(s0[i], s1[i], g2, md, pos, p, T, C0, C1, C2, F0, F1, done, last);
                if (wave_done(done)) break;
            }
        } else {
            for (int i = 0; i < nb; ++i) {
                const float4 g2 = s2[i];
                const float2 md = FLOW ? s3[i] : make_float2(0.f, 0.f);
                const uint32_t pos = __float_as_uint(g2.y) & 0x7fffffffu;
                if (__builtin_amdgcn_readfirstlane(__float_as_uint(g2.y)) >> 31)
                    blend_splat<PX, STATE, true, FLOW>(s0[i], s1[i], g2, md, pos, p, T, C0, C1, C2, F0, F1, done,
                                                       last);
                else
                    blend_splat<PX, STATE, false, FLOW>(s0[i], s1[i], g2, md, pos, p, T, C0, C1, C2, F0, F1, done,
                                                        last);
                if (wave_done(done)) break;
            }
        }
        wave_sync();
    }
    const size_t plane = (size_t)c.W * c.H;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
        const int py = ry0 + ln / RW + LR * k;
        if (px >= c.W || py >= c.H) continue;
        const size_t pi = (size_t)py * c.W + px;
        img[pi] = C0[k] + T[k] * bg0;
        img[plane + pi] = C1[k] + T[k] * bg1;
        img[2 * plane + pi] = C2[k] + T[k] * bg2;
        if (STATE) {
            final_T[pi] = T[k];
            ncontrib[pi] = last[k];
        }
        if (FLOW) {
            flow[pi] = F0[k];
            flow[plane + pi] = F1[k];
        }
    }
}

// With events e0/e1 the launch goes through hipExtLaunchKernel, which sets them to the
// kernel's own start and end (a stream-ordered event pair would also time the dispatch).
template <int PX, int RW, bool STATE>
void launch_px(const float4 *rec, const uint32_t *vals, const uint32_t *ranges, const uint32_t *order, const CamK &c,
               const float bg[3], float *img, float *final_T, uint32_t *n_contrib, hipStream_t st, hipEvent_t e0,
               hipEvent_t e1) {
    const dim3 grid(tile_grid(c.TX, c.TY, 1)), block(kWave * (4 / PX));
    const float2 *no_mdot = nullptr;
    float *no_flow = nullptr;
    if (e0)
        hipExtLaunchKernelGGL((k_blend<PX, RW, STATE, false>), grid, block, 0, st, e0, e1, 0, rec, vals, ranges, order,
                              c, bg[0], bg[1], bg[2], img, final_T, n_contrib, no_mdot, no_flow);
    else
        hipLaunchKernelGGL((k_blend<PX, RW, STATE, false>), grid, block, 0, st, rec, vals, ranges, order, c, bg[0],
                           bg[1], bg[2], img, final_T, n_contrib, no_mdot, no_flow);
}

}  // namespace

hipError_t launch_blend(const float4 *rec, const uint32_t *vals, const uint32_t *ranges, const uint32_t *order,
                        const CamK &c, const float bg[3], float *img, float *final_T, uint32_t *n_contrib,
                        hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (c.TX * c.TY == 0) return hipSuccess;
    // the wavefront region is a template parameter (PX pixels per lane in one column, RW
    // columns): 8x8 with one pixel per lane measured fastest of 8x8, 16x4, 8x16 and 16x16
    if (final_T)
        launch_px<1, 8, true>(rec, vals, ranges, order, c, bg, img, final_T, n_contrib, st, e0, e1);
    else
        launch_px<1, 8, false>(rec, vals, ranges, order, c, bg, img, final_T, n_contrib, st, e0, e1);
    return hipGetLastError();
}

hipError_t launch_blend_flow(const float4 *rec, const float2 *mdot, const uint32_t *vals, const uint32_t *ranges,
                             const uint32_t *order, const CamK &c, const float bg[3], float *img, float *flow, float *final_T,
                             uint32_t *n_contrib, hipStream_t st) {
    if (c.TX * c.TY == 0) return hipSuccess;
    const dim3 grid(tile_grid(c.TX, c.TY, 1)), block(4 * kWave);  // one pixel per lane, 8x8 squares
    if (final_T)
        hipLaunchKernelGGL((k_blend<1, 8, true, true>), grid, block, 0, st, rec, vals, ranges, order, c,
                           bg[0], bg[1], bg[2], img, final_T, n_contrib, mdot, flow);
    else
        hipLaunchKernelGGL((k_blend<1, 8, false, true>), grid, block, 0, st, rec, vals, ranges,
                           order, c, bg[0], bg[1], bg[2], img, final_T, n_contrib, mdot, flow);
    return hipGetLastError();
}

}  // namespace d4
