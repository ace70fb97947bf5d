// Adjoint of the render path (the differentiable pipeline of Fig. 3).
//
// k_blend_bwd   one 4-wave workgroup per 16x16 tile, a wavefront per 8x8 quadrant, one
//               pixel per lane, walking the tile's list from the tile's last contributor
//               back to the front.  Each pixel's transmittance is replayed backwards
//               from its final value, T_i = T_{i+1} / (1 - alpha_i), and, with g = dL/dC
//               the pixel's upstream
//               gradient and S_i = sum_{j>i} c_j alpha_j T_j + T_final bg the colour
//               behind splat i, the scalar g.S_i is carried along, so
//                 dL/dc_i     = g alpha_i T_i
//                 dL/dalpha_i = (g.c_i) T_i - (g.S_i) / (1 - alpha_i).
//               No per-splat forward state is stored.  alpha_i is recomputed by the same
//               instructions as the forward, so skip decisions match exactly.
//               Splats that cannot reach alpha >= 1/255 at a pixel of the quadrant
//               (splat_reaches) are dropped while a batch is staged (their gradient is
//               zero); the rest are compacted.  Per splat a
//               lane sums over its pixels dp = dL/dpower and its moments about the splat
//               mean (dp dx, dp dy, dp dx^2, dp dx dy, dp dy^2; d = pixel - m) and the
//               three colour gradients; the wave reduces the nine sums with cross-lane
//               moves (no LDS), and after the batch one lane per splat turns the moments
//               into the gradients of the 2D mean, the conic and amax and writes the
//               instance's own slot: slot = offset[g] + position of the tile inside g's
//               rectangle, i.e. the instance's pre-sort emission index.  Every slot is
//               written exactly once; no atomics.
// k_project_bwd one thread per Gaussian: sums its contiguous slots in a fixed order
//               (deterministic), then applies the chain rule through the time stage
//               (alpha_max = o w, w = exp(-tau^2 / 2 s_t^2), m = m0 + tau mdot, Jacobian at
//               the moved mean, Sigma' = J V J^T + 0.3 I, conic = Sigma'^-1) and the camera
//               stage (V = R Sigma R^T, Sigma = (Rq S)(Rq S)^T, normalised quaternion,
//               p = R mu + T, u = R v, spherical-harmonic colour along mu - campos).
//               Adds into the caller's gradient arrays.
#include <hip/hip_ext.h>

#include "internal.hpp"

namespace d4 {

namespace {


__device__ __forceinline__ uint32_t inst_slot(const float4 &r2, uint32_t off, int tx, int ty) {
    const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
    const uint32_t x0 = lo & 0xffffu, y0 = lo >> 16, x1 = hi & 0xffffu;
    return off + ((uint32_t)ty - y0) * (x1 - x0) + ((uint32_t)tx - x0);
}

__device__ __forceinline__ void zero_slot(float4 *__restrict__ ig, uint32_t slot) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    ig[3 * (size_t)slot + 0] = z;
    ig[3 * (size_t)slot + 1] = z;
    ig[3 * (size_t)slot + 2] = z;
}

// Cross-lane moves within a row of 16 lanes (DPP): quad permutations [1,0,3,2] and
// [2,3,0,1] (partner lane l ^ 1, l ^ 2) and row rotations by 4 and 8.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRor4 = 0x124, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// v + v of lane l ^ 16, and v + v of lane l ^ 32 (row swaps).
__device__ __forceinline__ float sum_xor16(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float sum_xor32(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wavefront total of y, in every lane.
__device__ __forceinline__ float wave_allsum(float y) {
    y += dpp_move<kDppXor1>(y);
    y += dpp_move<kDppXor2>(y);
    y += dpp_move<kDppRor4>(y);
    y += dpp_move<kDppRor8>(y);
    return sum_xor32(sum_xor16(y));
}

// Which of the eight reduce-scattered values lane l holds after wave_sum9.
__device__ __forceinline__ int red_index(int l) { return 4 * (l & 1) + 2 * ((l >> 1) & 1) + ((l >> 2) & 1); }

// Wavefront totals of nine per-lane values.  v[0..7] are reduce-scattered over the low
// three lane bits -- at each step a lane keeps half of its values and adds its partner's
// copy of that half (partners: l ^ 1, l ^ 2, then a rotation by 4 inside the row, which
// pairs every lane with one of equal bits 0-1 and opposite bit 2) -- and then summed
// over the other lanes; lane l ends with the total of v[red_index(l)] in x.  y is the
// total of v[8].
__device__ __forceinline__ void wave_sum9(const float v[9], float &x, float &y) {
    const int l = lane_id();
    const bool b0 = l & 1, b1 = (l >> 1) & 1, b2 = (l >> 2) & 1;
    float u[4], w[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float keep = b0 ? v[j + 4] : v[j], send = b0 ? v[j] : v[j + 4];
        u[j] = keep + dpp_move<kDppXor1>(send);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float keep = b1 ? u[j + 2] : u[j], send = b1 ? u[j] : u[j + 2];
        w[j] = keep + dpp_move<kDppXor2>(send);
    }
    {
        const float keep = b2 ? w[1] : w[0], send = b2 ? w[0] : w[1];
        x = keep + dpp_move<kDppRor4>(send);
    }
    x += dpp_move<kDppRor8>(x);
    x = sum_xor32(sum_xor16(x));
    y = wave_allsum(v[8]);
}

// FLOW: the flow F = sum mdot alpha T (background 0) is two more colour channels with
// upstream gradient dLf; their colour gradients dL/dmdot go to the slot's third float4.
//
// One workgroup of four wavefronts per tile; wavefront w owns the 8x8 quadrant
// (w & 1, w >> 1), one pixel per lane.  Per batch of 64 list entries (last batch first):
// wavefront 0 stages the splats once; each wavefront culls them against its quadrant
// and walks its kept splats from the back (a scalar bit mask), reducing its nine (or
// eleven) per-splat sums into LDS; then 64 threads add the four quadrants' sums in a
// fixed order, form the splat gradients and write the instance slots.  Splitting a tile
// over four wavefronts shortens the serial chain of the longest tiles fourfold.
constexpr int kBwdThreads = 4 * kWave;

// The colour-only kernel is held to 64 VGPRs (8 waves per SIMD; it fits without
// spilling); the flow kernel keeps its larger register set.
template <bool FLOW>
__global__ __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(FLOW ? 1 : 8))) void k_blend_bwd(const float4 *__restrict__ rec,
                                                           const uint32_t *__restrict__ offset,
                                                           const uint32_t *__restrict__ vals,
                                                           const uint32_t *__restrict__ ranges,
                                                           const uint32_t *__restrict__ order, CamK c, float bg0,
                                                           float bg1, float bg2, const float *__restrict__ final_T,
                                                           const uint32_t *__restrict__ ncontrib,
                                                           const float *__restrict__ dL, float4 *__restrict__ ig,
                                                           uint32_t capacity, const float2 *__restrict__ mdot,
                                                           const float *__restrict__ dLf) {
    constexpr int NR = FLOW ? 11 : 9;  // sums reduced per splat
    int tile, tx, ty, unused;
    if (!tile_unit(blockIdx.x, c.TX, c.TY, c.txm, 1, order, tile, tx, ty, unused)) return;  // the same for the whole workgroup
    const int tid = threadIdx.x, w = tid / kWave, ln = lane_id();
    const size_t plane = (size_t)c.W * c.H;
    // this wavefront's 8x8 quadrant and this lane's pixel
    const int qx0 = tx * kTile + (w & 1) * 8, qy0 = ty * kTile + (w >> 1) * 8;
    const int px = qx0 + (ln & 7), py = qy0 + (ln >> 3);
    const float sx = (float)px + 0.5f, sy = (float)py + 0.5f;
    const float wx0 = (float)qx0 + 0.5f, wx1 = wx0 + 7.0f, wy0 = (float)qy0 + 0.5f, wy1 = wy0 + 7.0f;
    // the forward's exponent: coefficients about the quadrant's centre, the lane's offset
    const float xc = (float)qx0 + 4.0f, yc = (float)qy0 + 4.0f;
    const PixUV pu = pix_uv((float)(ln & 7) - 3.5f, (float)(ln >> 3) - 3.5f);
    const bool in = px < c.W && py < c.H;
    const size_t pi = (size_t)py * c.W + px;
    float Tc = in ? final_T[pi] : 1.0f;
    const uint32_t nc = in ? ncontrib[pi] : 0u;
    const float g0 = in ? dL[pi] : 0.0f, g1 = in ? dL[plane + pi] : 0.0f, g2 = in ? dL[2 * plane + pi] : 0.0f;
    const float g3 = FLOW && in ? dLf[pi] : 0.0f, g4 = FLOW && in ? dLf[plane + pi] : 0.0f;
    float GS = Tc * (g0 * bg0 + g1 * bg1 + g2 * bg2);  // g . S with S = T_final bg
    // tile-wide last contributor
    __shared__ uint32_t wmax[4];
    const uint32_t wm = __builtin_amdgcn_readfirstlane(wave_max_u32(nc));
    if (ln == 0) wmax[w] = wm;
    __syncthreads();
    const uint32_t nmax = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    // instances behind every pixel's last contributor get zero gradients
    for (uint32_t j = start + nmax + tid; j < end; j += kBwdThreads) {
        const uint32_t gi = vals[j];
        const uint32_t slot = inst_slot(rec[3 * (size_t)gi + 2], offset[gi], tx, ty);
        if (slot < capacity) zero_slot(ig, slot);  // false only after an instance overflow
    }
    // staged batch: s2 = {b, bits(plain << 31 | list position), -, -},
    // s3 = {conic a, b, c, amax}
    __shared__ float4 s0[kWave], s1[kWave], s2[kWave], s3[kWave];
    __shared__ uint32_t sslot[kWave];
    __shared__ float2 s4[FLOW ? kWave : 1];  // mdot
    __shared__ uint64_t kmask[4];
    __shared__ float4 sqc[4][kWave];  // per quadrant: {K, Lx, Ly, -} of the staged splats it keeps
    __shared__ float red[4 * kWave * NR];
    for (uint32_t jb = start + nmax; jb > start;) {
        const uint32_t j0 = jb - start > (uint32_t)kWave ? jb - kWave : start;
        const uint32_t nb = jb - j0;
        if (w == 0 && (uint32_t)ln < nb) {
            const uint32_t j = j0 + ln;
            const uint32_t gi = vals[j];
            const float4 r0 = rec[3 * (size_t)gi + 0], r1 = rec[3 * (size_t)gi + 1], r2 = rec[3 * (size_t)gi + 2];
            float4 f0, f1, f2;
            fold_raw(r0, r1, r2, f0, f1, f2);
            s0[ln] = f0;
            s1[ln] = f1;
            s2[ln] = make_float4(f2.x, __uint_as_float((splat_plain(r0, r1) ? 0x80000000u : 0u) | (j - start)), 0.0f,
                                 0.0f);
            s3[ln] = make_float4(r0.z, r0.w, r1.x, r1.y);
            sslot[ln] = inst_slot(r2, offset[gi], tx, ty);
            if (FLOW) s4[ln] = mdot[gi];
        }
        __syncthreads();
        // this quadrant's splats: lane i tests staged splat i
        bool keep = false;
        if ((uint32_t)ln < nb) {
            const float4 h0 = s0[ln];
            keep = splat_reaches(h0, s1[ln], wx0, wx1, wy0, wy1);
            if (keep) sqc[w][ln] = square_coeffs(h0, s1[ln], xc, yc);
        }
        // sqc[w] is written and read by this wavefront alone (LDS accesses of a wavefront
        // complete in order); keep the compiler from moving the reads above the writes
        __builtin_amdgcn_wave_barrier();
        uint64_t km = __ballot(keep);
        // splats that no pixel of the quadrant blends (behind every pixel's last
        // contributor, or below 1/255 at every pixel) contribute exact zeros: they are
        // dropped from the quadrant's mask instead of reduced
        uint64_t used = km;
        while (km) {
            const int i = 63 - __builtin_clzll(km);  // from the back of the list
            km &= ~(1ull << i);
            const float4 h0 = s0[i], h1 = s1[i];
            const float2 h2 = *reinterpret_cast<const float2 *>(&s2[i]);
            const uint32_t tag = __builtin_amdgcn_readfirstlane(__float_as_uint(h2.y));
            const uint32_t jj = tag & 0x7fffffffu;  // position in the tile's list
            const uint64_t live = __ballot(jj < nc);
            if (live == 0) {
                used &= ~(1ull << i);
                continue;
            }
            // the forward's per-splat tests: no "exponent > 0" skip for plain splats
            const uint64_t pos_ok = (tag >> 31) ? ~0ull : 0ull;
            const float dx = sx - h0.x, dy = sy - h0.y;
            const float4 kc = sqc[w][i];
            const float q = sq_exponent(kc.x, kc.y, kc.z, h0.z, h0.w, h1.x, pu);
            const float e = exp2_fast(q);
            const float alpha = fminf(kAlphaMax, e);
            const uint64_t ok = live & (pos_ok | __ballot(!(q > h1.y))) & __ballot(alpha >= kAlphaMin);
            if (ok == 0) {
                used &= ~(1ull << i);
                continue;
            }
            const bool okb = __builtin_amdgcn_inverse_ballot_w64(ok);
            const bool unclamped = __builtin_amdgcn_inverse_ballot_w64(ok & __ballot(e <= kAlphaMax));
            const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
            const float Ti = Tc * inv;  // transmittance in front of this splat
            float gc = __builtin_fmaf(g2, h2.x, __builtin_fmaf(g1, h1.w, g0 * h1.z));
            float2 h4 = make_float2(0.f, 0.f);
            if (FLOW) {
                h4 = s4[i];
                gc = __builtin_fmaf(g4, h4.y, __builtin_fmaf(g3, h4.x, gc));
            }
            const float wgt = okb ? alpha * Ti : 0.0f;
            const float da = __builtin_fmaf(-inv, GS, Ti * gc);
            GS = __builtin_fmaf(gc, wgt, GS);
            Tc = okb ? Ti : Tc;
            // d/d(power); zero where alpha is clamped (alpha = amax exp(power) otherwise)
            const float dp = unclamped ? da * alpha : 0.0f;
            const float dpx = dp * dx, dpy = dp * dy;
            const float v[9] = {dp, dpx, dpy, dpx * dx, dpx * dy, dpy * dy, g0 * wgt, g1 * wgt, g2 * wgt};
            float x, y;
            wave_sum9(v, x, y);
            float* rw = &red[(w * kWave + i) * NR];
            if (ln < 9) rw[ln < 8 ? red_index(ln) : 8] = ln < 8 ? x : y;
            if (FLOW) {
                const float f0 = wave_allsum(g3 * wgt), f1 = wave_allsum(g4 * wgt);
                if (ln == 0) {
                    rw[9] = f0;
                    rw[10] = f1;
                }
            }
        }
        if (ln == 0) kmask[w] = used;
        __syncthreads();
        // one thread per staged splat: add the quadrants' sums (fixed order), turn the
        // moments into the gradients of the 2D mean (d power / d m = Q d), the conic
        // (-d d^T / 2, off-diagonal -dx dy) and amax (alpha / amax where unclamped)
        if (tid < (int)nb) {
            const uint32_t sl = sslot[tid];
            float m[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) m[k] = 0.0f;
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!((kmask[q] >> tid) & 1ull)) continue;
                any = true;
                const float *rq = &red[(q * kWave + tid) * NR];
#pragma unroll
                for (int k = 0; k < NR; ++k) m[k] += rq[k];
            }
            if (sl < capacity) {  // false only after an instance overflow
                if (!any) {
                    zero_slot(ig, sl);  // no pixel of the tile blends it
                } else {
                    const float4 h3 = s3[tid];
                    const float P0 = m[0], Sx = m[1], Sy = m[2], Sxx = m[3], Sxy = m[4], Syy = m[5];
                    ig[3 * (size_t)sl + 0] =
                        make_float4(h3.x * Sx + h3.y * Sy, h3.z * Sy + h3.y * Sx, -0.5f * Sxx, -Sxy);
                    ig[3 * (size_t)sl + 1] = make_float4(-0.5f * Syy, P0 / h3.w, m[6], m[7]);
                    ig[3 * (size_t)sl + 2] = make_float4(m[8], FLOW ? m[9] : 0.f, FLOW ? m[10] : 0.f, 0.f);
                }
            }
        }
        __syncthreads();
        jb = j0;
    }
}

// d Y_k / d(x, y, z) of the polynomial basis used in the forward (any extension of
// Y_k off the unit sphere works: the radial part is projected out afterwards).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float Y[16], float dY[16][3]) {
    const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f;
    const float C2a = 1.0925484305920792f, C2b = 0.31539156525252005f, C2c = 0.5462742152960396f;
    const float C3a = -0.5900435899266435f, C3b = 2.890611442640554f, C3c = -0.4570457994644658f;
    const float C3d = 0.3731763325901154f, C3e = 1.445305721320277f;
    Y[0] = C0;
    dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
    if (DEG >= 1) {
        Y[1] = -C1 * y; dY[1][0] = 0.f; dY[1][1] = -C1; dY[1][2] = 0.f;
        Y[2] = C1 * z;  dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = C1;
        Y[3] = -C1 * x; dY[3][0] = -C1; dY[3][1] = 0.f; dY[3][2] = 0.f;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = C2a * (x * y);       dY[4][0] = C2a * y;  dY[4][1] = C2a * x;  dY[4][2] = 0.f;
        Y[5] = -C2a * (y * z);      dY[5][0] = 0.f;      dY[5][1] = -C2a * z; dY[5][2] = -C2a * y;
        Y[6] = C2b * (3.f * zz - 1.f); dY[6][0] = 0.f;   dY[6][1] = 0.f;      dY[6][2] = 6.f * C2b * z;
        Y[7] = -C2a * (x * z);      dY[7][0] = -C2a * z; dY[7][1] = 0.f;      dY[7][2] = -C2a * x;
        Y[8] = C2c * (xx - yy);     dY[8][0] = 2.f * C2c * x; dY[8][1] = -2.f * C2c * y; dY[8][2] = 0.f;
        if (DEG >= 3) {
            Y[9] = C3a * y * (3.f * xx - yy);
            dY[9][0] = C3a * 6.f * x * y; dY[9][1] = C3a * (3.f * xx - 3.f * yy); dY[9][2] = 0.f;
            Y[10] = C3b * (x * y) * z;
            dY[10][0] = C3b * y * z; dY[10][1] = C3b * x * z; dY[10][2] = C3b * x * y;
            Y[11] = C3c * y * (5.f * zz - 1.f);
            dY[11][0] = 0.f; dY[11][1] = C3c * (5.f * zz - 1.f); dY[11][2] = C3c * 10.f * y * z;
            Y[12] = C3d * z * (5.f * zz - 3.f);
            dY[12][0] = 0.f; dY[12][1] = 0.f; dY[12][2] = C3d * (15.f * zz - 3.f);
            Y[13] = C3c * x * (5.f * zz - 1.f);
            dY[13][0] = C3c * (5.f * zz - 1.f); dY[13][1] = 0.f; dY[13][2] = C3c * 10.f * x * z;
            Y[14] = C3e * z * (xx - yy);
            dY[14][0] = 2.f * C3e * x * z; dY[14][1] = -2.f * C3e * y * z; dY[14][2] = C3e * (xx - yy);
            Y[15] = C3a * x * (xx - 3.f * yy);
            dY[15][0] = C3a * (3.f * xx - 3.f * yy); dY[15][1] = -6.f * C3a * x * y; dY[15][2] = 0.f;
        }
    }
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_bwd(SceneK s, CamK c, float t, const float4 *__restrict__ rec,
                                                        const uint32_t *__restrict__ count,
                                                        const uint32_t *__restrict__ offset,
                                                        const float4 *__restrict__ ig, uint32_t capacity,
                                                        d4dgs_grads out, int motion) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int n = s.n;
    // the block's drawn Gaussians (count > 0), compacted in LDS so that the busy
    // wavefronts are full: about half of the Gaussians are culled at any t
    __shared__ uint32_t list[kBlock];
    __shared__ uint32_t wcnt[kBlock / kWave];
    {
        const int g0 = blockIdx.x * kBlock + threadIdx.x;
        const bool drawn = g0 < n && count[g0] > 0;
        const uint64_t bal = __ballot(drawn);
        const uint32_t rank = __popcll(bal & lanemask_lt());
        if (lane_id() == 0) wcnt[threadIdx.x / kWave] = __popcll(bal);
        __syncthreads();
        uint32_t base = 0;
        for (int i = 0; i < (int)threadIdx.x / kWave; ++i) base += wcnt[i];
        if (drawn) list[base + rank] = (uint32_t)g0;
        __syncthreads();
    }
    const uint32_t ndrawn = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (threadIdx.x >= ndrawn) return;
    const int gi = (int)list[threadIdx.x];
    const uint32_t cnt = count[gi];
    if ((uint64_t)offset[gi] + cnt > capacity) return;  // instances lost to an overflow
    // 1. sum this Gaussian's instance gradients in emission order
    float gmx = 0.f, gmy = 0.f, gA = 0.f, gB = 0.f, gC = 0.f, gam = 0.f, gr = 0.f, gg = 0.f, gb = 0.f;
    float gfx = 0.f, gfy = 0.f;  // dL/dmdot from the flow (zero when no flow was rendered)
    const uint32_t o0 = offset[gi];
    // the scene parameters are loaded first, so that their latency overlaps the slot sum
    const float q0 = s.quat[gi], q1 = s.quat[n + gi], q2 = s.quat[2 * n + gi], q3 = s.quat[3 * n + gi];
    const float sc[3] = {s.scale[gi], s.scale[n + gi], s.scale[2 * n + gi]};
    const float mu[3] = {s.mean[gi], s.mean[n + gi], s.mean[2 * n + gi]};
    const float v[3] = {s.velocity[gi], s.velocity[n + gi], s.velocity[2 * n + gi]};
    const float op = s.opacity[gi], mut = s.t_mean[gi], st = s.t_scale[gi];
    const float4 r0 = rec[3 * (size_t)gi], r1 = rec[3 * (size_t)gi + 1];
#pragma unroll 4
    for (uint32_t k = 0; k < cnt; ++k) {
        const size_t sl = 3 * (size_t)(o0 + k);
        const float4 a = ig[sl], b4 = ig[sl + 1], c4 = ig[sl + 2];
        gmx += a.x; gmy += a.y; gA += a.z; gB += a.w;
        gC += b4.x; gam += b4.y; gr += b4.z; gg += b4.w;
        gb += c4.x;
        gfx += c4.y;
        gfy += c4.z;
    }
    // 2. recompute the forward quantities (camera stage + time stage)
    const float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    const float nrm = sqrtf(n2);
    const float qw = q0 / nrm, qx = q1 / nrm, qy = q2 / nrm, qz = q3 / nrm;
    float Rq[9];
    Rq[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
    Rq[1] = 2.0f * (qx * qy - qw * qz);
    Rq[2] = 2.0f * (qx * qz + qw * qy);
    Rq[3] = 2.0f * (qx * qy + qw * qz);
    Rq[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
    Rq[5] = 2.0f * (qy * qz - qw * qx);
    Rq[6] = 2.0f * (qx * qz - qw * qy);
    Rq[7] = 2.0f * (qy * qz + qw * qx);
    Rq[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
    const float *R = c.R;
    float p[3], u[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = R[3 * i + 0] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + c.T[i];
        u[i] = R[3 * i + 0] * v[0] + R[3 * i + 1] * v[1] + R[3 * i + 2] * v[2];
    }
    const float tau = t - mut;
    const float w = expf(-0.5f * ((tau * tau) / (st * st)));
    const float pt[3] = {p[0] + tau * u[0], p[1] + tau * u[1], p[2] + tau * u[2]};
    const float md[2] = {(c.fx * u[0]) / p[2], (c.fy * u[1]) / p[2]};
    // the point the Jacobian is taken at: the moved mean, or the camera stage's mean
    const bool frozen = motion == D4DGS_MOTION_FROZEN_J, exact = motion == D4DGS_MOTION_EXACT;
    const float *pj = frozen ? p : pt;
    const float z = pj[2];
    float rx = pj[0] / z, ry = pj[1] / z;
    const bool clx = rx > c.limx || rx < -c.limx, cly = ry > c.limy || ry < -c.limy;
    rx = fminf(c.limx, fmaxf(-c.limx, rx));
    ry = fminf(c.limy, fmaxf(-c.limy, ry));
    const float tx = rx * z, ty = ry * z;
    const float J00 = c.fx / z, J11 = c.fy / z;
    const float J02 = -(c.fx * tx) / (z * z), J12 = -(c.fy * ty) / (z * z);
    // conic (A, B, C) of the record
    const float QA = r0.z, QB = r0.w, QC = r1.x;

    // 3. chain rule, time stage
    float g_o = w * gam;
    const float g_w = op * gam;
    float g_tau = g_w * (-w * tau / (st * st));
    float g_st = g_w * (w * tau * tau / (st * st * st));
    // covariance.  The forward's 2D covariance is Sigma' = J V J^T + dilation with
    // V = sum_j s_j^2 w_j w_j^T, w_j = R Rq e_j (axis j of the Gaussian in the camera
    // frame), i.e. Sigma' - dilation = sum_j s_j^2 a_j a_j^T with a_j = J w_j, and the
    // conic is Q = Sigma'^-1, so dQ = -Q dSigma' Q.  With G_Q = dL/dQ (symmetric, off
    // diagonal gB / 2), n_j = Q a_j and c_j = -Q G_Q n_j:
    //   dL/ds_j = -2 s_j n_j . (G_Q n_j),   dL/da_j = 2 s_j^2 c_j,
    // and a_j = J w_j passes that on to J (dL/dJ = sum_j 2 s_j^2 c_j w_j^T) and to w_j
    // (2 s_j^2 J^T c_j), hence to Rq (R^T of it).  Contracting with n_j before any 2x2 or
    // 3x3 gradient matrix is formed keeps elongated splats accurate: their conic is
    // nearly singular, Q a_j is small along the long axis, and forming -Q G_Q Q first
    // would cancel down to that size in FP32.
    const float h = 0.5f * gB;
    float gJ[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float g_s[3], gRq[9];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float wj[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) wj[i] = R[3 * i + 0] * Rq[j] + R[3 * i + 1] * Rq[3 + j] + R[3 * i + 2] * Rq[6 + j];
        const float ax = J00 * wj[0] + J02 * wj[2], ay = J11 * wj[1] + J12 * wj[2];
        const float nx = QA * ax + QB * ay, ny = QB * ax + QC * ay;
        const float mx = gA * nx + h * ny, my = h * nx + gC * ny;
        g_s[j] = -2.f * sc[j] * (nx * mx + ny * my);
        const float cx = -(QA * mx + QB * my), cy = -(QB * mx + QC * my);
        const float s2 = 2.f * sc[j] * sc[j];
        gJ[0][0] += s2 * cx * wj[0];
        gJ[0][2] += s2 * cx * wj[2];
        gJ[1][1] += s2 * cy * wj[1];
        gJ[1][2] += s2 * cy * wj[2];
        const float gw[3] = {s2 * (J00 * cx), s2 * (J11 * cy), s2 * (J02 * cx + J12 * cy)};
#pragma unroll
        for (int k = 0; k < 3; ++k) gRq[3 * k + j] = R[k] * gw[0] + R[3 + k] * gw[1] + R[6 + k] * gw[2];
    }
    const float z2 = z * z, z3 = z2 * z;
    float g_pj[3] = {0.f, 0.f, 0.f};  // through the Jacobian's point
    g_pj[2] += gJ[0][0] * (-c.fx / z2) + gJ[0][2] * (2.f * c.fx * tx / z3) + gJ[1][1] * (-c.fy / z2) +
               gJ[1][2] * (2.f * c.fy * ty / z3);
    const float g_tx = gJ[0][2] * (-c.fx / z2), g_ty = gJ[1][2] * (-c.fy / z2);
    if (clx) g_pj[2] += g_tx * rx; else g_pj[0] += g_tx;
    if (cly) g_pj[2] += g_ty * ry; else g_pj[1] += g_ty;
    float g_pt[3], g_p[3], g_u[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3; ++i) {
        g_pt[i] = frozen ? 0.f : g_pj[i];
        g_p[i] = frozen ? g_pj[i] : 0.f;
    }
    const float ipz = 1.f / p[2];
    if (exact) {
        // m = f pt_xy / pt_z + c; the flow velocity vel = f (u_xy pt_z - pt_xy u_z) / pt_z^2
        const float zt = pt[2], izt = 1.f / zt, izt2 = izt * izt;
        g_pt[0] += c.fx * gmx * izt - c.fx * u[2] * gfx * izt2;
        g_pt[1] += c.fy * gmy * izt - c.fy * u[2] * gfy * izt2;
        g_pt[2] += -(c.fx * pt[0] * gmx + c.fy * pt[1] * gmy) * izt2 +
                   (c.fx * (2.f * pt[0] * u[2] - u[0] * zt) * gfx + c.fy * (2.f * pt[1] * u[2] - u[1] * zt) * gfy) *
                       izt2 * izt;
        g_u[0] += c.fx * gfx * izt;
        g_u[1] += c.fy * gfy * izt;
        g_u[2] += -(c.fx * pt[0] * gfx + c.fy * pt[1] * gfy) * izt2;
    } else {
        // m = m0 + tau md; the flow velocity is md.  Camera stage: m0 = f p_xy / p_z + c,
        // md = f u_xy / p_z
        g_tau += md[0] * gmx + md[1] * gmy;
        const float g_mdx = tau * gmx + gfx, g_mdy = tau * gmy + gfy;
        g_p[0] += c.fx * gmx * ipz;
        g_p[1] += c.fy * gmy * ipz;
        g_p[2] += -(c.fx * p[0] * gmx + c.fy * p[1] * gmy) * ipz * ipz;
        g_u[0] += c.fx * g_mdx * ipz;
        g_u[1] += c.fy * g_mdy * ipz;
        g_p[2] += -(c.fx * u[0] * g_mdx + c.fy * u[1] * g_mdy) * ipz * ipz;
    }
    // p_t = p + tau u
    for (int i = 0; i < 3; ++i) {
        g_p[i] += g_pt[i];
        g_u[i] += tau * g_pt[i];
    }
    g_tau += u[0] * g_pt[0] + u[1] * g_pt[1] + u[2] * g_pt[2];
    // p = R mu + T, u = R v
    float g_mu[3], g_v[3];
    for (int j = 0; j < 3; ++j) {
        g_mu[j] = R[j] * g_p[0] + R[3 + j] * g_p[1] + R[6 + j] * g_p[2];
        g_v[j] = R[j] * g_u[0] + R[3 + j] * g_u[1] + R[6 + j] * g_u[2];
    }
    // rotation matrix of the unit quaternion (w, x, y, z)
    float gqw = 2.f * (-qz * gRq[1] + qy * gRq[2] + qz * gRq[3] - qx * gRq[5] - qy * gRq[6] + qx * gRq[7]);
    float gqx = 2.f * (qy * gRq[1] + qz * gRq[2] + qy * gRq[3] - 2.f * qx * gRq[4] - qw * gRq[5] + qz * gRq[6] +
                       qw * gRq[7] - 2.f * qx * gRq[8]);
    float gqy = 2.f * (-2.f * qy * gRq[0] + qx * gRq[1] + qw * gRq[2] + qx * gRq[3] + qz * gRq[5] - qw * gRq[6] +
                       qz * gRq[7] - 2.f * qy * gRq[8]);
    float gqz = 2.f * (-2.f * qz * gRq[0] - qw * gRq[1] + qx * gRq[2] + qw * gRq[3] - 2.f * qz * gRq[4] +
                       qy * gRq[5] + qx * gRq[6] + qy * gRq[7]);
    const float dotq = qw * gqw + qx * gqx + qy * gqy + qz * gqz;
    const float g_q[4] = {(gqw - qw * dotq) / nrm, (gqx - qx * dotq) / nrm, (gqy - qy * dotq) / nrm,
                          (gqz - qz * dotq) / nrm};
    // colour: rgb = max(0, sum_k Y_k(d) sh_k + 0.5), d = (mu - campos) / |mu - campos|.
    // The gradient arrays are only written here and never alias the scene, so each group
    // of old values is loaded together before the stores (no serialised round trips).
    const float *__restrict__ shp = s.sh;
    float *__restrict__ osh = out.sh;
    {
        const float dx0 = mu[0] - c.campos[0], dy0 = mu[1] - c.campos[1], dz0 = mu[2] - c.campos[2];
        const float len = sqrtf(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
        const float d[3] = {dx0 / len, dy0 / len, dz0 / len};
        float Y[16], dY[16][3];
        sh_basis_grad<DEG>(d[0], d[1], d[2], Y, dY);
        const float grgb[3] = {gr, gg, gb};
        float g_d[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float shv[K], old[K];
#pragma unroll
            for (int k = 0; k < K; ++k) shv[k] = shp[(size_t)(k * 3 + ch) * n + gi];
            float raw = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) raw += Y[k] * shv[k];
            if (raw < 0.f) continue;  // clamped at 0: no gradient
#pragma unroll
            for (int k = 0; k < K; ++k) old[k] = osh[(size_t)(k * 3 + ch) * n + gi];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                osh[(size_t)(k * 3 + ch) * n + gi] = old[k] + Y[k] * grgb[ch];
                const float f = shv[k] * grgb[ch];
                g_d[0] += f * dY[k][0];
                g_d[1] += f * dY[k][1];
                g_d[2] += f * dY[k][2];
            }
        }
        const float dd = d[0] * g_d[0] + d[1] * g_d[1] + d[2] * g_d[2];
        for (int i = 0; i < 3; ++i) g_mu[i] += (g_d[i] - d[i] * dd) / len;
    }
    float *__restrict__ omean = out.mean;
    float *__restrict__ oscale = out.scale;
    float *__restrict__ ovel = out.velocity;
    float *__restrict__ oquat = out.quat;
    float *__restrict__ oop = out.opacity;
    float *__restrict__ omut = out.t_mean;
    float *__restrict__ ost = out.t_scale;
    float om[3], os[3], ov[3], oq[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        om[i] = omean[i * n + gi];
        os[i] = oscale[i * n + gi];
        ov[i] = ovel[i * n + gi];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) oq[i] = oquat[i * n + gi];
    const float oo = oop[gi], ot = omut[gi], o_s = ost[gi];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        omean[i * n + gi] = om[i] + g_mu[i];
        oscale[i * n + gi] = os[i] + g_s[i];
        ovel[i * n + gi] = ov[i] + g_v[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) oquat[i * n + gi] = oq[i] + g_q[i];
    oop[gi] = oo + g_o;
    omut[gi] = ot - g_tau;
    ost[gi] = o_s + g_st;
    // splitting statistics of this view: |dL/dmu_t| and |dL/dmu|
    if (out.split_count) {
        float *__restrict__ sgt = out.split_grad_t;
        float *__restrict__ sgx = out.split_grad_xyz;
        uint32_t *__restrict__ scn = out.split_count;
        const float a = sgt[gi], bx = sgx[gi];
        const uint32_t cn = scn[gi];
        sgt[gi] = a + fabsf(g_tau);
        sgx[gi] = bx + sqrtf(g_mu[0] * g_mu[0] + g_mu[1] * g_mu[1] + g_mu[2] * g_mu[2]);
        scn[gi] = cn + 1u;
    }
    (void)g_o;
}

}  // namespace

// With events e0/e1 each launch goes through hipExtLaunchKernel, which sets them to the
// kernel's own start and end (for measurement); without work they are recorded together.
hipError_t launch_blend_bwd(const float4 *rec, const uint32_t *offset, const uint32_t *vals, const uint32_t *ranges,
                            const uint32_t *order, const CamK &c, const float bg[3], const float *final_T, const uint32_t *n_contrib,
                            const float *dL_dimg, const float2 *mdot, const float *dL_dflow, float4 *inst_grads,
                            int64_t capacity, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const int ntiles = c.TX * c.TY;
    if (ntiles == 0) {
        if (e0 && hipEventRecord(e0, st) == hipSuccess) (void)hipEventRecord(e1, st);
        return hipGetLastError();
    }
    const dim3 grid(tile_grid(c.TX, c.TY, 1)), block(kBwdThreads);
    const uint32_t cap = (uint32_t)capacity;
    if (mdot && dL_dflow) {
        if (e0)
            hipExtLaunchKernelGGL(k_blend_bwd<true>, grid, block, 0, st, e0, e1, 0, rec, offset, vals, ranges, order, c,
                                  bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimg, inst_grads, cap, mdot, dL_dflow);
        else
            hipLaunchKernelGGL(k_blend_bwd<true>, grid, block, 0, st, rec, offset, vals, ranges, order, c, bg[0], bg[1],
                               bg[2], final_T, n_contrib, dL_dimg, inst_grads, cap, mdot, dL_dflow);
    } else {
        const float2 *no_mdot = nullptr;
        const float *no_dflow = nullptr;
        if (e0)
            hipExtLaunchKernelGGL(k_blend_bwd<false>, grid, block, 0, st, e0, e1, 0, rec, offset, vals, ranges, order, c,
                                  bg[0], bg[1], bg[2], final_T, n_contrib, dL_dimg, inst_grads, cap, no_mdot, no_dflow);
        else
            hipLaunchKernelGGL(k_blend_bwd<false>, grid, block, 0, st, rec, offset, vals, ranges, order, c, bg[0], bg[1],
                               bg[2], final_T, n_contrib, dL_dimg, inst_grads, cap, no_mdot, no_dflow);
    }
    return hipGetLastError();
}

namespace {

template <int DEG>
void launch_project_bwd_deg(const SceneK &s, const CamK &c, float t, const float4 *rec, const uint32_t *count,
                            const uint32_t *offset, const float4 *inst_grads, uint32_t cap, const d4dgs_grads &g,
                            int motion, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid((s.n + kBlock - 1) / kBlock), block(kBlock);
    if (e0)
        hipExtLaunchKernelGGL(k_project_bwd<DEG>, grid, block, 0, st, e0, e1, 0, s, c, t, rec, count, offset,
                              inst_grads, cap, g, motion);
    else
        hipLaunchKernelGGL(k_project_bwd<DEG>, grid, block, 0, st, s, c, t, rec, count, offset, inst_grads, cap, g,
                           motion);
}

}  // namespace

hipError_t launch_project_bwd(const SceneK &s, const CamK &c, float t, const float4 *rec, const uint32_t *count,
                              const uint32_t *offset, const float4 *inst_grads, int64_t capacity,
                              const d4dgs_grads &g, int motion, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    if (s.n == 0) {
        if (e0 && hipEventRecord(e0, st) == hipSuccess) (void)hipEventRecord(e1, st);
        return hipGetLastError();
    }
    const uint32_t cap = (uint32_t)capacity;
    switch (s.deg) {
        case 0: launch_project_bwd_deg<0>(s, c, t, rec, count, offset, inst_grads, cap, g, motion, st, e0, e1); break;
        case 1: launch_project_bwd_deg<1>(s, c, t, rec, count, offset, inst_grads, cap, g, motion, st, e0, e1); break;
        case 2: launch_project_bwd_deg<2>(s, c, t, rec, count, offset, inst_grads, cap, g, motion, st, e0, e1); break;
        default: launch_project_bwd_deg<3>(s, c, t, rec, count, offset, inst_grads, cap, g, motion, st, e0, e1); break;
    }
    return hipGetLastError();
}

}  // namespace d4
