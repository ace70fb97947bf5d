// Enumeration of the (tile, splat) instances of one block of 256 Gaussians, shared by
// the binning's count pass (a kernel of its own, or fused into the projection) and its
// scatter pass (tile binning of the rasteriser the paper renders with, Sec. 3.2.2).
//
// Device-scope atomics are expensive on this part, so the count pass aggregates them:
// when the block's splats together cover at most kCells tiles (a spatially coherent
// block, as when the scene is stored along a space-filling curve -- the synthetic scenes
// are in 3D Morton order), its instances are counted per tile in LDS and one atomic per
// (block, tile) on the tile's grouped counter reserves the group's range, kept in
// grp_off[block][cell]; otherwise every instance adds one to the tile's ungrouped
// counter.  After the tile scan a tile's list is laid out as [grouped instances |
// ungrouped instances]; the scatter pass recomputes the same enumeration and places a
// grouped instance at start + grp_off + its rank inside the group (an LDS atomic), an
// ungrouped one at an atomic cursor that starts after the grouped ones (any unique
// position will do: the per-tile sort fixes the final order).
#pragma once

#include "internal.hpp"

namespace d4 {

constexpr int kCells = 2048;

// LDS of one block's enumeration
struct EmitLds {
    uint32_t incl[kBlock];  // wave-inclusive prefix of the per-Gaussian counts
    uint32_t x0[kBlock], y0[kBlock], w[kBlock];
    uint32_t cell[kCells];  // per-tile counts (count pass) or ranks (scatter pass)
    uint32_t box[4][kBlock / kWave];
    uint32_t mark[kBlock];  // emit_each: 1 + the lane whose instances start at a position
};

// The block's union rectangle of tiles (origin bx0, by0; uw x uh tiles) and whether its
// instances are grouped (uw * uh <= kCells).
struct EmitBox {
    uint32_t bx0, by0, uw, uh;
    bool grouped;
};

// Rectangle bits of a splat record (x0 | y0 << 16, x1 | y1 << 16; tiles, half open).
__device__ __forceinline__ void rect_of(uint32_t lo, uint32_t hi, uint32_t &x0, uint32_t &y0, uint32_t &x1,
                                        uint32_t &y1) {
    x0 = lo & 0xffffu;
    y0 = lo >> 16;
    x1 = hi & 0xffffu;
    y1 = hi >> 16;
}

// Stages this thread's count and rectangle (lo, hi: its record's rectangle bits, read
// only when cnt > 0) and returns the block's union rectangle, with the grouped cells
// cleared.  block_sum (optional) receives the block's count sum, from the wave prefixes.
// Contains block-wide barriers: every thread of the block calls it.
__device__ __forceinline__ EmitBox emit_box(EmitLds &L, uint32_t cnt, uint32_t lo, uint32_t hi,
                                            uint32_t *block_sum = nullptr) {
    const int tid = threadIdx.x, wv = tid / kWave;
    L.incl[tid] = wave_incl_scan(cnt);
    uint32_t bx0 = 0xffffu, by0 = 0xffffu, bx1 = 0u, by1 = 0u;
    if (cnt) {
        rect_of(lo, hi, bx0, by0, bx1, by1);
        L.x0[tid] = bx0;
        L.y0[tid] = by0;
        L.w[tid] = bx1 - bx0;
    }
    bx0 = wave_min_u32_uniform(bx0);
    by0 = wave_min_u32_uniform(by0);
    bx1 = wave_max_u32_uniform(bx1);
    by1 = wave_max_u32_uniform(by1);
    if (lane_id() == 0) {
        L.box[0][wv] = bx0;
        L.box[1][wv] = by0;
        L.box[2][wv] = bx1;
        L.box[3][wv] = by1;
    }
    __syncthreads();
    if (block_sum && tid == 0) {
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i) sum += L.incl[i * kWave + kWave - 1];
        *block_sum = sum;
    }
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        bx0 = min(bx0, L.box[0][i]);
        by0 = min(by0, L.box[1][i]);
        bx1 = max(bx1, L.box[2][i]);
        by1 = max(by1, L.box[3][i]);
    }
    EmitBox B;
    B.bx0 = bx0;
    B.by0 = by0;
    B.uw = bx1 > bx0 ? bx1 - bx0 : 0u;
    B.uh = by1 > by0 ? by1 - by0 : 0u;
    B.grouped = B.uw * B.uh <= (uint32_t)kCells;
    if (B.grouped)
        for (uint32_t c = tid; c < B.uw * B.uh; c += kBlock) L.cell[c] = 0u;
    __syncthreads();
    return B;
}

// Visits every instance of the block once: f(o, tile, cell) with o the owning thread of
// the block.  A wave's instances are dealt to its lanes in rounds of 64 (lane l takes
// instance r0 + l of the wave's 64 Gaussians' instances, in order), so splats with large
// rectangles do not stall a wave.  An instance's owner is the last Gaussian (lane) whose
// instances start at or before it: each Gaussian whose first instance falls in the round
// marks that position with 1 + its lane, and an inclusive max-scan over the round's
// positions, floored by the owner of the previous round's last instance, gives every
// instance its owner.
template <class F>
__device__ __forceinline__ void emit_each(EmitLds &L, const EmitBox &B, int TX, F f) {
    const int wbase = (threadIdx.x / kWave) * kWave, ln = lane_id();
    const uint32_t wtotal = L.incl[wbase + kWave - 1];
    const uint32_t first = ln > 0 ? L.incl[wbase + ln - 1] : 0u;  // this lane's first instance
    const bool has = L.incl[wbase + ln] > first;
    uint32_t carry = 0u;  // 1 + the owner of the instance before the round (0: none yet)
    for (uint32_t r0 = 0; r0 < wtotal; r0 += kWave) {
        L.mark[wbase + ln] = 0u;
        wave_lds_sync();
        if (has && first >= r0 && first - r0 < (uint32_t)kWave) L.mark[wbase + (first - r0)] = (uint32_t)ln + 1u;
        wave_lds_sync();
        const uint32_t own = max(wave_incl_max(L.mark[wbase + ln]), carry);
        carry = __builtin_amdgcn_readlane(own, kWave - 1);
        const uint32_t j = r0 + ln;
        if (j < wtotal) {
            const int lo = (int)own - 1;
            const int o = wbase + lo;
            const uint32_t kk = j - (lo > 0 ? L.incl[o - 1] : 0u);
            const uint32_t w = L.w[o];
            const uint32_t tyy = L.y0[o] + kk / w, txx = L.x0[o] + kk % w;
            f(o, tyy * (uint32_t)TX + txx, (tyy - B.by0) * B.uw + (txx - B.bx0));
        }
        wave_lds_sync();  // every lane has read its mark before the next round clears them
    }
}

// The count pass of one block (block index blk): grouped, per-tile counts in LDS and one
// reservation per (block, tile) on cnt_g, its offset kept in grp_off[blk][cell];
// otherwise one increment of cnt_n per instance.  block_sum (optional) receives the
// block's count sum.  Block-wide barriers.
__device__ __forceinline__ void emit_count(EmitLds &L, uint32_t cnt, uint32_t lo, uint32_t hi, int TX, int blk,
                                           uint32_t *__restrict__ cnt_g, uint32_t *__restrict__ cnt_n,
                                           uint32_t *__restrict__ grp_off, uint32_t *block_sum = nullptr) {
    const EmitBox B = emit_box(L, cnt, lo, hi, block_sum);
    if (B.grouped) {
        emit_each(L, B, TX, [&](int, uint32_t, uint32_t cell) { atomicAdd(&L.cell[cell], 1u); });
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < B.uw * B.uh; c += kBlock) {
            const uint32_t k = L.cell[c];
            if (k) {
                const uint32_t tile = (B.by0 + c / B.uw) * (uint32_t)TX + (B.bx0 + c % B.uw);
                grp_off[(size_t)blk * kCells + c] = atomicAdd(&cnt_g[tile], k);
            }
        }
    } else {
        emit_each(L, B, TX, [&](int, uint32_t tile, uint32_t) { atomicAdd(&cnt_n[tile], 1u); });
    }
}

}  // namespace d4
