// Tile binning and depth-keyed sort (the tiled rasteriser of 3D Gaussian Splatting
// that the paper renders with, Sec. 3.2.2), designed for MI355X:
//
//   k_scan_partials  one block: exclusive scan of the per-block count sums written by
//                    the projection into block offsets; instance total; capacity check;
//                    clears the tile counters.
//   k_count          count pass per block of 256 Gaussians (emit.hpp): grouped
//                    reservations per (block, tile), or ungrouped increments.  The
//                    projection can do this pass itself (launch_bin_counted then follows).
//   k_tile_scan      one block: exclusive scan over tiles -> ranges and the ungrouped
//                    cursors; leaves the counters zero.  k_scan_both: both scans in one
//                    block, after a projection that counted.
//   k_scatter        per block: per-Gaussian offsets (block offset + block scan), then
//                    every instance's 64-bit sort key (float-bits(depth) << 32) | gaussian
//                    at its position in the tile's bucket.  (With a tile order, one more
//                    workgroup sorts the tiles by list length for the launches that
//                    follow.)
//   k_tile_sort      one wavefront per tile sorts its bucket by the 64-bit key -- depth,
//                    ties by Gaussian index: a unique order, so the result does not depend
//                    on the order the atomics handed out positions.  Up to 64 keys by
//                    ranking (the keys are unique, so a key's sorted position is the number
//                    of smaller keys, counted by each lane while the wavefront streams the
//                    list from LDS); up to 512 keys by ranking inside chunks of 64 and
//                    merging the chunks by binary search; longer lists by a stable
//                    least-significant-digit radix sort over the 64 key bits, 8-bit digits,
//                    ping-ponging between two global scratch arrays.  A workgroup of one
//                    wavefront per tile: most lists are short, and wavefronts that a
//                    larger workgroup would leave idle on them still hold compute-unit
//                    slots while their tile's range loads (measured: 4 wavefronts per
//                    tile, 24.9 k sweep frames/s; one, 26.5 k).  Writes
//                    keys = (tile << 32) | float-bits(depth) and values = gaussian.
//
// The instance total lives on the device; no host synchronisation is needed.  If it
// exceeds the capacity, a status word is set and every later stage does nothing.
#include "emit.hpp"

namespace d4 {

namespace {

constexpr int kScanThreads = 1024;
constexpr uint32_t kNoOffset = 0xffffffffu;  // offset of every Gaussian after a failed binning

__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *tmp4) {
    const int w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) tmp4[w] = inc;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) base += (i < w) ? tmp4[i] : 0u;
    __syncthreads();
    return base + inc - v;
}

// Scan of the per-block count sums written by the projection into block offsets (in
// place); instance total and capacity check.  misc[0] = instance total (0 on overflow),
// misc[1] = status (0 or CAPACITY).  Returns whether the total exceeds the capacity;
// *total_out receives the total (every thread).
__device__ __forceinline__ bool scan_block_sums(uint32_t *__restrict__ partial, int nb, int64_t capacity,
                                                int64_t *__restrict__ num_inst, uint32_t *__restrict__ misc,
                                                int32_t *__restrict__ d_status, uint64_t *wsum,
                                                uint64_t *total_out) {
    const int tid = threadIdx.x;
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    // up to kSumsPerThread sums per thread stay in registers between the two passes (all
    // loads in flight together); more are read again
    constexpr int kSumsPerThread = 8;
    const bool held = per <= kSumsPerThread;
    uint32_t v[kSumsPerThread];
    uint64_t s = 0;
    if (held) {
#pragma unroll
        for (int j = 0; j < kSumsPerThread; ++j) v[j] = b0 + j < b1 ? partial[b0 + j] : 0u;
#pragma unroll
        for (int j = 0; j < kSumsPerThread; ++j) s += v[j];
    } else {
        for (int i = b0; i < b1; ++i) s += partial[i];
    }
    const uint64_t inc = wave_incl_scan64(s);
    if (lane_id() == kWave - 1) wsum[tid / kWave] = inc;
    __syncthreads();
    uint64_t base = 0, total = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        base += (i < tid / kWave) ? wsum[i] : 0ull;
        total += wsum[i];
    }
    uint64_t run = base + inc - s;
    if (held) {
#pragma unroll
        for (int j = 0; j < kSumsPerThread; ++j) {
            if (b0 + j < b1) partial[b0 + j] = (uint32_t)min(run, (uint64_t)0xffffffffull);
            run += v[j];
        }
    } else {
        for (int i = b0; i < b1; ++i) {
            const uint32_t x = partial[i];
            partial[i] = (uint32_t)min(run, (uint64_t)0xffffffffull);
            run += x;
        }
    }
    const bool over = total > (uint64_t)capacity;
    *total_out = total;
    if (tid == 0) {
        *num_inst = (int64_t)total;
        misc[0] = (uint32_t)(over ? 0ull : total);
        misc[1] = over ? (uint32_t)D4DGS_ERR_CAPACITY : 0u;
        if (d_status && over) *d_status = D4DGS_ERR_CAPACITY;
    }
    return over;
}

constexpr int kScanPer = 8;                       // tiles per thread in one round of the tile scan
constexpr int kScanWaves = kScanThreads / kWave;  // waves of the scan's workgroup

// LDS of the tile scan: per slice, the waves' totals; the waves' 64-bit count sums
struct TileScanLds {
    uint32_t part[kScanPer][kScanWaves];
    uint64_t tot[kScanWaves];
};

// One round of tiles r0 + k * kScanThreads + thread (k < kScanPer: each slice of
// kScanThreads consecutive tiles is read with coalesced loads, all issued together).
__device__ __forceinline__ void load_counts(const uint32_t *__restrict__ cnt_g, const uint32_t *__restrict__ cnt_n,
                                            int tiles, int r0, uint32_t (&g)[kScanPer], uint32_t (&n)[kScanPer]) {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int i = r0 + k * kScanThreads + (int)threadIdx.x;
        g[k] = i < tiles ? cnt_g[i] : 0u;
        n[k] = i < tiles ? cnt_n[i] : 0u;
    }
}

// Wave-inclusive scans of the round's slices; the waves' slice totals go to LDS.
__device__ __forceinline__ void round_publish(const uint32_t (&c)[kScanPer], uint32_t (&inc)[kScanPer],
                                              TileScanLds &L) {
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        inc[k] = wave_incl_scan(c[k]);
        if (lane_id() == kWave - 1) L.part[k][w] = inc[k];
    }
}

// After the barrier that follows round_publish: writes the round's ranges and cursors
// (starting at carry; all empty if `empty`) and clears its counters; returns the
// round's total.
__device__ __forceinline__ uint32_t round_write(const uint32_t (&g)[kScanPer], const uint32_t (&c)[kScanPer],
                                                const uint32_t (&inc)[kScanPer], const TileScanLds &L,
                                                uint32_t carry, int r0, int tiles, bool empty,
                                                uint32_t *__restrict__ ranges, uint32_t *__restrict__ cur_n,
                                                uint32_t *__restrict__ cnt_g, uint32_t *__restrict__ cnt_n) {
    const int w = threadIdx.x / kWave;
    uint32_t running = carry;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        uint32_t row = 0, before = 0;
#pragma unroll
        for (int v = 0; v < kScanWaves; ++v) {
            const uint32_t x = L.part[k][v];
            row += x;
            before += v < w ? x : 0u;
        }
        const uint32_t start = empty ? 0u : running + before + inc[k] - c[k];
        const int i = r0 + k * kScanThreads + (int)threadIdx.x;
        if (i < tiles) {
            ranges[2 * i] = start;
            ranges[2 * i + 1] = empty ? 0u : start + c[k];
            cur_n[i] = start + g[k];
            cnt_g[i] = 0u;
            cnt_n[i] = 0u;
        }
        running += row;
    }
    return running - carry;
}

// Exclusive scan of the tile counts (grouped + ungrouped) into ranges and the ungrouped
// cursors (start + grouped count); the counters are left zero for the next frame.
// Ranges are empty on overflow, and also when the tile counts do not add up to the
// instance total `expect` (counters that were not zero when the count pass started: a
// workspace that was not initialised); then misc and *d_status report INVALID_ARG.
// Up to kScanThreads * kScanPer tiles (1352 x 1014 has 5,440) take one round: one batch
// of loads, one barrier.  Larger images add the counts up first (the check needs the
// total before any range is written), then scan round by round.
// pre (optional, one-round images only): the counts, already loaded by the caller.
__device__ __forceinline__ void scan_tiles(uint32_t *__restrict__ cnt_g, uint32_t *__restrict__ cnt_n,
                                           uint32_t *__restrict__ cur_n, int tiles, uint32_t *__restrict__ ranges,
                                           bool over, uint64_t expect, uint32_t *__restrict__ misc,
                                           int32_t *__restrict__ d_status, TileScanLds &L,
                                           const uint32_t (*pre_g)[kScanPer] = nullptr,
                                           const uint32_t (*pre_n)[kScanPer] = nullptr) {
    const int tid = threadIdx.x, w = tid / kWave;
    constexpr int RS = kScanThreads * kScanPer;
    uint32_t g[kScanPer], n[kScanPer], c[kScanPer], inc[kScanPer];
    uint64_t mine = 0;
    const bool one = tiles <= RS;
    if (one) {
        if (pre_g) {
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) {
                g[k] = (*pre_g)[k];
                n[k] = (*pre_n)[k];
            }
        } else {
            load_counts(cnt_g, cnt_n, tiles, 0, g, n);
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            mine += (uint64_t)g[k] + n[k];
            c[k] = g[k] + n[k];
        }
        round_publish(c, inc, L);
    } else {
        for (int r0 = 0; r0 < tiles; r0 += RS) {
            load_counts(cnt_g, cnt_n, tiles, r0, g, n);
#pragma unroll
            for (int k = 0; k < kScanPer; ++k) mine += (uint64_t)g[k] + n[k];
        }
    }
    mine = wave_sum_u64_uniform(mine);
    if (lane_id() == 0) L.tot[w] = mine;
    __syncthreads();
    uint64_t total = 0;
#pragma unroll
    for (int v = 0; v < kScanWaves; ++v) total += L.tot[v];
    const bool empty = over || total != expect;  // otherwise every prefix fits: total <= capacity < 2^31
    if (tid == 0 && empty && !over) {
        misc[0] = 0u;
        misc[1] = (uint32_t)D4DGS_ERR_INVALID_ARG;
        if (d_status) *d_status = D4DGS_ERR_INVALID_ARG;
    }
    if (one) {
        round_write(g, c, inc, L, 0u, 0, tiles, empty, ranges, cur_n, cnt_g, cnt_n);
        return;
    }
    uint32_t carry = 0;
    for (int r0 = 0; r0 < tiles; r0 += RS) {
        load_counts(cnt_g, cnt_n, tiles, r0, g, n);
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) c[k] = g[k] + n[k];
        round_publish(c, inc, L);
        __syncthreads();
        carry += round_write(g, c, inc, L, carry, r0, tiles, empty, ranges, cur_n, cnt_g, cnt_n);
        __syncthreads();  // the next round rewrites L.part
    }
}

// The two scans as separate kernels (binning after a plain projection): the first also
// clears the tile counters, so that a workspace needs no initialisation.
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t *__restrict__ partial, int nb,
                                                               int64_t capacity, int64_t *__restrict__ num_inst,
                                                               uint32_t *__restrict__ misc,
                                                               int32_t *__restrict__ d_status,
                                                               uint32_t *__restrict__ cnt_g,
                                                               uint32_t *__restrict__ cnt_n, int tiles) {
    __shared__ uint64_t wsum[kScanThreads / kWave];
    for (int i = threadIdx.x; i < tiles; i += kScanThreads) {
        cnt_g[i] = 0u;
        cnt_n[i] = 0u;
    }
    uint64_t total;
    scan_block_sums(partial, nb, capacity, num_inst, misc, d_status, wsum, &total);
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint32_t *__restrict__ cnt_g, uint32_t *__restrict__ cnt_n,
                                                           uint32_t *__restrict__ cur_n, int tiles,
                                                           uint32_t *__restrict__ ranges, uint32_t *__restrict__ misc,
                                                           int32_t *__restrict__ d_status) {
    __shared__ TileScanLds L;
    const bool over = misc[1] != 0u;
    const uint64_t expect = misc[0];
    __syncthreads();  // every thread has read misc before thread 0 may rewrite it
    scan_tiles(cnt_g, cnt_n, cur_n, tiles, ranges, over, expect, misc, d_status, L);
}

// Both scans in one workgroup, after the projection that counted the instances (its
// counters started at zero, as every scan leaves them).
__global__ __launch_bounds__(kScanThreads) void k_scan_both(uint32_t *__restrict__ partial, int nb, int64_t capacity,
                                                           int64_t *__restrict__ num_inst,
                                                           uint32_t *__restrict__ misc,
                                                           int32_t *__restrict__ d_status,
                                                           uint32_t *__restrict__ cnt_g,
                                                           uint32_t *__restrict__ cnt_n,
                                                           uint32_t *__restrict__ cur_n, int tiles,
                                                           uint32_t *__restrict__ ranges) {
    __shared__ uint64_t wsum64[kScanThreads / kWave];
    __shared__ TileScanLds L;
    // an image of one round: its tile counts are loaded first, so that their latency
    // overlaps the block sums' (the two scans only meet at the capacity check)
    uint32_t g[kScanPer], n[kScanPer];
    const bool one = tiles <= kScanThreads * kScanPer;
    if (one) load_counts(cnt_g, cnt_n, tiles, 0, g, n);
    uint64_t total;
    const bool over = scan_block_sums(partial, nb, capacity, num_inst, misc, d_status, wsum64, &total);
    if (one)
        scan_tiles(cnt_g, cnt_n, cur_n, tiles, ranges, over, total, misc, d_status, L, &g, &n);
    else
        scan_tiles(cnt_g, cnt_n, cur_n, tiles, ranges, over, total, misc, d_status, L);
}

// Tile order of the per-tile launches (see tile_unit): the tiles of row class x (rows
// x, x + 8, ...: the tiles XCD x takes) form the x-th segment of the order, and inside a
// segment the tiles are ordered by list length, longest first, in steps of 8 (lists of
// 2,040 or more share the first step).  Work on a tile (its sort, its blend, its
// adjoint) grows with its list, so each XCD starts with its long lists and they do not
// run alone at the end of a launch.  One extra workgroup of the scatter pass builds it
// (a counting sort in LDS), next to the scatter and off the frame's critical path.
constexpr int kOrderShift = 3;
constexpr int kOrderKeys = 8 * kRadix;  // row class x 256 length steps
__device__ __forceinline__ uint32_t order_key(int tile, int TX, uint32_t count) {
    return (uint32_t)((tile / TX) & 7) * kRadix + (255u - min(count >> kOrderShift, 255u));
}

// hist: kOrderKeys words of LDS; 256 threads
__device__ void build_tile_order(const uint32_t *__restrict__ ranges, int tiles, int TX, uint32_t *__restrict__ order,
                                 uint32_t *hist, uint32_t *tmp4) {
    constexpr int KPT = kOrderKeys / kBlock;  // keys per thread in the scan
    const int tid = threadIdx.x;
    for (int k = tid; k < kOrderKeys; k += kBlock) hist[k] = 0u;
    __syncthreads();
    for (int i0 = tid; i0 < tiles; i0 += 4 * kBlock) {
        uint2 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = i0 + u * kBlock < tiles ? make_uint2(ranges[2 * (i0 + u * kBlock)], ranges[2 * (i0 + u * kBlock) + 1])
                                              : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * kBlock < tiles) atomicAdd(&hist[order_key(i0 + u * kBlock, TX, r[u].y - r[u].x)], 1u);
    }
    __syncthreads();
    uint32_t v[KPT], sum = 0;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        v[j] = hist[KPT * tid + j];
        sum += v[j];
    }
    uint32_t base = block_excl_scan_256(sum, tmp4);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        hist[KPT * tid + j] = base;
        base += v[j];
    }
    __syncthreads();
    // the order inside a key is whatever the LDS atomics give: it only decides when a
    // tile is processed, never a result
    for (int i0 = tid; i0 < tiles; i0 += 4 * kBlock) {
        uint2 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = i0 + u * kBlock < tiles ? make_uint2(ranges[2 * (i0 + u * kBlock)], ranges[2 * (i0 + u * kBlock) + 1])
                                              : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * kBlock;
            if (i < tiles) order[atomicAdd(&hist[order_key(i, TX, r[u].y - r[u].x)], 1u)] = (uint32_t)i;
        }
    }
}


// Count pass over a block of 256 projected splats (binning after a plain projection).
__global__ __launch_bounds__(kBlock) void k_count(const float4 *__restrict__ rec, const uint32_t *__restrict__ count,
                                                  int n, int TX, uint32_t *__restrict__ cnt_g,
                                                  uint32_t *__restrict__ cnt_n, uint32_t *__restrict__ grp_off) {
    __shared__ EmitLds L;
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t cnt = gi < n ? count[gi] : 0u;
    uint32_t lo = 0u, hi = 0u;
    if (cnt) {
        const float4 r2 = rec[3 * (size_t)gi + 2];
        lo = __float_as_uint(r2.z);
        hi = __float_as_uint(r2.w);
    }
    emit_count(L, cnt, lo, hi, TX, blockIdx.x, cnt_g, cnt_n, grp_off);
}

// Scatter pass, after the scans: per-Gaussian offsets (block offset + block scan), then
// every instance's 64-bit sort key (float-bits(depth) << 32) | gaussian at its position
// in the tile's bucket.  With a tile order the launch has one extra workgroup, the
// first (so that it starts first), which builds the order (also on overflow: the
// blends read it).
__global__ __launch_bounds__(kBlock) void k_scatter(const float4 *__restrict__ rec, const uint32_t *__restrict__ count,
                                                    const uint32_t *__restrict__ partial,
                                                    uint32_t *__restrict__ offset, int n, int TX,
                                                    const uint32_t *__restrict__ misc,
                                                    const uint32_t *__restrict__ grp_off,
                                                    uint32_t *__restrict__ cur_n, uint64_t *__restrict__ bucket,
                                                    const uint32_t *__restrict__ ranges, int tiles,
                                                    uint32_t *__restrict__ order) {
    static_assert(kCells >= kOrderKeys, "the tile order's histogram lives in the cell array");
    __shared__ EmitLds L;
    __shared__ uint32_t tmp4[kBlock / kWave];
    __shared__ uint32_t s_dbits[kBlock];
    const int blk = (int)blockIdx.x - (order ? 1 : 0);
    if (blk < 0) {
        build_tile_order(ranges, tiles, TX, order, L.cell, tmp4);
        return;
    }
    const int tid = threadIdx.x, gi = blk * kBlock + tid;
    if (misc[1] != 0u) {
        // capacity exceeded (or a bad workspace): nothing is emitted and every range is
        // empty.  An offset past any capacity tells the adjoint that this Gaussian owns no
        // instance slot (the slots hold nothing of this frame).
        if (gi < n) offset[gi] = kNoOffset;
        return;
    }
    const uint32_t total = misc[0];
    const uint32_t cnt = gi < n ? count[gi] : 0u;
    const uint32_t excl = block_excl_scan_256(cnt, tmp4);
    if (gi < n) offset[gi] = partial[blk] + excl;
    uint32_t lo = 0u, hi = 0u;
    if (cnt) {
        const float4 r2 = rec[3 * (size_t)gi + 2];
        lo = __float_as_uint(r2.z);
        hi = __float_as_uint(r2.w);
        s_dbits[tid] = __float_as_uint(r2.y);
    }
    const EmitBox B = emit_box(L, cnt, lo, hi);
    if (B.grouped) {
        // each cell's first free position, the tile's start + the block's reservation,
        // loaded for the whole union rectangle at once (a cell without instances reads a
        // reservation the count pass did not write, and never uses it); an LDS atomic on
        // it then hands out the positions
        for (uint32_t c = tid; c < B.uw * B.uh; c += kBlock) {
            const uint32_t tile = (B.by0 + c / B.uw) * (uint32_t)TX + (B.bx0 + c % B.uw);
            L.cell[c] = ranges[2 * tile] + grp_off[(size_t)blk * kCells + c];
        }
        __syncthreads();
    }
    emit_each(L, B, TX, [&](int o, uint32_t tile, uint32_t cell) {
        const uint32_t pos = B.grouped ? atomicAdd(&L.cell[cell], 1u) : atomicAdd(&cur_n[tile], 1u);
        if (pos < total)  // always, when the counters started at zero; a guard for the bucket otherwise
            bucket[pos] = ((uint64_t)s_dbits[o] << 32) | (uint32_t)(blk * kBlock + o);
    });
}

__device__ __forceinline__ void write_out(uint64_t k, uint32_t pos, uint32_t tile, uint64_t *__restrict__ keys,
                                          uint32_t *__restrict__ vals) {
    keys[pos] = ((uint64_t)tile << 32) | (k >> 32);
    vals[pos] = (uint32_t)k;
}

// Orders the wavefront's LDS (and, with the workgroup being one wavefront, global)
// accesses before the ones that follow: a barrier of a one-wavefront workgroup.
__device__ __forceinline__ void wave_step() { __syncthreads(); }

// Number of keys of chunk c of sk (64 keys, sorted or not) below k: np broadcast reads of
// two keys each, np = ceil(len / 2) for a chunk holding len keys (the padding after them,
// ~0, is never below a key).
__device__ __forceinline__ uint32_t chunk_rank(const uint64_t *sk, int c, uint64_t k, uint32_t np) {
    const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(sk + c * kWave);
    uint32_t r = 0;
    if (np == kWave / 2) {
#pragma unroll 8
        for (int j = 0; j < kWave / 2; ++j) {
            const ulonglong2 kk = p[j];
            r += (kk.x < k) + (kk.y < k);
        }
    } else {  // the list's last chunk, partly filled
#pragma unroll 4
        for (uint32_t j = 0; j < np; ++j) {
            const ulonglong2 kk = p[j];
            r += (kk.x < k) + (kk.y < k);
        }
    }
    return r;
}

// ceil(len / 2) for the len = min(64, s - 64 c) keys of chunk c of an s-key list
__device__ __forceinline__ uint32_t chunk_pairs(uint32_t s, int c) {
    return (min(s - (uint32_t)c * kWave, (uint32_t)kWave) + 1u) >> 1;
}

// Lower bound of k in chunk c of sk once it is sorted: the number of its keys below k (0..64),
// by binary search (seven dependent broadcast reads).
__device__ __forceinline__ uint32_t chunk_lower_bound(const uint64_t *sk, int c, uint64_t k) {
    const uint64_t *o = sk + c * kWave;
    uint32_t lb = 0;
#pragma unroll
    for (int step = kWave / 2; step >= 1; step >>= 1) lb += o[lb + step - 1] < k ? (uint32_t)step : 0u;
    return lb + (o[lb] < k ? 1u : 0u);
}

// A list of s <= MAXC * 64 keys, sorted by one wavefront.  Lane l holds keys c * 64 + l
// (chunk c < nch = ceil(s / 64)); the list is staged in sk with the last chunk padded by ~0
// (never below a key: a key's high word is a non-negative float's bits).  Each key is
// ranked inside its chunk (the keys are unique: the rank is the number of the chunk's keys
// below it) and every chunk is rewritten in sorted order in place; a key's position in the
// tile's list is then its rank plus, for every other chunk, its lower bound there.  Per key
// that is at most 64 comparisons (the last chunk's keys only, padding skipped) and
// 7 (nch - 1) probes instead of the s comparisons of ranking against the whole list.  Two chunks are ranked, and two keys searched, side by side, and
// each key's searches of the other chunks are interleaved, so that the dependent LDS reads
// overlap.
template <int MAXC>
__device__ __forceinline__ void wave_merge_sort(const uint64_t *__restrict__ bucket, uint32_t start, uint32_t s,
                                                uint64_t *sk, uint32_t tile, uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    static_assert(MAXC % 2 == 0, "chunks go in pairs");
    const uint32_t ln = lane_id();
    const int nch = (int)((s + kWave - 1) / kWave);
    uint64_t k[MAXC];
    uint32_t r[MAXC];
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
        const uint32_t i = c * kWave + ln;
        k[c] = c < nch && i < s ? bucket[start + i] : ~0ull;
        r[c] = ln;  // padding keeps its own slot at the end of the last chunk
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
        if (c < nch) sk[c * kWave + ln] = k[c];
    wave_step();
#pragma unroll
    for (int c = 0; c < MAXC; c += 2) {
        if (c >= nch) break;
        const uint32_t ra = chunk_rank(sk, c, k[c], chunk_pairs(s, c));
        const uint32_t rb = c + 1 < nch ? chunk_rank(sk, c + 1, k[c + 1], chunk_pairs(s, c + 1)) : 0u;
        if (k[c] != ~0ull) r[c] = ra;
        if (k[c + 1] != ~0ull) r[c + 1] = rb;
    }
    wave_step();  // every lane has read every chunk before they are rewritten
#pragma unroll
    for (int c = 0; c < MAXC; ++c)
        if (c < nch) sk[c * kWave + r[c]] = k[c];
    wave_step();
#pragma unroll
    for (int c = 0; c < MAXC; c += 2) {
        if (c >= nch) break;
        uint32_t pa = r[c], pb = r[c + 1];
#pragma unroll
        for (int d = 0; d < MAXC; ++d) {
            if (d >= nch) continue;
            if (d != c) pa += chunk_lower_bound(sk, d, k[c]);
            if (d != c + 1 && c + 1 < nch) pb += chunk_lower_bound(sk, d, k[c + 1]);
        }
        if (c * kWave + ln < s) write_out(k[c], start + pa, tile, keys, vals);
        if ((c + 1) * kWave + ln < s) write_out(k[c + 1], start + pb, tile, keys, vals);
    }
}

// Stable LSD radix sort of src0[0, s) by all 64 key bits, by one wavefront, 8-bit digits:
// pass 1 reads src0 and writes a, later passes alternate a -> b -> a, so the eighth pass
// leaves the result in b.  Per pass: the digits counted in LDS (cnt, 256 counters), their
// exclusive scan (four counters per lane), then the list in chunks of 64 in order, each
// element placed at its digit's next free slot plus its rank among the chunk's elements of
// the same digit (ballot matching on the eight digit bits): stable.
__device__ void wave_radix_sort(const uint64_t *src0, uint64_t *a, uint64_t *b, uint32_t s, uint32_t *cnt) {
    const uint32_t ln = lane_id();
    const uint64_t lt = lanemask_lt();
    const uint64_t *src = src0;
    uint64_t *dst = a;
    for (int shift = 0; shift < 64; shift += 8) {
#pragma unroll
        for (int q = 0; q < kRadix / kWave; ++q) cnt[q * kWave + ln] = 0u;
        wave_step();
        for (uint32_t i = ln; i < s; i += kWave) atomicAdd(&cnt[(uint32_t)(src[i] >> shift) & 0xffu], 1u);
        wave_step();
        uint32_t c4[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c4[q] = cnt[4 * ln + q];
            sum += c4[q];
        }
        uint32_t run = wave_incl_scan(sum) - sum;
        wave_step();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cnt[4 * ln + q] = run;
            run += c4[q];
        }
        wave_step();
        for (uint32_t r0 = 0; r0 < s; r0 += kWave) {
            const uint32_t i = r0 + ln;
            const bool valid = i < s;
            const uint64_t key = valid ? src[i] : 0ull;
            const uint32_t d = (uint32_t)(key >> shift) & 0xffu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bt = 0; bt < 8; ++bt) {
                const bool bit = (d >> bt) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t base = cnt[d];
            if (valid) dst[base + __popcll(peers & lt)] = key;
            wave_step();  // every lane has read its digit's slot before it moves on
            if (valid && (peers & lt) == 0ull) cnt[d] = base + __popcll(peers);
            wave_step();
        }
        src = dst;
        dst = dst == a ? b : a;
    }
}

// One wavefront per tile.  Lists of up to kWave keys: ranking against the whole list (two
// keys per broadcast read); up to kMergeMax keys: chunk ranks merged by binary search
// (wave_merge_sort); longer lists: radix sort.
constexpr int kMergeMax = 8 * kWave;
static_assert(kRadix == 4 * kWave, "four digit counters per lane");

__device__ __forceinline__ void wave_rank_sort(const uint64_t *__restrict__ bucket, uint32_t start, uint32_t s,
                                               uint64_t *sk, uint32_t tile, uint64_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals) {
    const uint32_t ln = lane_id();
    const uint64_t k = ln < s ? bucket[start + ln] : ~0ull;
    sk[ln] = k;
    wave_step();
    const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(sk);
    const uint32_t np = (s + 1) >> 1;  // an odd list reads the ~0 of lane s as well
    uint32_t r = 0;
    for (uint32_t j = 0; j < np; ++j) {
        const ulonglong2 kk = p[j];
        r += (kk.x < k) + (kk.y < k);
    }
    if (ln < s) write_out(k, start + r, tile, keys, vals);
}

__global__ __launch_bounds__(kWave) void k_tile_sort(const uint64_t *__restrict__ bucket, uint64_t *__restrict__ alt,
                                                    const uint32_t *__restrict__ ranges, int tiles,
                                                    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                    const uint32_t *__restrict__ misc,
                                                    const uint32_t *__restrict__ order, int TX, int TY,
                                                    uint32_t txm) {
    if (misc[1] != 0u) return;
    __shared__ uint64_t sk[kMergeMax];
    int tile, tx, ty, unused;
    if (!tile_unit(blockIdx.x, TX, TY, txm, 1, order, tile, tx, ty, unused)) return;
    const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    const uint32_t s = end - start;
    if (s == 0) return;
    const uint32_t t = (uint32_t)tile;
    if (s <= (uint32_t)kWave) {
        wave_rank_sort(bucket, start, s, sk, t, keys, vals);
    } else if (s <= (uint32_t)(2 * kWave)) {
        wave_merge_sort<2>(bucket, start, s, sk, t, keys, vals);
    } else if (s <= (uint32_t)(4 * kWave)) {
        wave_merge_sort<4>(bucket, start, s, sk, t, keys, vals);
    } else if (s <= (uint32_t)kMergeMax) {
        wave_merge_sort<8>(bucket, start, s, sk, t, keys, vals);
    } else {
        // 8 radix passes bucket -> alt -> keys -> alt ... -> keys (same index range of each);
        // the last pass leaves the sorted list in keys, which write_out then rewrites in
        // place, element by element
        wave_radix_sort(bucket + start, alt + start, keys + start, s, reinterpret_cast<uint32_t *>(sk));
        for (uint32_t i = lane_id(); i < s; i += kWave) write_out(keys[start + i], start + i, t, keys, vals);
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// workspace: bucket keys [cap] u64, alt keys [cap] u64 (the large-bucket radix sort's
// scratch), group reservations [blocks][kCells] u32, grouped and ungrouped tile counters
// and ungrouped cursors [tiles] u32 each, misc [64] u32
size_t sort_workspace_bytes(int n, int64_t capacity, int tiles) {
    const int64_t cap = capacity > 0 ? capacity : 1;
    const size_t nb = (size_t)((n > 0 ? n : 1) + kBlock - 1) / kBlock;
    const size_t tb = align256((size_t)(tiles > 0 ? tiles : 1) * 4);
    return align256(cap * 8) * 2 + align256(nb * kCells * 4) + 3 * tb + align256(64 * 4);
}

SortWs carve_workspace(void *ws, int n, int64_t capacity, int tiles) {
    const int64_t cap = capacity > 0 ? capacity : 1;
    const size_t nb = (size_t)((n > 0 ? n : 1) + kBlock - 1) / kBlock;
    const size_t tb = align256((size_t)(tiles > 0 ? tiles : 1) * 4);
    SortWs w;
    char *p = (char *)ws;
    w.bucket = (uint64_t *)p;
    p += align256(cap * 8);
    w.alt = (uint64_t *)p;
    p += align256(cap * 8);
    w.grp_off = (uint32_t *)p;
    p += align256(nb * kCells * 4);
    w.cnt_g = (uint32_t *)p;
    p += tb;
    w.cnt_n = (uint32_t *)p;
    p += tb;
    w.cur_n = (uint32_t *)p;
    p += tb;
    w.misc = (uint32_t *)p;
    w.counter_bytes = 2 * tb;
    return w;
}

hipError_t clear_bin_counters(const SortWs &ws, hipStream_t st) {
    return hipMemsetAsync(ws.cnt_g, 0, ws.counter_bytes, st);  // cnt_g and cnt_n, adjacent
}

namespace {

// the passes after the count: scatter (with the tile order's extra workgroup) and sort
void launch_scatter_sort(const float4 *rec, const uint32_t *count, uint32_t *offset, const uint32_t *partial, int n,
                         const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                         uint32_t *order, hipStream_t st) {
    const int tiles = c.TX * c.TY;
    const int nb = (n + kBlock - 1) / kBlock;
    if (nb > 0 || order)
        hipLaunchKernelGGL(k_scatter, dim3(nb + (order ? 1 : 0)), dim3(kBlock), 0, st, rec, count, partial, offset, n,
                           c.TX, (const uint32_t *)ws.misc, (const uint32_t *)ws.grp_off, ws.cur_n, ws.bucket,
                           (const uint32_t *)ranges, tiles, order);
    hipLaunchKernelGGL(k_tile_sort, dim3(tile_grid(c.TX, c.TY, 1)), dim3(kWave), 0, st,
                       (const uint64_t *)ws.bucket, ws.alt, ranges, tiles, keys, vals, ws.misc,
                       (const uint32_t *)order, c.TX, c.TY, c.txm);
}

}  // namespace

hipError_t launch_bin_sort(const float4 *rec, const uint32_t *count, uint32_t *offset, uint32_t *partial, int n,
                           const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                           int64_t *num_inst, int64_t capacity, int32_t *d_status, uint32_t *order,
                           hipStream_t st) {
    const int tiles = c.TX * c.TY;
    const int nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partial, nb, capacity, num_inst,
                       ws.misc, d_status, ws.cnt_g, ws.cnt_n, tiles);
    if (nb > 0)
        hipLaunchKernelGGL(k_count, dim3(nb), dim3(kBlock), 0, st, rec, count, n, c.TX, ws.cnt_g, ws.cnt_n,
                           ws.grp_off);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, st, ws.cnt_g, ws.cnt_n, ws.cur_n, tiles, ranges,
                       ws.misc, d_status);
    launch_scatter_sort(rec, count, offset, partial, n, c, ws, keys, vals, ranges, order, st);
    return hipGetLastError();
}

hipError_t launch_bin_counted(const float4 *rec, const uint32_t *count, uint32_t *offset, uint32_t *partial, int n,
                              const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges,
                              int64_t *num_inst, int64_t capacity, int32_t *d_status, uint32_t *order,
                              hipStream_t st) {
    const int nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_scan_both, dim3(1), dim3(kScanThreads), 0, st, partial, nb, capacity, num_inst, ws.misc,
                       d_status, ws.cnt_g, ws.cnt_n, ws.cur_n, c.TX * c.TY, ranges);
    launch_scatter_sort(rec, count, offset, partial, n, c, ws, keys, vals, ranges, order, st);
    return hipGetLastError();
}

}  // namespace d4
