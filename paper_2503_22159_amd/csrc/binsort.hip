// Tile binning and depth-keyed radix sort (the tiled rasteriser of 3D Gaussian
// Splatting that the paper renders with, Sec. 3.2.2).
//
//   k_scan_partials  one block: exclusive scan of the per-block count sums written by
//                    the projection kernel; instance total; capacity check; clears the
//                    tile ranges.
//   k_emit           per block of 256 Gaussians: block-exclusive scan of counts ->
//                    per-Gaussian offsets; then each wave emits the instances of its 64
//                    Gaussians cooperatively (lane j takes instance j of the wave, finds
//                    its owner by binary search over the wave's prefix), so a splat with
//                    a large rectangle does not stall the wave and writes coalesce.
//                    key = (tile << 32) | float-bits(depth), value = Gaussian index, in
//                    ascending Gaussian order (ties in key therefore stay index-ordered).
//   radix sort       least-significant-digit, 8-bit digits over the 31 depth bits (bit 31
//                    of a positive float is always 0) and the tile bits.  Per pass:
//                    per-chunk digit histograms, one-block scan in digit-major order,
//                    then a stable scatter: wave64 ballot "multi-split" ranking of 16
//                    rounds of 256 keys, local reorder in LDS so that every digit's run
//                    leaves the block as contiguous writes.
//   k_ranges         [start, end) of each tile's run in the sorted keys.
//
// The instance count lives on the device; sort kernels loop over chunks up to it, so the
// host never waits for it.
#include "internal.hpp"

namespace d4 {

namespace {

constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *tmp4, uint32_t *total) {
    // 256-thread exclusive scan; tmp4: __shared__ [4]
    const int w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) tmp4[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        const uint32_t x = tmp4[i];
        base += (i < w) ? x : 0u;
        tot += x;
    }
    __syncthreads();
    if (total) *total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint32_t *__restrict__ partial, int nb,
                                                               int64_t capacity, int64_t *__restrict__ num_inst,
                                                               uint32_t *__restrict__ misc,
                                                               int32_t *__restrict__ d_status,
                                                               uint32_t *__restrict__ ranges, int tiles) {
    __shared__ uint64_t wsum[kScanThreads / kWave];
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * tiles; i += kScanThreads) ranges[i] = 0u;
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    uint64_t s = 0;
    for (int i = b0; i < b1; ++i) s += partial[i];
    // block-wide exclusive scan of s (64-bit)
    uint64_t inc = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t u = __shfl_up(inc, o, kWave);
        if (lane_id() >= o) inc += u;
    }
    if (lane_id() == kWave - 1) wsum[tid / kWave] = inc;
    __syncthreads();
    uint64_t base = 0, total = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        base += (i < tid / kWave) ? wsum[i] : 0ull;
        total += wsum[i];
    }
    uint64_t run = base + inc - s;
    for (int i = b0; i < b1; ++i) {
        const uint32_t v = partial[i];
        partial[i] = (uint32_t)min(run, (uint64_t)0xffffffffull);
        run += v;
    }
    if (tid == 0) {
        *num_inst = (int64_t)total;
        const uint64_t eff = min(total, (uint64_t)capacity);
        misc[0] = (uint32_t)eff;
        misc[1] = (total > (uint64_t)capacity) ? (uint32_t)D4DGS_ERR_CAPACITY : 0u;
        if (d_status && total > (uint64_t)capacity) *d_status = D4DGS_ERR_CAPACITY;
    }
}

__global__ __launch_bounds__(kBlock) void k_emit(const float4 *__restrict__ rec, const uint32_t *__restrict__ count,
                                                 const uint32_t *__restrict__ partial, uint32_t *__restrict__ offset,
                                                 int n, int TX, int64_t capacity, uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals) {
    __shared__ uint32_t tmp4[kBlock / kWave];
    __shared__ uint32_t s_incl[kBlock];
    __shared__ uint32_t s_x0[kBlock], s_y0[kBlock], s_w[kBlock], s_dbits[kBlock];
    const int tid = threadIdx.x, gi = blockIdx.x * kBlock + tid;
    const uint32_t cnt = gi < n ? count[gi] : 0u;
    const uint32_t excl = block_excl_scan_256(cnt, tmp4, nullptr);
    const uint32_t boff = partial[blockIdx.x];
    const uint64_t off64 = (uint64_t)boff + excl;
    if (gi < n) offset[gi] = (uint32_t)min(off64, (uint64_t)0xffffffffull);
    // wave-local inclusive prefix and the rectangle of each lane's splat
    const uint32_t winc = wave_incl_scan(cnt);
    s_incl[tid] = winc;
    if (cnt) {
        const float4 r2 = rec[3 * (size_t)gi + 2];
        const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
        s_x0[tid] = lo & 0xffffu;
        s_y0[tid] = lo >> 16;
        s_w[tid] = (hi & 0xffffu) - (lo & 0xffffu);
        s_dbits[tid] = __float_as_uint(r2.y);
    }
    __syncthreads();
    const int wbase = (tid / kWave) * kWave;
    const uint32_t wtotal = s_incl[wbase + kWave - 1];
    // offset of the wave's first instance
    const uint64_t wstart = (uint64_t)boff + (uint64_t)__shfl(excl, 0, kWave);
    for (uint32_t j = lane_id(); j < wtotal; j += kWave) {
        // owner: first lane whose inclusive prefix exceeds j
        int lo = 0, hi = kWave - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_incl[wbase + mid] > j) hi = mid; else lo = mid + 1;
        }
        const int o = wbase + lo;
        const uint32_t first = lo > 0 ? s_incl[o - 1] : 0u;
        const uint32_t kk = j - first;
        const uint32_t w = s_w[o];
        const uint32_t ty = s_y0[o] + kk / w, tx = s_x0[o] + kk % w;
        const uint64_t pos = wstart + j;
        if (pos < (uint64_t)capacity) {
            keys[pos] = ((uint64_t)(ty * (uint32_t)TX + tx) << 32) | s_dbits[o];
            vals[pos] = (uint32_t)(blockIdx.x * kBlock + o);
        }
    }
}

__device__ __forceinline__ uint32_t sort_digit(uint64_t key, int shift) {
    const uint64_t L = ((key >> 32) << 31) | (key & 0x7fffffffull);
    return (uint32_t)(L >> shift) & (kRadix - 1);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint64_t *__restrict__ keys,
                                                           const uint32_t *__restrict__ misc, int shift,
                                                           uint32_t *__restrict__ hist, int64_t max_chunks) {
    __shared__ uint32_t h[kSortThreads / kWave][kRadix];
    const uint32_t n = misc[0];
    const uint32_t nchunks = (n + kSortChunk - 1) / kSortChunk;
    const int tid = threadIdx.x, w = tid / kWave;
    for (uint32_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
#pragma unroll
        for (int i = 0; i < kSortThreads / kWave; ++i) h[i][tid] = 0u;
        __syncthreads();
        const uint32_t base = ch * kSortChunk;
#pragma unroll 4
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t i = base + r * kSortThreads + tid;
            if (i < n) atomicAdd(&h[w][sort_digit(keys[i], shift)], 1u);
        }
        __syncthreads();
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kSortThreads / kWave; ++i) s += h[i][tid];
        hist[(size_t)tid * max_chunks + ch] = s;
        __syncthreads();
    }
}

// Exclusive scan of hist in digit-major order (digit d, then chunk c): offsets of each
// (digit, chunk) run in the output.
__global__ __launch_bounds__(kScanThreads) void k_sort_scan(uint32_t *__restrict__ hist,
                                                           const uint32_t *__restrict__ misc, int64_t max_chunks) {
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const uint32_t n = misc[0];
    const uint32_t nchunks = (n + kSortChunk - 1) / kSortChunk;
    if (nchunks == 0) return;
    const uint32_t L = kRadix * nchunks;
    const int tid = threadIdx.x;
    const uint32_t per = (L + kScanThreads - 1) / kScanThreads;
    const uint32_t i0 = min(L, tid * per), i1 = min(L, i0 + per);
    auto phys = [&](uint32_t i) { return (size_t)(i / nchunks) * max_chunks + (i % nchunks); };
    uint32_t s = 0;
    for (uint32_t i = i0; i < i1; ++i) s += hist[phys(i)];
    uint32_t inc = wave_incl_scan(s);
    if (lane_id() == kWave - 1) wsum[tid / kWave] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < tid / kWave; ++i) base += wsum[i];
    uint32_t run = base + inc - s;
    for (uint32_t i = i0; i < i1; ++i) {
        const size_t p = phys(i);
        const uint32_t v = hist[p];
        hist[p] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint64_t *__restrict__ kin,
                                                              const uint32_t *__restrict__ vin,
                                                              uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                              const uint32_t *__restrict__ misc, int shift,
                                                              const uint32_t *__restrict__ hist, int64_t max_chunks) {
    __shared__ uint64_t skeys[kSortChunk];
    __shared__ uint32_t svals[kSortChunk];
    __shared__ uint32_t cnt[kRadix], dstart[kRadix], goff[kRadix];
    __shared__ uint32_t wcnt[kSortThreads / kWave][kRadix], woff[kSortThreads / kWave][kRadix];
    __shared__ uint32_t tmp4[kSortThreads / kWave];
    const uint32_t n = misc[0];
    const uint32_t nchunks = (n + kSortChunk - 1) / kSortChunk;
    const int tid = threadIdx.x, w = tid / kWave;
    const uint64_t ltmask = lanemask_lt();
    for (uint32_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const uint32_t base = ch * kSortChunk;
        const uint32_t nvalid = min((uint32_t)kSortChunk, n - base);
        uint64_t k[kSortItems];
        uint32_t v[kSortItems], d[kSortItems], lr[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t li = r * kSortThreads + tid;
            const bool valid = li < nvalid;
            k[r] = valid ? kin[base + li] : 0ull;
            v[r] = valid ? vin[base + li] : 0u;
            d[r] = valid ? sort_digit(k[r], shift) : 0xffffffffu;
        }
        cnt[tid] = 0u;
#pragma unroll
        for (int i = 0; i < kSortThreads / kWave; ++i) wcnt[i][tid] = 0u;
        goff[tid] = hist[(size_t)tid * max_chunks + ch];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const bool valid = (uint32_t)(r * kSortThreads + tid) < nvalid;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kRadixBits; ++b) {
                const bool bit = (d[r] >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            const uint32_t rank = __popcll(peers & ltmask);
            if (valid && rank == 0) wcnt[w][d[r]] = __popcll(peers);
            __syncthreads();
            {
                uint32_t run = cnt[tid];
#pragma unroll
                for (int i = 0; i < kSortThreads / kWave; ++i) {
                    const uint32_t c = wcnt[i][tid];
                    woff[i][tid] = run;
                    run += c;
                    wcnt[i][tid] = 0u;
                }
                cnt[tid] = run;
            }
            __syncthreads();
            lr[r] = valid ? woff[w][d[r]] + rank : 0u;
        }
        // chunk-local start of every digit's run
        const uint32_t ds = block_excl_scan_256(cnt[tid], tmp4, nullptr);
        dstart[tid] = ds;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            if ((uint32_t)(r * kSortThreads + tid) < nvalid) {
                const uint32_t lp = dstart[d[r]] + lr[r];
                skeys[lp] = k[r];
                svals[lp] = v[r];
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < nvalid; i += kSortThreads) {
            const uint64_t key = skeys[i];
            const uint32_t dd = sort_digit(key, shift);
            const uint32_t gp = goff[dd] + (i - dstart[dd]);
            kout[gp] = key;
            vout[gp] = svals[i];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_ranges(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ misc,
                                                   uint32_t *__restrict__ ranges) {
    const uint32_t n = misc[0];
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const uint32_t tile = (uint32_t)(keys[j] >> 32);
        if (j == 0 || (uint32_t)(keys[j - 1] >> 32) != tile) ranges[2 * tile] = j;
        if (j == n - 1 || (uint32_t)(keys[j + 1] >> 32) != tile) ranges[2 * tile + 1] = j + 1;
    }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

int sort_passes(int tiles) {
    int tb = 0;
    while ((1ll << tb) < (long long)tiles) ++tb;
    const int bits = 31 + tb;
    return (bits + kRadixBits - 1) / kRadixBits;
}

size_t sort_workspace_bytes(int n, int64_t capacity) {
    (void)n;
    const int64_t cap = capacity > 0 ? capacity : 1;
    const int64_t max_chunks = (cap + kSortChunk - 1) / kSortChunk;
    return align256(cap * 8) + align256(cap * 4) + align256((size_t)kRadix * max_chunks * 4) + align256(64 * 4);
}

SortWs carve_workspace(void *ws, int n, int64_t capacity) {
    (void)n;
    const int64_t cap = capacity > 0 ? capacity : 1;
    SortWs w;
    w.max_chunks = (cap + kSortChunk - 1) / kSortChunk;
    char *p = (char *)ws;
    w.block_sums = nullptr;
    w.alt_keys = (uint64_t *)p;
    p += align256(cap * 8);
    w.alt_vals = (uint32_t *)p;
    p += align256(cap * 4);
    w.hist = (uint32_t *)p;
    p += align256((size_t)kRadix * w.max_chunks * 4);
    w.misc = (uint32_t *)p;
    return w;
}

hipError_t launch_bin_sort(const float4 *rec, const uint32_t *count, uint32_t *offset, uint32_t *partial, int n,
                           const CamK &c, const SortWs &ws, uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t *num_inst,
                           int64_t capacity, int32_t *d_status, hipStream_t st) {
    const int tiles = c.TX * c.TY;
    const int nb = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partial, nb, capacity, num_inst,
                       ws.misc, d_status, ranges, tiles);
    const int passes = sort_passes(tiles);
    // emit into the buffer that the last pass does not write, so the result ends in keys/vals
    uint64_t *k0 = (passes % 2 == 0) ? keys : ws.alt_keys;
    uint32_t *v0 = (passes % 2 == 0) ? vals : ws.alt_vals;
    uint64_t *k1 = (passes % 2 == 0) ? ws.alt_keys : keys;
    uint32_t *v1 = (passes % 2 == 0) ? ws.alt_vals : vals;
    if (nb > 0)
        hipLaunchKernelGGL(k_emit, dim3(nb), dim3(kBlock), 0, st, rec, count, partial, offset, n, c.TX,
                           capacity, k0, v0);
    const int grid = (int)std::min<int64_t>(kSortGrid, ws.max_chunks);
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        hipLaunchKernelGGL(k_sort_hist, dim3(grid), dim3(kSortThreads), 0, st, k0, ws.misc, shift, ws.hist,
                           ws.max_chunks);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, st, ws.hist, ws.misc, ws.max_chunks);
        hipLaunchKernelGGL(k_sort_scatter, dim3(grid), dim3(kSortThreads), 0, st, k0, v0, k1, v1, ws.misc, shift,
                           ws.hist, ws.max_chunks);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    const int rgrid = (int)std::min<int64_t>(2048, (capacity + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ranges, dim3(rgrid > 0 ? rgrid : 1), dim3(kBlock), 0, st, keys, ws.misc, ranges);
    return hipGetLastError();
}

}  // namespace d4
