// Spatial order of a scene (a one-time step at scene load).
//
// The binning's count pass reserves tile ranges per (block of 256 Gaussians, tile) with
// one device atomic each, which pays off when a block's Gaussians are close in space and
// so cover few tiles from any camera; otherwise every instance takes an atomic of its own.
// d4dgs_spatial_order gives the order that makes blocks coherent -- the Gaussians sorted
// along a 3D Morton (Z-order) curve of their means over the scene's bounding box, 10 bits
// per axis, ties by index -- and d4dgs_scene_permute stores a scene in that order.
//
//   k_bbox_init / k_bbox   bounding box of the means (float min / max through atomics on
//                          order-preserving integer images of the floats)
//   k_morton_keys          key = code << 32 | index, padded with ~0 to a power of two
//   k_bitonic_lds          bitonic steps whose partners lie within 2 * kSortT keys, in LDS
//   k_bitonic_global       one bitonic step with a larger partner distance
//   k_perm                 the permutation: the low words of the sorted keys
//   k_permute              dst[j] = src[perm[j]] for every planar parameter array
// The keys are unique (the index is part of each), so the unstable bitonic network still
// gives one order.
#include <algorithm>
#include <string>

#include "internal.hpp"

namespace d4 {

namespace {

constexpr int kSortT = 512;          // threads of a bitonic LDS block
constexpr int kSortL = 2 * kSortT;   // keys of a bitonic LDS block

// float <-> unsigned integer with the same order
__device__ __forceinline__ uint32_t f2ord(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// bb[0..2] = min, bb[3..5] = max (order images)
__global__ void k_bbox_init(uint32_t *__restrict__ bb) {
    if (threadIdx.x < 3) bb[threadIdx.x] = 0xffffffffu;
    else if (threadIdx.x < 6) bb[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_bbox(const float *__restrict__ mean, int n, uint32_t *__restrict__ bb) {
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const uint32_t o = f2ord(mean[(size_t)a * n + i]);
            lo[a] = min(lo[a], o);
            hi[a] = max(hi[a], o);
        }
    }
    // wave, then block reduction: one atomic per block and bound (device atomics on the six
    // words serialise, so the grid is kept to one block per compute unit)
    __shared__ uint32_t part[6][256 / kWave];
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min_u32_uniform(lo[a]);
        hi[a] = wave_max_u32_uniform(hi[a]);
        if (lane_id() == 0) {
            part[a][w] = lo[a];
            part[3 + a][w] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        uint32_t v = part[a][0];
#pragma unroll
        for (int i = 1; i < 256 / kWave; ++i) v = a < 3 ? min(v, part[a][i]) : max(v, part[a][i]);
        if (a < 3)
            atomicMin(&bb[a], v);
        else
            atomicMax(&bb[a], v);
    }
}

// the low 10 bits of x spread to every third bit
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ __launch_bounds__(256) void k_morton_keys(const float *__restrict__ mean, int n, int n2,
                                                     const uint32_t *__restrict__ bb, uint64_t *__restrict__ keys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    uint32_t code = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = ord2f(bb[a]), hi = ord2f(bb[3 + a]);
        const float span = fmaxf(hi - lo, 1e-30f);
        const float q = floorf(((mean[(size_t)a * n + i] - lo) / span) * 1023.0f);
        const uint32_t qi = (uint32_t)fminf(fmaxf(q, 0.0f), 1023.0f);
        code |= spread10(qi) << a;
    }
    keys[i] = ((uint64_t)code << 32) | (uint32_t)i;
}

// Compare-exchange of positions i < l (l = i ^ j) in the ascending bitonic network for
// merge size k: the pair is ordered ascending when i & k == 0.
__device__ __forceinline__ void cmpx(uint64_t &a, uint64_t &b, bool up) {
    if ((a > b) == up) {
        const uint64_t t = a;
        a = b;
        b = t;
    }
}

// Steps of the network whose partner distance j is below kSortL, on the block's kSortL
// keys in LDS.  k_lo == 0: the whole network up to merge size kSortL (sorts each block);
// otherwise the steps j = kSortL / 2 ... 1 of merge size k_lo.
__global__ __launch_bounds__(kSortT) void k_bitonic_lds(uint64_t *__restrict__ keys, int k_lo) {
    __shared__ uint64_t s[kSortL];
    const size_t base = (size_t)blockIdx.x * kSortL;
    const int t = threadIdx.x;
    s[t] = keys[base + t];
    s[t + kSortT] = keys[base + t + kSortT];
    __syncthreads();
    const int k0 = k_lo ? k_lo : 2, k1 = k_lo ? k_lo : kSortL;
    for (int k = k0; k <= k1; k <<= 1) {
        for (int j = min(k, kSortL) >> 1; j > 0; j >>= 1) {
            // thread t handles the pair (i, i + j) with i's bit j clear
            const int i = 2 * t - (t & (j - 1));
            const bool up = ((base + (size_t)i) & (size_t)k) == 0;
            cmpx(s[i], s[i + j], up);
            __syncthreads();
        }
    }
    keys[base + t] = s[t];
    keys[base + t + kSortT] = s[t + kSortT];
}

__global__ __launch_bounds__(256) void k_bitonic_global(uint64_t *__restrict__ keys, int n2, int j, int k) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 / 2) return;
    const int i = 2 * t - (t & (j - 1));
    const bool up = (i & k) == 0;
    uint64_t a = keys[i], b = keys[i + j];
    if ((a > b) == up) {
        keys[i] = b;
        keys[i + j] = a;
    }
}

__global__ __launch_bounds__(256) void k_perm(const uint64_t *__restrict__ keys, int n, uint32_t *__restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (uint32_t)keys[i];
}

// dst[c][j] = src[c][perm[j]] for c < comps (planar [comps][n])
__global__ __launch_bounds__(256) void k_permute(const float *__restrict__ src, float *__restrict__ dst,
                                                 const uint32_t *__restrict__ perm, int n, int comps) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t g = perm[j];
    for (int c = 0; c < comps; ++c) dst[(size_t)c * n + j] = src[(size_t)c * n + g];
}

int pow2_keys(int n) {
    int n2 = kSortL;
    while (n2 < n) n2 <<= 1;
    return n2;
}

}  // namespace

size_t spatial_order_workspace_bytes(int n) {
    return (size_t)pow2_keys(std::max(n, 1)) * sizeof(uint64_t) + 256;
}

hipError_t launch_spatial_order(const float *mean, int n, uint32_t *perm, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int n2 = pow2_keys(n);
    uint64_t *keys = (uint64_t *)ws;
    uint32_t *bb = (uint32_t *)((char *)ws + (size_t)n2 * sizeof(uint64_t));
    hipLaunchKernelGGL(k_bbox_init, dim3(1), dim3(64), 0, st, bb);
    hipLaunchKernelGGL(k_bbox, dim3(std::min(256, (n + 255) / 256)), dim3(256), 0, st, mean, n, bb);
    hipLaunchKernelGGL(k_morton_keys, dim3((n2 + 255) / 256), dim3(256), 0, st, mean, n, n2, (const uint32_t *)bb,
                       keys);
    const int blocks = n2 / kSortL;
    hipLaunchKernelGGL(k_bitonic_lds, dim3(blocks), dim3(kSortT), 0, st, keys, 0);
    for (int k = 2 * kSortL; k <= n2; k <<= 1) {
        for (int j = k >> 1; j >= kSortL; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3((n2 / 2 + 255) / 256), dim3(256), 0, st, keys, n2, j, k);
        hipLaunchKernelGGL(k_bitonic_lds, dim3(blocks), dim3(kSortT), 0, st, keys, k);
    }
    hipLaunchKernelGGL(k_perm, dim3((n + 255) / 256), dim3(256), 0, st, (const uint64_t *)keys, n, perm);
    return hipGetLastError();
}

hipError_t launch_permute(const float *src, float *dst, const uint32_t *perm, int n, int comps, hipStream_t st) {
    if (n == 0 || comps == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, perm, n, comps);
    return hipGetLastError();
}

}  // namespace d4
