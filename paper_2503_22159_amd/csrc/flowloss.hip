// Flow-gradient guided consistency loss (Sec. 3.3, Eq. 16-17) on a rendered image and
// optical flow, and its gradient with respect to the flow.
//
//   M = sqrt(u^2 + v^2 + eps)                                   (Eq. 16)
//   |grad M|, |grad I| by 3x3 Sobel filters (Kx = [[-1,0,1],[-2,0,2],[-1,0,1]] along a
//   row, Ky its transpose) at the pixels whose 3x3 neighbourhood lies in the image;
//   |grad I|^2 = sum over the three channels of Gx^2 + Gy^2;
//   nM, nI = each magnitude over its maximum (floored at 1e-6);
//   L = lambda / N * sum nM (1 - nI)                            (Eq. 17)
// The gradient treats the edge weight (1 - nI) and both maxima as constants:
//   dL/dGxM = lambda/N (1 - nI) / maxM * GxM / |grad M|, the transposed Sobel taps carry
//   it to M, and dM/du = u / M.
// Kernels (one thread per pixel, image-sized, HBM-bound): magnitude; Sobel + per-block
// maxima folded with integer atomicMax on the float bits (exact for non-negative values,
// so the result is deterministic); per-pixel terms with a fixed-order block sum; one
// workgroup summing the block sums in order; the transposed Sobel for dL/dflow.
#include "internal.hpp"

namespace d4 {

namespace {

constexpr int kFlT = 256;
constexpr float kNormFloor = 1e-6f;

struct FlowWs {
    float *M, *gx, *gy, *gM, *gI, *cx, *cy, *part;
    uint32_t *maxbits;  // [0] max |grad M|, [1] max |grad I|
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

int fl_blocks(int W, int H) { return (W * H + kFlT - 1) / kFlT; }

FlowWs carve(void *ws, int W, int H) {
    const size_t P = (size_t)W * H;
    char *p = (char *)ws;
    FlowWs w;
    float **bufs[7] = {&w.M, &w.gx, &w.gy, &w.gM, &w.gI, &w.cx, &w.cy};
    for (float **b : bufs) {
        *b = (float *)p;
        p += a256(P * 4);
    }
    w.part = (float *)p;
    p += a256((size_t)fl_blocks(W, H) * 4);
    w.maxbits = (uint32_t *)p;
    return w;
}

__device__ __forceinline__ float block_max(float v, float *sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    float m = sh[0];
#pragma unroll
    for (int i = 1; i < kFlT / kWave; ++i) m = fmaxf(m, sh[i]);
    return m;
}

// fixed-order tree sum over the block (same order on every run)
__device__ __forceinline__ float block_sum(float v, float *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kFlT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    return sh[0];
}

__global__ __launch_bounds__(kFlT) void k_fl_mag(const float *__restrict__ flow, int P, float eps, FlowWs w) {
    const int p = blockIdx.x * kFlT + threadIdx.x;
    if (p == 0) w.maxbits[0] = w.maxbits[1] = 0u;
    if (p >= P) return;
    const float u = flow[p], v = flow[P + p];
    w.M[p] = sqrtf((u * u + v * v) + eps);
}

__device__ __forceinline__ void sobel3(const float *__restrict__ f, int W, int x, int y, float &gx, float &gy) {
    const float *r0 = f + (size_t)(y - 1) * W + x, *r1 = r0 + W, *r2 = r1 + W;
    const float a = r0[-1], b = r0[0], c = r0[1], d = r1[-1], e = r1[1], g = r2[-1], h = r2[0], k = r2[1];
    gx = ((c - a) + 2.0f * (e - d)) + (k - g);
    gy = ((g - a) + 2.0f * (h - b)) + (k - c);
}

__global__ __launch_bounds__(kFlT) void k_fl_sobel(const float *__restrict__ img, int W, int H, FlowWs w) {
    __shared__ float sh[kFlT / kWave];
    const int p = blockIdx.x * kFlT + threadIdx.x;
    const int x = p % W, y = p / W;
    const bool in = p < W * H && x >= 1 && x <= W - 2 && y >= 1 && y <= H - 2;
    float gM = 0.f, gI = 0.f;
    if (in) {
        float gx, gy;
        sobel3(w.M, W, x, y, gx, gy);
        w.gx[p] = gx;
        w.gy[p] = gy;
        gM = sqrtf(gx * gx + gy * gy);
        float s = 0.f;
        const size_t P = (size_t)W * H;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            sobel3(img + ch * P, W, x, y, gx, gy);
            s += gx * gx + gy * gy;
        }
        gI = sqrtf(s);
        w.gM[p] = gM;
        w.gI[p] = gI;
    }
    const float mM = block_max(gM, sh);
    __syncthreads();
    const float mI = block_max(gI, sh);
    if (threadIdx.x == 0) {
        atomicMax(&w.maxbits[0], __float_as_uint(mM));  // non-negative: bit order = value order
        atomicMax(&w.maxbits[1], __float_as_uint(mI));
    }
}

__global__ __launch_bounds__(kFlT) void k_fl_terms(int W, int H, float scale /* lambda / N */, FlowWs w) {
    __shared__ float sh[kFlT];
    const int p = blockIdx.x * kFlT + threadIdx.x;
    const int x = p % W, y = p / W;
    const bool in = p < W * H && x >= 1 && x <= W - 2 && y >= 1 && y <= H - 2;
    const float mM = fmaxf(__uint_as_float(w.maxbits[0]), kNormFloor);
    const float mI = fmaxf(__uint_as_float(w.maxbits[1]), kNormFloor);
    float term = 0.f, cx = 0.f, cy = 0.f;
    if (in) {
        const float gM = w.gM[p];
        const float nM = gM / mM, nI = w.gI[p] / mI;
        term = nM * (1.0f - nI);
        if (gM > 0.0f) {
            const float k = scale * (1.0f - nI) / mM / gM;
            cx = k * w.gx[p];
            cy = k * w.gy[p];
        }
    }
    if (p < W * H) {
        w.cx[p] = cx;
        w.cy[p] = cy;
    }
    const float s = block_sum(term, sh);
    if (threadIdx.x == 0) w.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kFlT) void k_fl_finish(int nb, float scale, const FlowWs w, float *__restrict__ loss) {
    __shared__ float sh[kFlT];
    float s = 0.f;
    for (int i = threadIdx.x; i < nb; i += kFlT) s += w.part[i];
    const float tot = block_sum(s, sh);
    if (threadIdx.x == 0) *loss = scale * tot;
}

// dL/dM(p) = sum over taps (j, i) of Kx[j][i] cx(q) + Ky[j][i] cy(q), q = p - (i - 1, j - 1)
__global__ __launch_bounds__(kFlT) void k_fl_grad(const float *__restrict__ flow, int W, int H, FlowWs w,
                                                 float *__restrict__ dflow) {
    const int p = blockIdx.x * kFlT + threadIdx.x;
    if (p >= W * H) return;
    const int x = p % W, y = p / W;
    const float KX[3][3] = {{-1.f, 0.f, 1.f}, {-2.f, 0.f, 2.f}, {-1.f, 0.f, 1.f}};
    float d = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int qx = x - (i - 1), qy = y - (j - 1);
            if (qx < 1 || qx > W - 2 || qy < 1 || qy > H - 2) continue;
            const size_t q = (size_t)qy * W + qx;
            d += KX[j][i] * w.cx[q] + KX[i][j] * w.cy[q];
        }
    const size_t P = (size_t)W * H;
    const float u = flow[p], v = flow[P + p], M = w.M[p];
    const float r = M > 0.0f ? d / M : 0.0f;
    dflow[p] = r * u;
    dflow[P + p] = r * v;
}

}  // namespace

size_t flow_loss_workspace_bytes(int W, int H) {
    const size_t P = (size_t)W * H;
    return 7 * a256(P * 4) + a256((size_t)fl_blocks(W, H) * 4) + 256;
}

hipError_t launch_flow_loss(const float *img, const float *flow, int W, int H, float lambda, float eps, void *ws,
                            float *loss, float *dL_dflow, hipStream_t st) {
    const FlowWs w = carve(ws, W, H);
    const int P = W * H, nb = fl_blocks(W, H);
    const long long N = (W >= 3 && H >= 3) ? (long long)(W - 2) * (H - 2) : 0;
    const float scale = N > 0 ? lambda / (float)N : 0.0f;
    hipLaunchKernelGGL(k_fl_mag, dim3(nb), dim3(kFlT), 0, st, flow, P, eps, w);
    hipLaunchKernelGGL(k_fl_sobel, dim3(nb), dim3(kFlT), 0, st, img, W, H, w);
    hipLaunchKernelGGL(k_fl_terms, dim3(nb), dim3(kFlT), 0, st, W, H, scale, w);
    hipLaunchKernelGGL(k_fl_finish, dim3(1), dim3(kFlT), 0, st, nb, scale, w, loss);
    if (dL_dflow) hipLaunchKernelGGL(k_fl_grad, dim3(nb), dim3(kFlT), 0, st, flow, W, H, w, dL_dflow);
    return hipGetLastError();
}

}  // namespace d4
