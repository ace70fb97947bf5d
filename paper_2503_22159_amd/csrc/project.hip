// Projection of disentangled 4D Gaussians into dynamic 2D Gaussians (Alg. 1; Eq. 9-15).
//
// Camera stage (runs when the camera changes): camera-space mean (Eq. 9-10) and
// velocity (Eq. 11), pixel-space mean and its first-order velocity (Eq. 12-13),
// W Sigma W^T, and the view-dependent colour.  Sigma = (Rq S)(Rq S)^T depends on the
// Gaussian only and is formed once per Gaussian, also when one launch projects a batch
// of cameras (the server's batched projection reads each Gaussian's parameters once).
// Time stage (runs every frame): temporal weight of the conditional slice, the moved
// mean, the Jacobian at the moved camera-space mean (Eq. 14), Sigma' (Eq. 15), conic,
// screen extent and tile rectangle.  No 4D slicing and no 4x4 work.
//
// FP contract: every quantity that decides an integer (culls, rectangle, depth key) is
// computed with IEEE float +,-,*,/ and sqrt in the written order (compiled with
// -ffp-contract=off; correctly rounded division and square root).  One thread per
// Gaussian; planar loads coalesce across the wave.
#include "emit.hpp"

namespace d4 {

namespace {

struct CamRec {
    float p[3], u[3], cv[6], m0[2], md[2], rgb[3];
};

// Parameters of one Gaussian and its camera-independent covariance.
template <int DEG>
struct GParams {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    bool ok;  // false for a zero quaternion
    float S[9];
    float mu[3], v[3];
    float sh[3 * K];  // [k][rgb]
};

template <int DEG>
__device__ __forceinline__ void load_params(const SceneK &s, int gi, GParams<DEG> &P) {
    const int n = s.n;
    const float q0 = s.quat[gi], q1 = s.quat[n + gi], q2 = s.quat[2 * n + gi], q3 = s.quat[3 * n + gi];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        P.mu[i] = s.mean[i * n + gi];
        P.v[i] = s.velocity[i * n + gi];
    }
#pragma unroll
    for (int k = 0; k < 3 * GParams<DEG>::K; ++k) P.sh[k] = s.sh[(size_t)k * n + gi];
    const float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    P.ok = n2 > 0.0f;
    if (!P.ok) return;
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
    const float sx = s.scale[gi], sy = s.scale[n + gi], sz = s.scale[2 * n + gi];
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        M[3 * i + 0] = Rq[3 * i + 0] * sx;
        M[3 * i + 1] = Rq[3 * i + 1] * sy;
        M[3 * i + 2] = Rq[3 * i + 2] * sz;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            P.S[3 * i + j] =
                (M[3 * i + 0] * M[3 * j + 0] + M[3 * i + 1] * M[3 * j + 1]) + M[3 * i + 2] * M[3 * j + 2];
}

// Real spherical harmonics (Condon-Shortley phase), degrees 0..3, as polynomials in
// the unit direction; constants are the normalisations sqrt((2l+1)/4pi (l-m)!/(l+m)!)
// (times sqrt 2 for m != 0).
template <int DEG>
__device__ __forceinline__ void sh_colour(const float *sh, float x, float y, float z, float rgb[3]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    float Y[16];
    Y[0] = 0.28209479177387814f;
    if (DEG >= 1) {
        Y[1] = -0.4886025119029199f * y;
        Y[2] = 0.4886025119029199f * z;
        Y[3] = -0.4886025119029199f * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = 1.0925484305920792f * (x * y);
        Y[5] = -1.0925484305920792f * (y * z);
        Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
        Y[7] = -1.0925484305920792f * (x * z);
        Y[8] = 0.5462742152960396f * (xx - yy);
        if (DEG >= 3) {
            Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
            Y[10] = 2.890611442640554f * (x * y) * z;
            Y[11] = -0.4570457994644658f * y * (5.0f * zz - 1.0f);
            Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
            Y[13] = -0.4570457994644658f * x * (5.0f * zz - 1.0f);
            Y[14] = 1.445305721320277f * z * (xx - yy);
            Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc = __builtin_fmaf(Y[k], sh[k * 3 + c], acc);
        acc = acc + 0.5f;
        rgb[c] = acc < 0.0f ? 0.0f : acc;
    }
}

// Camera stage (the camera-dependent part).  Requires P.ok.
template <int DEG>
__device__ __forceinline__ void camera_stage(const GParams<DEG> &P, const CamK &c, CamRec &o) {
    const float *R = c.R;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        o.p[i] = ((R[3 * i + 0] * P.mu[0] + R[3 * i + 1] * P.mu[1]) + R[3 * i + 2] * P.mu[2]) + c.T[i];
        o.u[i] = (R[3 * i + 0] * P.v[0] + R[3 * i + 1] * P.v[1]) + R[3 * i + 2] * P.v[2];
    }
    float A[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            A[3 * i + j] =
                (R[3 * i + 0] * P.S[0 * 3 + j] + R[3 * i + 1] * P.S[1 * 3 + j]) + R[3 * i + 2] * P.S[2 * 3 + j];
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int i = ii[e], j = jj[e];
        o.cv[e] = (A[3 * i + 0] * R[3 * j + 0] + A[3 * i + 1] * R[3 * j + 1]) + A[3 * i + 2] * R[3 * j + 2];
    }
    o.m0[0] = (c.fx * o.p[0]) / o.p[2] + c.cx;
    o.m0[1] = (c.fy * o.p[1]) / o.p[2] + c.cy;
    o.md[0] = (c.fx * o.u[0]) / o.p[2];
    o.md[1] = (c.fy * o.u[1]) / o.p[2];
    // colour from the direction camera centre -> static mean
    const float dx = P.mu[0] - c.campos[0], dy = P.mu[1] - c.campos[1], dz = P.mu[2] - c.campos[2];
    const float len = sqrtf((dx * dx + dy * dy) + dz * dz);
    sh_colour<DEG>(P.sh, dx / len, dy / len, dz / len, o.rgb);
}

// Time stage.  Returns the tile count (0 = culled) and fills the splat record.
// motion: D4DGS_MOTION_LINEAR (m = m0 + tau mdot, Jacobian at the moved mean),
// D4DGS_MOTION_EXACT (m = projection of the moved mean), D4DGS_MOTION_FROZEN_J (linear
// motion, Jacobian at the camera stage's mean).  vel receives the 2D mean's velocity at t.
__device__ __forceinline__ uint32_t time_stage(const CamRec &cr, float o_, float mut, float st, float t,
                                               const CamK &c, float4 &r0, float4 &r1, float4 &r2, int motion,
                                               float2 &vel) {
    const float tau = t - mut;
    if (tau * tau > kTemporalCull * (st * st)) return 0;  // temporal weight below 1/255
    const float pz = cr.p[2];
    const float ptx = cr.p[0] + tau * cr.u[0];
    const float pty = cr.p[1] + tau * cr.u[1];
    const float z = pz + tau * cr.u[2];
    if (pz <= c.znear || z <= c.znear) return 0;
    float mx, my;
    if (motion == D4DGS_MOTION_EXACT) {
        mx = (c.fx * ptx) / z + c.cx;
        my = (c.fy * pty) / z + c.cy;
        vel = make_float2((c.fx * (cr.u[0] * z - ptx * cr.u[2])) / (z * z),
                          (c.fy * (cr.u[1] * z - pty * cr.u[2])) / (z * z));
    } else {
        mx = cr.m0[0] + tau * cr.md[0];
        my = cr.m0[1] + tau * cr.md[1];
        vel = make_float2(cr.md[0], cr.md[1]);
    }
    const bool frozen = motion == D4DGS_MOTION_FROZEN_J;
    const float jx = frozen ? cr.p[0] : ptx, jy = frozen ? cr.p[1] : pty, jz = frozen ? pz : z;
    float rx = jx / jz, ry = jy / jz;
    rx = fminf(c.limx, fmaxf(-c.limx, rx));
    ry = fminf(c.limy, fmaxf(-c.limy, ry));
    const float tx = rx * jz, ty = ry * jz;
    const float J00 = c.fx / jz, J11 = c.fy / jz;
    const float J02 = -((c.fx * tx) / (jz * jz)), J12 = -((c.fy * ty) / (jz * jz));
    const float *C = cr.cv;  // 00 01 02 11 12 22
    const float T00 = J00 * C[0] + J02 * C[2];
    const float T02 = J00 * C[2] + J02 * C[5];
    const float T11 = J11 * C[3] + J12 * C[4];
    const float T12 = J11 * C[4] + J12 * C[5];
    const float T01 = J00 * C[1] + J02 * C[4];
    const float a = (T00 * J00 + T02 * J02) + kDilation;
    const float b = T01 * J11 + T02 * J12;
    const float cc = (T11 * J11 + T12 * J12) + kDilation;
    const float det = a * cc - b * b;
    if (!(det > 0.0f)) return 0;
    const float ca = cc / det, cb = -(b / det), ccn = a / det;
    const float mid = 0.5f * (a + cc);
    const float disc = fmaxf(mid * mid - det, 0.1f);
    const float lam1 = mid + sqrtf(disc);
    const float rad = ceilf(3.0f * sqrtf(lam1));
    const float TXf = (float)c.TX, TYf = (float)c.TY;
    const float fx0 = fminf(fmaxf(floorf((mx - rad) / 16.0f), 0.0f), TXf);
    const float fx1 = fminf(fmaxf(floorf((mx + rad) / 16.0f) + 1.0f, 0.0f), TXf);
    const float fy0 = fminf(fmaxf(floorf((my - rad) / 16.0f), 0.0f), TYf);
    const float fy1 = fminf(fmaxf(floorf((my + rad) / 16.0f) + 1.0f, 0.0f), TYf);
    const uint32_t x0 = (uint32_t)fx0, x1 = (uint32_t)fx1, y0 = (uint32_t)fy0, y1 = (uint32_t)fy1;
    const uint32_t cnt = (x1 - x0) * (y1 - y0);
    if (cnt == 0) return 0;
    const float w = expf(-0.5f * ((tau * tau) / (st * st)));
    r0 = make_float4(mx, my, ca, cb);
    r1 = make_float4(ccn, o_ * w, cr.rgb[0], cr.rgb[1]);
    r2 = make_float4(cr.rgb[2], z, __uint_as_float(x0 | (y0 << 16)), __uint_as_float(x1 | (y1 << 16)));
    return cnt;
}

// Block-wide sum of the counts (for the two-level scan in the binning stage).
__device__ __forceinline__ void block_count_sum(uint32_t cnt, uint32_t *block_sums) {
    __shared__ uint32_t part[kBlock / kWave];
    const uint32_t v = wave_sum_u32_uniform(cnt);
    if (lane_id() == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kBlock / kWave; ++w) s += part[w];
        block_sums[blockIdx.x] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ void store_rec(float4 *__restrict__ rec, int gi, const float4 &r0, const float4 &r1,
                                          const float4 &r2) {
    rec[3 * (size_t)gi + 0] = r0;
    rec[3 * (size_t)gi + 1] = r1;
    rec[3 * (size_t)gi + 2] = r2;
}

// MODE 0: camera + time stage; 1: camera + time stage and store the camera record;
// 2: time stage from a stored camera record.  Also writes each block's count sum.  BIN:
// also the binning's count pass over the block's splats (emit.hpp), from the rectangles
// just computed.
template <int MODE, int DEG, bool BIN>
__global__ __launch_bounds__(kBlock) void k_project(SceneK s, CamK c, float t, float *__restrict__ cam_rec,
                                                   int cap, float4 *__restrict__ rec,
                                                   uint32_t *__restrict__ count, uint32_t *__restrict__ block_sums,
                                                   float2 *__restrict__ mdot, int motion, BinK bin) {
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    uint32_t cnt = 0, rlo = 0, rhi = 0;
    if (gi < s.n) {
        CamRec cr;
        bool ok;
        if (MODE == 2) {
            // temporal cull first: the record is only read for Gaussians alive at t
            const float tau = t - s.t_mean[gi], st = s.t_scale[gi];
            ok = !(tau * tau > kTemporalCull * (st * st));
            if (ok) {
#pragma unroll
                for (int i = 0; i < 3; ++i) cr.p[i] = cam_rec[(size_t)i * cap + gi];
#pragma unroll
                for (int i = 0; i < 3; ++i) cr.u[i] = cam_rec[(size_t)(3 + i) * cap + gi];
#pragma unroll
                for (int i = 0; i < 6; ++i) cr.cv[i] = cam_rec[(size_t)(6 + i) * cap + gi];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    cr.m0[i] = cam_rec[(size_t)(12 + i) * cap + gi];
                    cr.md[i] = cam_rec[(size_t)(14 + i) * cap + gi];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) cr.rgb[i] = cam_rec[(size_t)(16 + i) * cap + gi];
            }
        } else {
            GParams<DEG> P;
            load_params<DEG>(s, gi, P);
            ok = P.ok;
            if (ok) {
                camera_stage<DEG>(P, c, cr);
            } else {
                // a zero quaternion: mark the record so that the time stage culls it
#pragma unroll
                for (int i = 0; i < 3; ++i) cr.p[i] = 0.0f;
                cr.p[2] = -1.0f;
            }
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) cam_rec[(size_t)i * cap + gi] = cr.p[i];
                if (ok) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) cam_rec[(size_t)(3 + i) * cap + gi] = cr.u[i];
#pragma unroll
                    for (int i = 0; i < 6; ++i) cam_rec[(size_t)(6 + i) * cap + gi] = cr.cv[i];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        cam_rec[(size_t)(12 + i) * cap + gi] = cr.m0[i];
                        cam_rec[(size_t)(14 + i) * cap + gi] = cr.md[i];
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) cam_rec[(size_t)(16 + i) * cap + gi] = cr.rgb[i];
                }
            }
        }
        if (ok) {
            float4 r0, r1, r2;
            float2 vel;
            cnt = time_stage(cr, s.opacity[gi], s.t_mean[gi], s.t_scale[gi], t, c, r0, r1, r2, motion, vel);
            if (cnt) {
                store_rec(rec, gi, r0, r1, r2);
                if (mdot) mdot[gi] = vel;  // dm/dt at t
                rlo = __float_as_uint(r2.z);
                rhi = __float_as_uint(r2.w);
            }
        }
        count[gi] = cnt;
    }
    if (BIN) {  // the count pass also writes the block's count sum
        __shared__ EmitLds L;
        emit_count(L, cnt, rlo, rhi, bin.TX, blockIdx.x, bin.cnt_g, bin.cnt_n, bin.grp_off, &block_sums[blockIdx.x]);
    } else {
        block_count_sum(cnt, block_sums);
    }
}

// Batched projection for the server: one thread per Gaussian loads its parameters and
// covariance once, then runs the camera and time stages for every request of the batch
// (the same arithmetic as k_project<0>, so each request's record is bit-identical to a
// single-request projection).  A request with counters (q.bin) also gets the binning's
// count pass, as in the single-request projection that counts.
template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_batch(SceneK s, BatchArgs args) {
    __shared__ EmitLds L;
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = gi < s.n;
    GParams<DEG> P;
    float op = 0.f, mut = 0.f, st = 1.f;
    if (valid) {
        load_params<DEG>(s, gi, P);
        op = s.opacity[gi];
        mut = s.t_mean[gi];
        st = s.t_scale[gi];
    } else {
        P.ok = false;
    }
    for (int r = 0; r < args.nreq; ++r) {
        const ReqK &q = args.r[r];
        uint32_t cnt = 0, rlo = 0, rhi = 0;
        if (valid && P.ok) {
            CamRec cr;
            camera_stage<DEG>(P, q.cam, cr);
            float4 r0, r1, r2;
            float2 vel;
            cnt = time_stage(cr, op, mut, st, q.t, q.cam, r0, r1, r2, D4DGS_MOTION_LINEAR, vel);
            if (cnt) {
                store_rec(q.rec, gi, r0, r1, r2);
                rlo = __float_as_uint(r2.z);
                rhi = __float_as_uint(r2.w);
            }
        }
        if (valid) q.count[gi] = cnt;
        if (q.bin.cnt_g) {  // the same for the whole block
            emit_count(L, cnt, rlo, rhi, q.bin.TX, blockIdx.x, q.bin.cnt_g, q.bin.cnt_n, q.bin.grp_off,
                       &q.partial[blockIdx.x]);
            __syncthreads();  // the next request's count pass rewrites the LDS
        } else {
            block_count_sum(cnt, q.partial);
        }
    }
}

// Fixed-viewpoint multi-timestamp projection (Alg. 1 with one camera and many t): each
// thread obtains its Gaussian's camera record once -- from the cache (MODE 2), or by the
// camera stage (MODE 0; MODE 1 also stores it in the cache) -- and runs the time stage for
// every frame of the launch, writing each frame's record, count and block sums.  The
// arithmetic is that of k_project, so every frame is bit-identical to a single-frame
// projection at its t.
template <int MODE, int DEG>
__global__ __launch_bounds__(kBlock) void k_project_times(SceneK s, CamK c, float *__restrict__ cam_rec, int cap,
                                                         TimesArgs args) {
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = gi < s.n;
    CamRec cr;
    bool ok = false;
    float op = 0.f, mut = 0.f, st = 1.f;
    if (valid) {
        op = s.opacity[gi];
        mut = s.t_mean[gi];
        st = s.t_scale[gi];
        if (MODE == 2) {
            ok = true;
#pragma unroll
            for (int i = 0; i < 3; ++i) cr.p[i] = cam_rec[(size_t)i * cap + gi];
#pragma unroll
            for (int i = 0; i < 3; ++i) cr.u[i] = cam_rec[(size_t)(3 + i) * cap + gi];
#pragma unroll
            for (int i = 0; i < 6; ++i) cr.cv[i] = cam_rec[(size_t)(6 + i) * cap + gi];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                cr.m0[i] = cam_rec[(size_t)(12 + i) * cap + gi];
                cr.md[i] = cam_rec[(size_t)(14 + i) * cap + gi];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) cr.rgb[i] = cam_rec[(size_t)(16 + i) * cap + gi];
            // a Gaussian the camera stage culled is stored with p = (0, 0, -1): the time
            // stage's near test culls it
        } else {
            GParams<DEG> P;
            load_params<DEG>(s, gi, P);
            ok = P.ok;
            if (ok) {
                camera_stage<DEG>(P, c, cr);
            } else {
#pragma unroll
                for (int i = 0; i < 3; ++i) cr.p[i] = 0.0f;
                cr.p[2] = -1.0f;
            }
            if (MODE == 1) {
#pragma unroll
                for (int i = 0; i < 3; ++i) cam_rec[(size_t)i * cap + gi] = cr.p[i];
                if (ok) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) cam_rec[(size_t)(3 + i) * cap + gi] = cr.u[i];
#pragma unroll
                    for (int i = 0; i < 6; ++i) cam_rec[(size_t)(6 + i) * cap + gi] = cr.cv[i];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        cam_rec[(size_t)(12 + i) * cap + gi] = cr.m0[i];
                        cam_rec[(size_t)(14 + i) * cap + gi] = cr.md[i];
                    }
#pragma unroll
                    for (int i = 0; i < 3; ++i) cam_rec[(size_t)(16 + i) * cap + gi] = cr.rgb[i];
                }
            }
        }
    }
    for (int f = 0; f < args.nt; ++f) {
        const FrameK &q = args.f[f];
        uint32_t cnt = 0;
        if (valid && ok) {
            float4 r0, r1, r2;
            float2 vel;
            cnt = time_stage(cr, op, mut, st, q.t, c, r0, r1, r2, args.motion, vel);
            if (cnt) store_rec(q.rec, gi, r0, r1, r2);
        }
        if (valid) q.count[gi] = cnt;
        block_count_sum(cnt, q.partial);
    }
}

}  // namespace

hipError_t launch_project(const SceneK &s, const CamK &c, float t, int mode, float *cam_rec, int cam_cap,
                          float4 *rec, uint32_t *count, uint32_t *block_sums, float2 *mdot, int motion,
                          hipStream_t st, const BinK *bin) {
    if (s.n == 0) return hipSuccess;
    const int grid = (s.n + kBlock - 1) / kBlock;
    const BinK nobin = {nullptr, nullptr, nullptr, 0};
#define D4_LAUNCH(M, D)                                                                                        \
    do {                                                                                                       \
        if (bin)                                                                                               \
            hipLaunchKernelGGL((k_project<M, D, true>), dim3(grid), dim3(kBlock), 0, st, s, c, t, cam_rec,     \
                               cam_cap, rec, count, block_sums, mdot, motion, *bin);                           \
        else                                                                                                   \
            hipLaunchKernelGGL((k_project<M, D, false>), dim3(grid), dim3(kBlock), 0, st, s, c, t, cam_rec,    \
                               cam_cap, rec, count, block_sums, mdot, motion, nobin);                          \
    } while (0)
    if (mode == 2) {
        D4_LAUNCH(2, 0);
    } else {
        switch (s.deg * 2 + mode) {
            case 0: D4_LAUNCH(0, 0); break;
            case 1: D4_LAUNCH(1, 0); break;
            case 2: D4_LAUNCH(0, 1); break;
            case 3: D4_LAUNCH(1, 1); break;
            case 4: D4_LAUNCH(0, 2); break;
            case 5: D4_LAUNCH(1, 2); break;
            case 6: D4_LAUNCH(0, 3); break;
            default: D4_LAUNCH(1, 3); break;
        }
    }
#undef D4_LAUNCH
    return hipGetLastError();
}

hipError_t launch_project_batch(const SceneK &s, const BatchArgs &args, hipStream_t st) {
    if (s.n == 0 || args.nreq == 0) return hipSuccess;
    const int grid = (s.n + kBlock - 1) / kBlock;
    switch (s.deg) {
        case 0: hipLaunchKernelGGL(k_project_batch<0>, dim3(grid), dim3(kBlock), 0, st, s, args); break;
        case 1: hipLaunchKernelGGL(k_project_batch<1>, dim3(grid), dim3(kBlock), 0, st, s, args); break;
        case 2: hipLaunchKernelGGL(k_project_batch<2>, dim3(grid), dim3(kBlock), 0, st, s, args); break;
        default: hipLaunchKernelGGL(k_project_batch<3>, dim3(grid), dim3(kBlock), 0, st, s, args); break;
    }
    return hipGetLastError();
}

}  // namespace d4

namespace d4 {

hipError_t launch_project_times(const SceneK &s, const CamK &c, int mode, float *cam_rec, int cam_cap,
                                const TimesArgs &args, hipStream_t st) {
    if (s.n == 0 || args.nt == 0) return hipSuccess;
    const int grid = (s.n + kBlock - 1) / kBlock;
#define D4_LAUNCH(M, D) \
    hipLaunchKernelGGL((k_project_times<M, D>), dim3(grid), dim3(kBlock), 0, st, s, c, cam_rec, cam_cap, args)
    if (mode == 2) {
        D4_LAUNCH(2, 0);
    } else {
        switch (s.deg * 2 + mode) {
            case 0: D4_LAUNCH(0, 0); break;
            case 1: D4_LAUNCH(1, 0); break;
            case 2: D4_LAUNCH(0, 1); break;
            case 3: D4_LAUNCH(1, 1); break;
            case 4: D4_LAUNCH(0, 2); break;
            case 5: D4_LAUNCH(1, 2); break;
            case 6: D4_LAUNCH(0, 3); break;
            default: D4_LAUNCH(1, 3); break;
        }
    }
#undef D4_LAUNCH
    return hipGetLastError();
}

}  // namespace d4
