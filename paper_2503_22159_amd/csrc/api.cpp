// C ABI of libd4dgs: argument checks, the camera-stage cache, workspace carving and
// launches.  Every entry point enqueues on the caller's stream and returns
// (d4dgs_render_times forks onto its own streams and joins back onto the caller's).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace d4 {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

CamK make_camk(const d4dgs_camera &c) {
    CamK k;
    for (int i = 0; i < 9; ++i) k.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) {
        k.T[i] = c.T[i];
        k.campos[i] = c.campos[i];
    }
    k.fx = c.fx;
    k.fy = c.fy;
    k.cx = c.cx;
    k.cy = c.cy;
    // guard band of the Jacobian: 1.3 x the half field of view, rounded as in float
    volatile float g = kGuard;
    k.limx = g * c.tan_fovx;
    k.limy = g * c.tan_fovy;
    k.znear = c.znear;
    k.W = c.width;
    k.H = c.height;
    k.TX = (c.width + kTile - 1) / kTile;
    k.TY = (c.height + kTile - 1) / kTile;
    k.txm = div_magic((uint32_t)k.TX);
    return k;
}

static bool finite_f(float x) { return std::isfinite(x); }

bool image_size_ok(int32_t w, int32_t h) {
    // tile rectangles pack tile coordinates into 16 bits, and the per-tile launches have
    // 4 workgroups per tile in a grid of 32-bit size
    if (w <= 0 || h <= 0 || w > 65535 * kTile || h > 65535 * kTile) return false;
    const int64_t tiles = (int64_t)((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
    return tiles <= ((int64_t)1 << 26);
}

const char *camera_problem(const d4dgs_camera &c) {
    if (!image_size_ok(c.width, c.height)) return "camera size out of range";
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !finite_f(c.fx) || !finite_f(c.fy) || !finite_f(c.cx) ||
        !finite_f(c.cy))
        return "camera intrinsics invalid";
    if (!(c.tan_fovx > 0.f) || !(c.tan_fovy > 0.f) || !finite_f(c.tan_fovx) || !finite_f(c.tan_fovy))
        return "camera field of view invalid";
    if (!(c.znear > 0.f) || !finite_f(c.znear)) return "znear must be > 0";
    for (int i = 0; i < 9; ++i)
        if (!finite_f(c.R[i])) return "camera rotation not finite";
    for (int i = 0; i < 3; ++i)
        if (!finite_f(c.T[i]) || !finite_f(c.campos[i])) return "camera position not finite";
    return nullptr;
}

SceneK make_scenek(const d4dgs_scene &s) {
    SceneK k;
    k.n = s.n;
    k.deg = s.sh_degree;
    k.mean = s.mean;
    k.scale = s.scale;
    k.quat = s.quat;
    k.opacity = s.opacity;
    k.t_mean = s.t_mean;
    k.t_scale = s.t_scale;
    k.velocity = s.velocity;
    k.sh = s.sh;
    return k;
}

}  // namespace d4

using namespace d4;

namespace {

d4dgs_status fail(d4dgs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

d4dgs_status hip_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return D4DGS_OK;
    set_error(std::string(where) + ": " + hipGetErrorString(e));
    return D4DGS_ERR_HIP;
}

d4dgs_status check_scene(const d4dgs_scene *s) {
    if (!s) return fail(D4DGS_ERR_INVALID_ARG, "scene is NULL");
    if (s->n < 0) return fail(D4DGS_ERR_INVALID_ARG, "scene n < 0");
    if (s->sh_degree < 0 || s->sh_degree > D4DGS_MAX_SH_DEGREE)
        return fail(D4DGS_ERR_INVALID_ARG, "sh_degree must be 0..3");
    if (s->n > 0 && (!s->mean || !s->scale || !s->quat || !s->opacity || !s->t_mean || !s->t_scale ||
                     !s->velocity || !s->sh))
        return fail(D4DGS_ERR_INVALID_ARG, "scene array is NULL");
    return D4DGS_OK;
}

d4dgs_status check_camera(const d4dgs_camera *c) {
    if (!c) return fail(D4DGS_ERR_INVALID_ARG, "camera is NULL");
    const char *why = camera_problem(*c);
    return why ? fail(D4DGS_ERR_INVALID_ARG, why) : D4DGS_OK;
}

d4dgs_status check_splats(const d4dgs_splats *sp, int n) {
    if (sp && (sp->motion < D4DGS_MOTION_LINEAR || sp->motion > D4DGS_MOTION_FROZEN_J))
        return fail(D4DGS_ERR_INVALID_ARG, "splats->motion is not a d4dgs_motion");
    if (!sp) return fail(D4DGS_ERR_INVALID_ARG, "splats is NULL");
    if (sp->capacity < n) return fail(D4DGS_ERR_OUT_OF_MEMORY, "splats capacity smaller than n");
    if (n > 0 && (!sp->rec || !sp->count || !sp->offset || !sp->partial))
        return fail(D4DGS_ERR_INVALID_ARG, "splats array is NULL");
    return D4DGS_OK;
}

d4dgs_status check_bins(const d4dgs_bins *b) {
    if (!b) return fail(D4DGS_ERR_INVALID_ARG, "bins is NULL");
    if (b->capacity < 1 || b->capacity > (int64_t)0x7fffffff)
        return fail(D4DGS_ERR_INVALID_ARG, "bins capacity must be in [1, 2^31)");
    if (!b->keys || !b->values || !b->ranges || !b->num_instances)
        return fail(D4DGS_ERR_INVALID_ARG, "bins array is NULL");
    return D4DGS_OK;
}

#define D4_TRY(x)                          \
    do {                                   \
        const d4dgs_status _s = (x);       \
        if (_s != D4DGS_OK) return _s;     \
    } while (0)

}  // namespace

extern "C" {

int32_t d4dgs_abi_version(void) { return D4DGS_ABI_VERSION; }

const char *d4dgs_last_error(void) { return g_err.c_str(); }

d4dgs_status d4dgs_workspace_size(int32_t n, int32_t width, int32_t height, int64_t max_instances, size_t *bytes) {
    if (!bytes) return fail(D4DGS_ERR_INVALID_ARG, "bytes is NULL");
    if (n < 0 || !image_size_ok(width, height) || max_instances < 1 || max_instances > (int64_t)0x7fffffff)
        return fail(D4DGS_ERR_INVALID_ARG, "workspace sizes out of range");
    *bytes = sort_workspace_bytes(n, max_instances, ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile));
    return D4DGS_OK;
}

}  // extern "C"

namespace {

// d4dgs_project, and with `bin` the projection that also runs the binning's count pass
d4dgs_status project_impl(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, d4dgs_cam_cache *cache,
                          d4dgs_splats *splats, d4dgs_stream stream, const BinK *bin) {
    const SceneK sk = make_scenek(*scene);
    const CamK ck = make_camk(*cam);
    int mode = 0;
    float *crec = nullptr;
    int ccap = 0;
    if (cache) {
        if (!cache->rec || cache->capacity < scene->n)
            return fail(D4DGS_ERR_OUT_OF_MEMORY, "camera cache capacity smaller than n");
        crec = cache->rec;
        ccap = cache->capacity;
        const bool hit = cache->valid && cache->scene_key == (const void *)scene->mean && cache->scene_n == scene->n &&
                         cache->scene_sh_degree == scene->sh_degree &&
                         std::memcmp(&cache->cam, cam, sizeof(d4dgs_camera)) == 0;
        if (hit) {
            mode = 2;
            cache->hits++;
        } else {
            mode = 1;
            cache->misses++;
        }
    }
    const hipError_t e = launch_project(sk, ck, t, mode, crec, ccap, (float4 *)splats->rec, splats->count,
                                        splats->partial, (float2 *)splats->mdot, splats->motion, (hipStream_t)stream,
                                        bin);
    if (e != hipSuccess) {
        if (cache) cache->valid = 0;
        return hip_status(e, "d4dgs_project");
    }
    if (cache && mode == 1) {
        cache->cam = *cam;
        cache->scene_key = (const void *)scene->mean;
        cache->scene_n = scene->n;
        cache->scene_sh_degree = scene->sh_degree;
        cache->valid = 1;
    }
    return D4DGS_OK;
}

// checks of a binning call: sizes, bins and workspace; the workspace's layout
d4dgs_status check_binning(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height, void *workspace,
                           size_t workspace_bytes, const d4dgs_bins *bins, CamK &ck, SortWs &ws) {
    if (n < 0) return fail(D4DGS_ERR_INVALID_ARG, "n < 0");
    D4_TRY(check_splats(splats, n));
    D4_TRY(check_bins(bins));
    if (!image_size_ok(width, height)) return fail(D4DGS_ERR_INVALID_ARG, "image size out of range");
    if (!workspace) return fail(D4DGS_ERR_INVALID_ARG, "workspace is NULL");
    d4dgs_camera dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.width = width;
    dummy.height = height;
    ck = make_camk(dummy);
    if (workspace_bytes < sort_workspace_bytes(n, bins->capacity, ck.TX * ck.TY))
        return fail(D4DGS_ERR_OUT_OF_MEMORY, "workspace smaller than d4dgs_workspace_size");
    ws = carve_workspace(workspace, n, bins->capacity, ck.TX * ck.TY);
    return D4DGS_OK;
}

}  // namespace

extern "C" {

d4dgs_status d4dgs_project(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, d4dgs_cam_cache *cache,
                           d4dgs_splats *splats, d4dgs_stream stream) {
    D4_TRY(check_scene(scene));
    D4_TRY(check_camera(cam));
    D4_TRY(check_splats(splats, scene->n));
    if (!std::isfinite(t)) return fail(D4DGS_ERR_INVALID_ARG, "t not finite");
    return project_impl(scene, cam, t, cache, splats, stream, nullptr);
}

d4dgs_status d4dgs_workspace_init(void *workspace, size_t workspace_bytes, int32_t n, int32_t width, int32_t height,
                                  int64_t max_instances, d4dgs_stream stream) {
    if (!workspace) return fail(D4DGS_ERR_INVALID_ARG, "workspace is NULL");
    if (n < 0 || !image_size_ok(width, height) || max_instances < 1 || max_instances > (int64_t)0x7fffffff)
        return fail(D4DGS_ERR_INVALID_ARG, "workspace sizes out of range");
    const int tiles = ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    if (workspace_bytes < sort_workspace_bytes(n, max_instances, tiles))
        return fail(D4DGS_ERR_INVALID_ARG, "workspace_bytes below d4dgs_workspace_size");
    return hip_status(clear_bin_counters(carve_workspace(workspace, n, max_instances, tiles), (hipStream_t)stream),
                      "d4dgs_workspace_init");
}

d4dgs_status d4dgs_project_bin(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, d4dgs_cam_cache *cache,
                               d4dgs_splats *splats, void *workspace, size_t workspace_bytes, d4dgs_bins *bins,
                               int32_t *d_status, d4dgs_stream stream) {
    D4_TRY(check_scene(scene));
    D4_TRY(check_camera(cam));
    if (!std::isfinite(t)) return fail(D4DGS_ERR_INVALID_ARG, "t not finite");
    CamK ck;
    SortWs ws;
    D4_TRY(check_binning(splats, scene->n, cam->width, cam->height, workspace, workspace_bytes, bins, ck, ws));
    const BinK bk = {ws.cnt_g, ws.cnt_n, ws.grp_off, ck.TX};
    D4_TRY(project_impl(scene, cam, t, cache, splats, stream, &bk));
    const hipError_t e = launch_bin_counted((const float4 *)splats->rec, splats->count, splats->offset,
                                            splats->partial, scene->n, ck, ws, bins->keys, bins->values,
                                            bins->ranges, bins->num_instances, bins->capacity, d_status,
                                            bins->order, (hipStream_t)stream);
    return hip_status(e, "d4dgs_project_bin");
}

d4dgs_status d4dgs_bin_sort(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height, void *workspace,
                            size_t workspace_bytes, d4dgs_bins *bins, int32_t *d_status, d4dgs_stream stream) {
    CamK ck;
    SortWs ws;
    D4_TRY(check_binning(splats, n, width, height, workspace, workspace_bytes, bins, ck, ws));
    const hipError_t e = launch_bin_sort((const float4 *)splats->rec, splats->count, splats->offset, splats->partial,
                                         n, ck, ws, bins->keys, bins->values, bins->ranges, bins->num_instances,
                                         bins->capacity, d_status, bins->order, (hipStream_t)stream);
    return hip_status(e, "d4dgs_bin_sort");
}

d4dgs_status d4dgs_bin_sort_sync(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height,
                                 void *workspace, size_t workspace_bytes, d4dgs_bins *bins, int64_t *num_instances,
                                 d4dgs_stream stream) {
    D4_TRY(d4dgs_bin_sort(splats, n, width, height, workspace, workspace_bytes, bins, nullptr, stream));
    const int tiles = ((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    const SortWs ws = carve_workspace(workspace, n, bins->capacity, tiles);
    int64_t total = 0;
    uint32_t misc[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(&total, bins->num_instances, sizeof(total), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(misc, ws.misc, sizeof(misc), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    D4_TRY(hip_status(e, "d4dgs_bin_sort_sync"));
    if (num_instances) *num_instances = total;
    if (misc[1] == (uint32_t)D4DGS_ERR_INVALID_ARG)
        return fail(D4DGS_ERR_INVALID_ARG, "workspace tile counters were not zero (see d4dgs_workspace_init)");
    if (misc[1] == (uint32_t)D4DGS_ERR_CAPACITY)
        return fail(D4DGS_ERR_CAPACITY, "tile instances (" + std::to_string(total) + ") exceed capacity (" +
                                            std::to_string(bins->capacity) + ")");
    return D4DGS_OK;
}

namespace {

d4dgs_status render_fwd_impl(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width, int32_t height,
                             const float bg[3], float *img, float *final_T, uint32_t *n_contrib, hipEvent_t e0,
                             hipEvent_t e1, d4dgs_stream stream) {
    if (!splats || !splats->rec) return fail(D4DGS_ERR_INVALID_ARG, "splats is NULL");
    D4_TRY(check_bins(bins));
    if (!image_size_ok(width, height))
        return fail(D4DGS_ERR_INVALID_ARG, "image size out of range");
    if (!bg || !img) return fail(D4DGS_ERR_INVALID_ARG, "bg or img is NULL");
    if ((final_T == nullptr) != (n_contrib == nullptr))
        return fail(D4DGS_ERR_INVALID_ARG, "final_T and n_contrib must both be given or both be NULL");
    d4dgs_camera dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.width = width;
    dummy.height = height;
    const CamK ck = make_camk(dummy);
    const hipError_t e = launch_blend((const float4 *)splats->rec, bins->values, bins->ranges, bins->order, ck, bg,
                                      img, final_T, n_contrib, (hipStream_t)stream, e0, e1);
    return hip_status(e, "d4dgs_render_fwd");
}

}  // namespace

d4dgs_status d4dgs_render_fwd(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width, int32_t height,
                              const float bg[3], float *img, float *final_T, uint32_t *n_contrib,
                              d4dgs_stream stream) {
    return render_fwd_impl(splats, bins, width, height, bg, img, final_T, n_contrib, nullptr, nullptr, stream);
}

d4dgs_status d4dgs_render_fwd_timed(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width,
                                    int32_t height, const float bg[3], float *img, float *final_T,
                                    uint32_t *n_contrib, void *start_event, void *stop_event, d4dgs_stream stream) {
    if (!start_event || !stop_event) return fail(D4DGS_ERR_INVALID_ARG, "start_event or stop_event is NULL");
    return render_fwd_impl(splats, bins, width, height, bg, img, final_T, n_contrib, (hipEvent_t)start_event,
                           (hipEvent_t)stop_event, stream);
}

}  // extern "C"

namespace {

d4dgs_status render_bwd_impl(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, const d4dgs_splats *splats,
                             const d4dgs_bins *bins, const float bg[3], const float *final_T,
                             const uint32_t *n_contrib, const float *dL_dimg, const float *dL_dflow,
                             float *inst_grads, d4dgs_grads *grads, d4dgs_stream stream,
                             void *const *events = nullptr) {
    D4_TRY(check_scene(scene));
    D4_TRY(check_camera(cam));
    D4_TRY(check_splats(splats, scene->n));
    D4_TRY(check_bins(bins));
    if (!bg || !final_T || !n_contrib || !dL_dimg || !inst_grads || !grads)
        return fail(D4DGS_ERR_INVALID_ARG, "render_bwd: NULL argument");
    if (dL_dflow && scene->n > 0 && !splats->mdot)
        return fail(D4DGS_ERR_INVALID_ARG, "render_bwd_flow: splats->mdot is NULL");
    if (scene->n > 0 && (!grads->mean || !grads->scale || !grads->quat || !grads->opacity || !grads->t_mean ||
                         !grads->t_scale || !grads->velocity || !grads->sh))
        return fail(D4DGS_ERR_INVALID_ARG, "render_bwd: gradient array is NULL");
    if ((grads->split_count != nullptr) != (grads->split_grad_t != nullptr) ||
        (grads->split_count != nullptr) != (grads->split_grad_xyz != nullptr))
        return fail(D4DGS_ERR_INVALID_ARG, "render_bwd: splitting statistics must be all set or all NULL");
    const SceneK sk = make_scenek(*scene);
    const CamK ck = make_camk(*cam);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (events)
        for (int i = 0; i < 4; ++i) ev[i] = (hipEvent_t)events[i];
    hipError_t e = launch_blend_bwd((const float4 *)splats->rec, splats->offset, bins->values, bins->ranges,
                                    bins->order, ck, bg,
                                    final_T, n_contrib, dL_dimg, dL_dflow ? (const float2 *)splats->mdot : nullptr,
                                    dL_dflow, (float4 *)inst_grads, bins->capacity, (hipStream_t)stream, ev[0], ev[1]);
    if (e == hipSuccess)
        e = launch_project_bwd(sk, ck, t, (const float4 *)splats->rec, splats->count, splats->offset,
                               (const float4 *)inst_grads, bins->capacity, *grads, splats->motion,
                               (hipStream_t)stream, ev[2], ev[3]);
    return hip_status(e, "d4dgs_render_bwd");
}

}  // namespace

extern "C" {

d4dgs_status d4dgs_render_bwd(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, const d4dgs_splats *splats,
                              const d4dgs_bins *bins, const float bg[3], const float *final_T,
                              const uint32_t *n_contrib, const float *dL_dimg, float *inst_grads, d4dgs_grads *grads,
                              d4dgs_stream stream) {
    return render_bwd_impl(scene, cam, t, splats, bins, bg, final_T, n_contrib, dL_dimg, nullptr, inst_grads, grads,
                           stream);
}

d4dgs_status d4dgs_render_bwd_timed(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                                    const d4dgs_splats *splats, const d4dgs_bins *bins, const float bg[3],
                                    const float *final_T, const uint32_t *n_contrib, const float *dL_dimg,
                                    float *inst_grads, d4dgs_grads *grads, void *const *events, d4dgs_stream stream) {
    if (!events || !events[0] || !events[1] || !events[2] || !events[3])
        return fail(D4DGS_ERR_INVALID_ARG, "render_bwd_timed: four events are needed");
    return render_bwd_impl(scene, cam, t, splats, bins, bg, final_T, n_contrib, dL_dimg, nullptr, inst_grads, grads,
                           stream, events);
}

d4dgs_status d4dgs_render_bwd_flow(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                                   const d4dgs_splats *splats, const d4dgs_bins *bins, const float bg[3],
                                   const float *final_T, const uint32_t *n_contrib, const float *dL_dimg,
                                   const float *dL_dflow, float *inst_grads, d4dgs_grads *grads,
                                   d4dgs_stream stream) {
    if (!dL_dflow) return fail(D4DGS_ERR_INVALID_ARG, "render_bwd_flow: dL_dflow is NULL");
    return render_bwd_impl(scene, cam, t, splats, bins, bg, final_T, n_contrib, dL_dimg, dL_dflow, inst_grads, grads,
                           stream);
}

d4dgs_status d4dgs_render_fwd_flow(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width,
                                   int32_t height, const float bg[3], float *img, float *flow, float *final_T,
                                   uint32_t *n_contrib, d4dgs_stream stream) {
    if (!splats || !splats->rec) return fail(D4DGS_ERR_INVALID_ARG, "splats is NULL");
    if (!splats->mdot) return fail(D4DGS_ERR_INVALID_ARG, "render_fwd_flow: splats->mdot is NULL");
    D4_TRY(check_bins(bins));
    if (!image_size_ok(width, height))
        return fail(D4DGS_ERR_INVALID_ARG, "image size out of range");
    if (!bg || !img || !flow) return fail(D4DGS_ERR_INVALID_ARG, "bg, img or flow is NULL");
    if ((final_T == nullptr) != (n_contrib == nullptr))
        return fail(D4DGS_ERR_INVALID_ARG, "final_T and n_contrib must both be given or both be NULL");
    d4dgs_camera dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    dummy.width = width;
    dummy.height = height;
    const CamK ck = make_camk(dummy);
    const hipError_t e = launch_blend_flow((const float4 *)splats->rec, (const float2 *)splats->mdot, bins->values,
                                           bins->ranges, bins->order, ck, bg, img, flow, final_T, n_contrib,
                                           (hipStream_t)stream);
    return hip_status(e, "d4dgs_render_fwd_flow");
}

d4dgs_status d4dgs_spatial_order_workspace_size(int32_t n, size_t *bytes) {
    if (!bytes) return fail(D4DGS_ERR_INVALID_ARG, "bytes is NULL");
    if (n < 0 || n > (1 << 30)) return fail(D4DGS_ERR_INVALID_ARG, "spatial_order: n outside [0, 2^30]");
    *bytes = spatial_order_workspace_bytes(n);
    return D4DGS_OK;
}

d4dgs_status d4dgs_spatial_order(const d4dgs_scene *scene, uint32_t *perm, void *workspace, size_t workspace_bytes,
                                 d4dgs_stream stream) {
    D4_TRY(check_scene(scene));
    if (scene->n > (1 << 30)) return fail(D4DGS_ERR_INVALID_ARG, "spatial_order: n above 2^30");
    if (scene->n > 0 && (!perm || !workspace)) return fail(D4DGS_ERR_INVALID_ARG, "spatial_order: NULL argument");
    if (workspace_bytes < spatial_order_workspace_bytes(scene->n))
        return fail(D4DGS_ERR_OUT_OF_MEMORY, "spatial_order: workspace smaller than d4dgs_spatial_order_workspace_size");
    return hip_status(launch_spatial_order(scene->mean, scene->n, perm, workspace, (hipStream_t)stream),
                      "d4dgs_spatial_order");
}

d4dgs_status d4dgs_scene_permute(const d4dgs_scene *src, const uint32_t *perm, const d4dgs_scene_arrays *dst,
                                 d4dgs_stream stream) {
    D4_TRY(check_scene(src));
    if (src->n == 0) return D4DGS_OK;
    if (!perm || !dst) return fail(D4DGS_ERR_INVALID_ARG, "scene_permute: NULL argument");
    const float *in[8] = {src->mean, src->scale, src->quat, src->opacity, src->t_mean, src->t_scale, src->velocity,
                          src->sh};
    float *out[8] = {dst->mean, dst->scale, dst->quat, dst->opacity, dst->t_mean, dst->t_scale, dst->velocity,
                     dst->sh};
    const int K = (src->sh_degree + 1) * (src->sh_degree + 1);
    const int comps[8] = {3, 3, 4, 1, 1, 1, 3, 3 * K};
    for (int i = 0; i < 8; ++i) {
        if (!out[i]) return fail(D4DGS_ERR_INVALID_ARG, "scene_permute: destination array is NULL");
        for (int k = 0; k < 8; ++k)
            if ((const float *)out[i] == in[k])
                return fail(D4DGS_ERR_INVALID_ARG, "scene_permute: a destination array is a source array");
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 8 && e == hipSuccess; ++i)
        e = launch_permute(in[i], out[i], perm, src->n, comps[i], (hipStream_t)stream);
    return hip_status(e, "d4dgs_scene_permute");
}

d4dgs_status d4dgs_flow_loss_workspace_size(int32_t width, int32_t height, size_t *bytes) {
    if (!bytes) return fail(D4DGS_ERR_INVALID_ARG, "bytes is NULL");
    if (width <= 0 || height <= 0 || (int64_t)width * height > (int64_t)1 << 30)
        return fail(D4DGS_ERR_INVALID_ARG, "image size out of range");
    *bytes = flow_loss_workspace_bytes(width, height);
    return D4DGS_OK;
}

d4dgs_status d4dgs_flow_loss(const float *img, const float *flow, int32_t width, int32_t height, float lambda,
                             float eps, void *workspace, size_t workspace_bytes, float *loss, float *dL_dflow,
                             d4dgs_stream stream) {
    if (!img || !flow || !workspace || !loss) return fail(D4DGS_ERR_INVALID_ARG, "flow_loss: NULL argument");
    if (width <= 0 || height <= 0 || (int64_t)width * height > (int64_t)1 << 30)
        return fail(D4DGS_ERR_INVALID_ARG, "image size out of range");
    if (!std::isfinite(lambda) || !std::isfinite(eps) || eps < 0.0f)
        return fail(D4DGS_ERR_INVALID_ARG, "flow_loss: lambda must be finite and eps finite and >= 0");
    if (workspace_bytes < flow_loss_workspace_bytes(width, height))
        return fail(D4DGS_ERR_OUT_OF_MEMORY, "workspace smaller than d4dgs_flow_loss_workspace_size");
    const hipError_t e =
        launch_flow_loss(img, flow, width, height, lambda, eps, workspace, loss, dL_dflow, (hipStream_t)stream);
    return hip_status(e, "d4dgs_flow_loss");
}

// Streams and events of d4dgs_render_times, one set per device, created on first use
// and kept until the process ends.
struct TimesPool {
    static constexpr int kStreams = 4;
    std::mutex mu;
    bool ready = false;
    hipStream_t s[kStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kStreams] = {};
};

static TimesPool *times_pool(int dev) {
    static std::mutex mu;
    static std::vector<std::unique_ptr<TimesPool>> pools;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)pools.size() <= dev) pools.resize(dev + 1);
    if (!pools[dev]) pools[dev].reset(new TimesPool());
    return pools[dev].get();
}

d4dgs_status d4dgs_render_times(const d4dgs_scene *scene, const d4dgs_camera *cam, int32_t T, const float *t,
                                d4dgs_cam_cache *cache, d4dgs_splats *splats, d4dgs_bins *bins,
                                void *const *workspace, size_t workspace_bytes, const float bg[3],
                                float *const *img, int32_t *d_status, d4dgs_stream stream) {
    D4_TRY(check_scene(scene));
    D4_TRY(check_camera(cam));
    if (T < 1 || T > (1 << 20)) return fail(D4DGS_ERR_INVALID_ARG, "render_times: T out of range");
    if (!t || !splats || !bins || !workspace || !img || !bg)
        return fail(D4DGS_ERR_INVALID_ARG, "render_times: NULL argument");
    const CamK ck = make_camk(*cam);
    const int tiles = ck.TX * ck.TY;
    for (int i = 0; i < T; ++i) {
        if (!std::isfinite(t[i])) return fail(D4DGS_ERR_INVALID_ARG, "render_times: t not finite");
        D4_TRY(check_splats(&splats[i], scene->n));
        D4_TRY(check_bins(&bins[i]));
        if (!workspace[i] || !img[i]) return fail(D4DGS_ERR_INVALID_ARG, "render_times: NULL frame buffer");
        if (splats[i].motion != splats[0].motion)
            return fail(D4DGS_ERR_INVALID_ARG, "render_times: frames with different motion models");
        if (workspace_bytes < sort_workspace_bytes(scene->n, bins[i].capacity, tiles))
            return fail(D4DGS_ERR_OUT_OF_MEMORY, "render_times: workspace smaller than d4dgs_workspace_size");
    }
    int mode = 0;
    float *crec = nullptr;
    int ccap = 0;
    if (cache) {
        if (!cache->rec || cache->capacity < scene->n)
            return fail(D4DGS_ERR_OUT_OF_MEMORY, "camera cache capacity smaller than n");
        crec = cache->rec;
        ccap = cache->capacity;
        const bool hit = cache->valid && cache->scene_key == (const void *)scene->mean && cache->scene_n == scene->n &&
                         cache->scene_sh_degree == scene->sh_degree &&
                         std::memcmp(&cache->cam, cam, sizeof(d4dgs_camera)) == 0;
        mode = hit ? 2 : 1;
        if (hit) cache->hits++; else cache->misses++;
    }
    int dev = 0;
    D4_TRY(hip_status(hipGetDevice(&dev), "render_times: hipGetDevice"));
    TimesPool *pool = times_pool(dev);
    std::lock_guard<std::mutex> lk(pool->mu);
    if (!pool->ready) {
        for (int k = 0; k < TimesPool::kStreams; ++k) {
            D4_TRY(hip_status(hipStreamCreateWithFlags(&pool->s[k], hipStreamNonBlocking), "render_times: stream"));
            D4_TRY(hip_status(hipEventCreateWithFlags(&pool->join[k], hipEventDisableTiming), "render_times: event"));
        }
        D4_TRY(hip_status(hipEventCreateWithFlags(&pool->fork, hipEventDisableTiming), "render_times: event"));
        pool->ready = true;
    }
    const hipStream_t st = (hipStream_t)stream;
    const SceneK sk = make_scenek(*scene);
    hipError_t e = hipSuccess;
    // time stages, kMaxTimes frames per launch; the first launch runs the camera stage
    for (int c0 = 0; c0 < T && e == hipSuccess; c0 += kMaxTimes) {
        TimesArgs a;
        a.motion = splats[0].motion;
        a.nt = std::min(kMaxTimes, T - c0);
        for (int f = 0; f < a.nt; ++f) {
            const d4dgs_splats &sp = splats[c0 + f];
            a.f[f] = FrameK{t[c0 + f], (float4 *)sp.rec, sp.count, sp.partial};
        }
        const int m = c0 == 0 ? mode : (cache ? 2 : 0);
        e = launch_project_times(sk, ck, m, crec, ccap, a, st);
    }
    if (e != hipSuccess) {
        if (cache) cache->valid = 0;
        return hip_status(e, "render_times: projection");
    }
    if (cache && mode == 1) {
        cache->cam = *cam;
        cache->scene_key = (const void *)scene->mean;
        cache->scene_n = scene->n;
        cache->scene_sh_degree = scene->sh_degree;
        cache->valid = 1;
    }
    // fork: per-frame binning, sort and blend over the pool's streams
    const int S = std::min(TimesPool::kStreams, T);
    e = hipEventRecord(pool->fork, st);
    for (int k = 0; k < S && e == hipSuccess; ++k) e = hipStreamWaitEvent(pool->s[k], pool->fork, 0);
    for (int i = 0; i < T && e == hipSuccess; ++i) {
        const hipStream_t fs = pool->s[i % S];
        const SortWs ws = carve_workspace(workspace[i], scene->n, bins[i].capacity, tiles);
        e = launch_bin_sort((const float4 *)splats[i].rec, splats[i].count, splats[i].offset, splats[i].partial,
                            scene->n, ck, ws, bins[i].keys, bins[i].values, bins[i].ranges, bins[i].num_instances,
                            bins[i].capacity, d_status, bins[i].order, fs);
        if (e == hipSuccess)
            e = launch_blend((const float4 *)splats[i].rec, bins[i].values, bins[i].ranges, bins[i].order, ck, bg,
                             img[i], nullptr, nullptr, fs);
    }
    // join (also after a failed launch, so that the caller's stream never runs ahead)
    for (int k = 0; k < S; ++k) {
        const hipError_t e2 = hipEventRecord(pool->join[k], pool->s[k]);
        const hipError_t e3 = e2 == hipSuccess ? hipStreamWaitEvent(st, pool->join[k], 0) : e2;
        if (e == hipSuccess) e = e3;
    }
    return hip_status(e, "render_times");
}

}  // extern "C"
