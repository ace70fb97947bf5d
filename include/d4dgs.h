/*
 * d4dgs.h -- C ABI of the MI355X (gfx950) render path for Disentangled 4D Gaussian
 * Splatting (Feng et al., "Disentangled 4D Gaussian Splatting: Rendering
 * High-Resolution Dynamic World at 343 FPS").
 *
 * A frame at camera C and time t is rendered in four stages, each enqueued
 * asynchronously on the caller's HIP stream:
 *
 *   d4dgs_project     camera stage (once per camera) + time stage (per frame):
 *                     Alg. 1; Eq. 9-15 (projection first, temporal processing
 *                     deferred: temporal opacity falloff and screen-space motion
 *                     are applied after the spatial projection).
 *   d4dgs_bin_sort    tile binning of the projected splats and a depth-keyed sort of
 *                     each tile's list, front to back (the tiled rasteriser the paper
 *                     adopts from 3D Gaussian Splatting, Sec. 3.2.2): one wavefront per
 *                     tile ranks lists of up to 512 keys (in chunks of 64, merged by
 *                     binary search) and radix-sorts longer ones.
 *   d4dgs_project_bin d4dgs_project + d4dgs_bin_sort with the binning's counting done
 *                     by the projection (fewer launches per frame; same output).
 *   d4dgs_render_fwd  per-tile front-to-back alpha blending, Eq. 4.
 *   d4dgs_render_bwd  adjoint of the three stages above (the differentiable
 *                     pipeline of Fig. 3): replays each pixel's transmittance in
 *                     reverse from its final value and returns gradients for every
 *                     per-Gaussian parameter, including mu_t, s_t and the velocity.
 *   d4dgs_serve_*     a continuous-batching render server over one resident scene.
 *   d4dgs_render_times  T frames of one camera at T times (one camera stage).
 *   d4dgs_render_fwd_flow, d4dgs_flow_loss, d4dgs_render_bwd_flow
 *                     the rendered optical flow and the flow-gradient guided
 *                     consistency loss (Sec. 3.3, Eq. 16-17) with their adjoints.
 *   d4dgs_spatial_order, d4dgs_scene_permute
 *                     a one-time reorder of a scene along a 3D Morton curve, which the
 *                     binning's per-(block, tile) counting relies on.
 *   d4dgs_bin_sort_noalloc
 *                     d4dgs_bin_sort with its workspace in a static device array.
 *
 * Conventions
 *  - Every pointer marked (device) is device memory owned by the caller; the library
 *    never frees it and never keeps it beyond the call (the server is the exception:
 *    it keeps the scene pointers until d4dgs_serve_destroy).
 *  - Compute entry points only enqueue work on `stream` (a hipStream_t; NULL is the
 *    legacy default stream) and return without waiting, unless documented otherwise.
 *  - No entry point allocates device memory on the render path: scratch comes from
 *    caller workspaces (d4dgs_workspace_size) or from the server's arena.
 *  - Errors are returned as d4dgs_status; nothing is thrown across the ABI.  A text
 *    description of the last error on the calling thread is in d4dgs_last_error().
 *  - Layouts are planar (structure of arrays) unless stated: a [3][n] array holds
 *    all x, then all y, then all z.
 */
#ifndef D4DGS_H
#define D4DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define D4DGS_ABI_VERSION 8
#define D4DGS_TILE 16           /* tile edge in pixels */
#define D4DGS_CAM_REC_FLOATS 19 /* camera-stage record: p3 u3 covc6 m0_2 md2 rgb3 */
#define D4DGS_REC_FLOATS 12     /* splat record, 3 x float4 per Gaussian */
#define D4DGS_GRAD_FLOATS 12    /* per-instance splat gradient, 3 x float4 */
#define D4DGS_MAX_SH_DEGREE 3

typedef enum {
    D4DGS_OK = 0,
    D4DGS_ERR_INVALID_ARG = 1,   /* a pointer, size or camera field is unusable */
    D4DGS_ERR_OUT_OF_MEMORY = 2, /* a caller buffer or the server arena is too small */
    D4DGS_ERR_CAPACITY = 3,      /* more tile instances than the instance capacity */
    D4DGS_ERR_HIP = 4,           /* the HIP runtime reported an error */
    D4DGS_ERR_BUSY = 5,          /* the server queue is full */
    D4DGS_ERR_NOT_FOUND = 6,     /* unknown ticket */
    D4DGS_ERR_TIMEOUT = 7        /* a wait ran out of time */
} d4dgs_status;

typedef void *d4dgs_stream; /* hipStream_t */

/* Disentangled 4D Gaussians (Eq. 8: s_4D, mu_4D, q, V_3D) plus opacity and colour.
 * All (device), float32, borrowed.  Activated values: scale > 0, t_scale > 0,
 * 0 < opacity < 1.  quat is scalar first (w, x, y, z) and need not be normalised;
 * a zero quaternion culls the Gaussian.  sh is [K][3][n], K = (sh_degree + 1)^2,
 * real spherical harmonics with the Condon-Shortley phase, k = l*l + l + m;
 * colour = max(0, sum_k Y_k(d) sh[k] + 0.5), d the unit direction from the
 * camera centre to the (static) spatial mean. */
typedef struct {
    int32_t n;
    int32_t sh_degree; /* 0..3 */
    const float *mean;     /* [3][n] mu_x, mu_y, mu_z */
    const float *scale;    /* [3][n] s_x, s_y, s_z */
    const float *quat;     /* [4][n] */
    const float *opacity;  /* [n] */
    const float *t_mean;   /* [n] mu_t */
    const float *t_scale;  /* [n] s_t */
    const float *velocity; /* [3][n] velocity of the mean, d mu / dt */
    const float *sh;       /* [K][3][n] */
} d4dgs_scene;

/* Pinhole camera (host struct).  R is world-to-camera, row major; the camera looks
 * along +z with x right and y down; pixel (px, py) is sampled at (px + 0.5, py + 0.5).
 * tan_fovx = width / (2 fx), tan_fovy = height / (2 fy): passed rather than derived
 * so that every implementation uses the same bits.  znear > 0. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float tan_fovx, tan_fovy;
    float znear;
    float R[9];
    float T[3];
    float campos[3]; /* camera centre in world space (= -R^T T) */
} d4dgs_camera;

/* Camera-stage cache (Alg. 1: the camera branch runs only when the camera changes).
 * `rec` (device) holds D4DGS_CAM_REC_FLOATS * capacity floats, planar
 * [p.xyz, u.xyz, covc(00,01,02,11,12,22), m0.xy, md.xy, rgb][capacity].  The library
 * fills the other fields; set `valid` to 0 after changing the scene's parameters.
 * A call hits or misses on the host, when it is made; a miss writes `rec` on the
 * call's stream.  One cache may serve calls on several streams (frames of one camera
 * rendered concurrently): the caller then orders a missing call after the other
 * streams' earlier calls with the cache, and their later calls after it (events). */
typedef struct {
    float *rec;
    int32_t capacity;
    int32_t valid;
    d4dgs_camera cam;
    const void *scene_key;
    int32_t scene_n, scene_sh_degree;
    uint64_t hits, misses; /* statistics */
} d4dgs_cam_cache;

/* Per-frame splat record written by d4dgs_project (all device, capacity >= scene n).
 *   rec    [n][12] floats (48 B per Gaussian, 16-byte aligned):
 *          {m.x, m.y, conic.a, conic.b, conic.c, amax, r, g, b, depth,
 *           rect0, rect1}
 *          m = 2D mean at t in pixels, conic = inverse of the dilated 2D covariance
 *          (a = inv[0][0], b = inv[0][1], c = inv[1][1]), amax = o * w(t), rgb the
 *          colour, depth = camera-space z of the mean at t; rect0/rect1 are uint32 bit
 *          patterns x0 | y0 << 16 and x1 | y1 << 16 (tiles, half open).  Only written
 *          for Gaussians with count > 0.
 *   count  [n] uint32 tiles touched (0 = culled).
 *   offset [n] uint32 exclusive prefix of count (written by d4dgs_bin_sort); 0xffffffff for
 *          every Gaussian when the binning failed (instance overflow or a workspace whose
 *          tile counters were not zero), so that d4dgs_render_bwd on such bins adds nothing.
 *   partial [ceil(capacity / 256)] uint32 scratch: per-block sums of count written by
 *          d4dgs_project and turned into block offsets by d4dgs_bin_sort.
 *   mdot   [n][2] floats, optional (NULL: not written): the velocity of the 2D mean at
 *          t in pixels per unit of t -- f u_xy / p_z under the linear motion of Eq. 13 --
 *          for Gaussians with count > 0.  Needed by the flow render and its adjoint.
 *   motion the time stage's motion / covariance model (d4dgs_motion), chosen by the
 *          caller: d4dgs_project computes with it and the adjoints differentiate it. */
typedef enum {
    D4DGS_MOTION_LINEAR = 0,   /* Eq. 13 as printed: m = m0 + tau mdot; Jacobian at the moved mean */
    D4DGS_MOTION_EXACT = 1,    /* m = projection of the moved camera-space mean p + tau u */
    D4DGS_MOTION_FROZEN_J = 2  /* linear motion; Jacobian at the camera stage's mean p, so the
                                  2D covariance does not change with t */
} d4dgs_motion;

typedef struct {
    int32_t capacity;
    float *rec;
    uint32_t *count;
    uint32_t *offset;
    uint32_t *partial;
    float *mdot;
    int32_t motion;
} d4dgs_splats;

/* Sorted tile lists written by d4dgs_bin_sort (all device, caller-owned).
 *   keys    [capacity] uint64 (tile << 32) | float-bits(depth), ascending
 *   values  [capacity] uint32 Gaussian index (ties in key by ascending index)
 *   ranges  [2 * tiles] uint32 [start, end) of each tile's list, tile = ty * TX + tx
 *   num_instances  one int64: total instances (may exceed capacity on overflow)
 *   order   [tiles] uint32, optional (NULL: not used): d4dgs_bin_sort writes the tiles
 *           grouped by tile row mod 8 (group 0 first) and, inside a group, ordered by
 *           list length, longest first (lengths in steps of 8, any order inside a
 *           step); the per-tile kernels of d4dgs_bin_sort, d4dgs_render_fwd*,
 *           d4dgs_render_bwd* and d4dgs_render_times then start on the long lists.
 *           Scheduling only: results are identical with or without it.  The blends
 *           need the order written by the d4dgs_bin_sort call of the same bins (entries
 *           >= tiles are skipped, never read out of bounds). */
typedef struct {
    int64_t capacity;
    uint64_t *keys;
    uint32_t *values;
    uint32_t *ranges;
    int64_t *num_instances;
    uint32_t *order;
} d4dgs_bins;

/* Parameter gradients, same planar shapes as d4dgs_scene (all device, float32).
 * d4dgs_render_bwd ADDS into them; zero them first.
 * Optional splitting statistics (Sec. 3.3, temporal splitting: time-domain splitting is
 * guided by the gradient of the t coordinate, spatial splitting by that of xyz), all [n],
 * NULL to skip: for every Gaussian drawn in the view (count > 0), each backward call adds
 * |dL/dmu_t| of this view to split_grad_t, the Euclidean norm of dL/dmu (xyz) of this
 * view to split_grad_xyz, and 1 to split_count. */
typedef struct {
    float *mean, *scale, *quat, *opacity, *t_mean, *t_scale, *velocity, *sh;
    float *split_grad_t, *split_grad_xyz;
    uint32_t *split_count;
} d4dgs_grads;

int32_t d4dgs_abi_version(void);
const char *d4dgs_last_error(void);

/* Bytes of scratch d4dgs_bin_sort and d4dgs_project_bin need for n Gaussians, a
 * width x height image and up to max_instances tile instances.  Writes *bytes; the
 * caller allocates them (device, 256-byte aligned). */
d4dgs_status d4dgs_workspace_size(int32_t n, int32_t width, int32_t height, int64_t max_instances,
                                  size_t *bytes);

/* Zeroes the tile counters of a workspace (same n, width, height, max_instances as its
 * d4dgs_workspace_size), enqueued on `stream`.  d4dgs_project_bin needs them zero when
 * it starts; every d4dgs_project_bin and d4dgs_bin_sort call leaves them zero, so a
 * workspace needs this once, after it is allocated (or after anything else wrote it).
 * INVALID_ARG (nothing written) if workspace_bytes is below what d4dgs_workspace_size
 * gives for these sizes.  Uses hipMemsetAsync: keep it out of captured graphs. */
d4dgs_status d4dgs_workspace_init(void *workspace, size_t workspace_bytes, int32_t n, int32_t width, int32_t height,
                                  int64_t max_instances, d4dgs_stream stream);

/* Camera stage (if `cache` is NULL or misses) and time stage at time t for all
 * scene Gaussians: Alg. 1 camera branch and per-timestamp steps; Eq. 9-15.  Writes
 * splats->rec (for survivors) and splats->count.  With a cache, a bitwise-equal camera
 * on the same scene skips the camera stage.  INVALID_ARG on a bad camera or sizes. */
d4dgs_status d4dgs_project(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                           d4dgs_cam_cache *cache, d4dgs_splats *splats, d4dgs_stream stream);

/* Tile binning and depth sort of the projected splats (the 3DGS tiled rasteriser the
 * paper uses, Sec. 3.2.2): exclusive scan of counts into splats->offset, emission of
 * every (tile, splat) instance of each splat's rectangle into per-tile buckets, a sort
 * of each bucket by (float-bits(depth), Gaussian index), per-tile ranges.  The output
 * is the ascending order of the 64-bit keys (tile << 32) | float-bits(depth) with ties
 * by index.  If the instance total exceeds bins->capacity, *d_status (device int32,
 * may be NULL) is set to D4DGS_ERR_CAPACITY, *num_instances still receives the total,
 * nothing is emitted and every range is empty (a render of such bins shows only the
 * background).  workspace: d4dgs_workspace_size bytes (device); it needs no
 * initialisation. */
d4dgs_status d4dgs_bin_sort(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height,
                            void *workspace, size_t workspace_bytes, d4dgs_bins *bins,
                            int32_t *d_status, d4dgs_stream stream);

/* d4dgs_project followed by d4dgs_bin_sort at the camera's width and height, with
 * identical outputs (splats, offsets, bins, *d_status), in fewer kernels: the
 * projection also counts each tile's instances (the first binning pass), and the two
 * scans run in one launch.  The workspace's tile counters must be zero when the call
 * starts (d4dgs_workspace_init once; every call leaves them zero).  Same errors as the
 * two calls; in addition, if the counters were not zero, *d_status is set to
 * D4DGS_ERR_INVALID_ARG and every range is empty (no write outside the bins). */
d4dgs_status d4dgs_project_bin(const d4dgs_scene *scene, const d4dgs_camera *cam, float t, d4dgs_cam_cache *cache,
                               d4dgs_splats *splats, void *workspace, size_t workspace_bytes, d4dgs_bins *bins,
                               int32_t *d_status, d4dgs_stream stream);

/* As d4dgs_bin_sort, then waits for the stream and returns D4DGS_ERR_CAPACITY on
 * overflow; *num_instances (host, may be NULL) receives the instance total. */
d4dgs_status d4dgs_bin_sort_sync(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height,
                                 void *workspace, size_t workspace_bytes, d4dgs_bins *bins,
                                 int64_t *num_instances, d4dgs_stream stream);

/* Front-to-back blending per tile (Eq. 4, alpha_i = o_i w_i G'_i): for each pixel,
 * over its tile's list: skip a splat whose exponent is positive or whose alpha
 * (= min(0.99, amax * G)) is below 1/255; stop before a splat that would bring the
 * transmittance below 1e-4.  img (device) [3][height][width] = C + T * bg.
 * final_T [height][width] and n_contrib [height][width] (device, uint32: list
 * position + 1 of the last blended splat) are the replay state of the backward;
 * pass NULL for both to render only. */
d4dgs_status d4dgs_render_fwd(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width,
                              int32_t height, const float bg[3], float *img, float *final_T,
                              uint32_t *n_contrib, d4dgs_stream stream);

/* d4dgs_render_fwd with the blend kernel timed: start_event and stop_event are
 * hipEvent_t handles, created by the caller with timing enabled, and are set to the
 * start and the end of the blend kernel itself (not of the stream position around
 * it), so that hipEventElapsedTime(start, stop) is the kernel's duration.  For
 * measurement; the output is that of d4dgs_render_fwd.  NULL events are an error. */
d4dgs_status d4dgs_render_fwd_timed(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width,
                                    int32_t height, const float bg[3], float *img, float *final_T,
                                    uint32_t *n_contrib, void *start_event, void *stop_event,
                                    d4dgs_stream stream);

/* Adjoint of d4dgs_project + d4dgs_render_fwd at the same (scene, camera, t) and the
 * same splats/bins/replay state.  dL_dimg (device) [3][height][width].  Replays each
 * pixel's transmittance backwards from final_T (no per-splat forward state), writes
 * one gradient per tile instance into inst_grads (device, D4DGS_GRAD_FLOATS * capacity
 * floats; exposed for stage tests), then sums each Gaussian's instances in a fixed
 * order and applies the chain rule through the time and camera stages.  Adds into
 * `grads`.  Deterministic: no atomics. */
d4dgs_status d4dgs_render_bwd(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                              const d4dgs_splats *splats, const d4dgs_bins *bins, const float bg[3],
                              const float *final_T, const uint32_t *n_contrib, const float *dL_dimg,
                              float *inst_grads, d4dgs_grads *grads, d4dgs_stream stream);

/* d4dgs_render_bwd with its two kernels timed: events (host array of four hipEvent_t,
 * created by the caller with timing enabled) are set to the start and end of the blend
 * adjoint (events[0], events[1]) and of the projection adjoint (events[2], events[3]),
 * the kernels' own execution.  For measurement; the result is that of d4dgs_render_bwd.
 * INVALID_ARG if any event is NULL. */
d4dgs_status d4dgs_render_bwd_timed(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                                    const d4dgs_splats *splats, const d4dgs_bins *bins, const float bg[3],
                                    const float *final_T, const uint32_t *n_contrib, const float *dL_dimg,
                                    float *inst_grads, d4dgs_grads *grads, void *const *events, d4dgs_stream stream);

/* Optical flow (Sec. 3.3): as d4dgs_render_fwd, and also blends each splat's screen
 * velocity splats->mdot with the colour weights, F = sum_i mdot_i alpha_i T_i (zero
 * behind the last splat), into flow (device) [2][height][width].  splats->mdot must be
 * set and written by d4dgs_project. */
d4dgs_status d4dgs_render_fwd_flow(const d4dgs_splats *splats, const d4dgs_bins *bins, int32_t width,
                                   int32_t height, const float bg[3], float *img, float *flow, float *final_T,
                                   uint32_t *n_contrib, d4dgs_stream stream);

/* Bytes of scratch d4dgs_flow_loss needs for a width x height image. */
d4dgs_status d4dgs_flow_loss_workspace_size(int32_t width, int32_t height, size_t *bytes);

/* Flow-gradient guided consistency loss (Sec. 3.3, Eq. 16-17) of a rendered image
 * img [3][H][W] and flow [2][H][W] (device):
 *   M = sqrt(u^2 + v^2 + eps); |grad M|, |grad I| by 3x3 Sobel filters over the pixels
 *   whose 3x3 neighbourhood lies in the image (N of them; |grad I| over the three
 *   channels: sqrt(sum_c Gx_c^2 + Gy_c^2)); each divided by its maximum over those
 *   pixels, floored at 1e-6: nM, nI;  L = lambda / N * sum nM (1 - nI).
 * Writes *loss (device float).  If dL_dflow (device [2][H][W]) is not NULL, also writes
 * the gradient of L with respect to the flow, taking the edge weight (1 - nI) and both
 * normalisers as constants (the loss shapes the motion).  Deterministic.  workspace:
 * d4dgs_flow_loss_workspace_size bytes (device, no initialisation needed). */
d4dgs_status d4dgs_flow_loss(const float *img, const float *flow, int32_t width, int32_t height, float lambda,
                             float eps, void *workspace, size_t workspace_bytes, float *loss, float *dL_dflow,
                             d4dgs_stream stream);

/* Adjoint of d4dgs_project + d4dgs_render_fwd_flow: as d4dgs_render_bwd, with the
 * upstream gradient of the flow dL_dflow (device [2][height][width]) as well;
 * splats->mdot must hold the projection's screen velocities. */
d4dgs_status d4dgs_render_bwd_flow(const d4dgs_scene *scene, const d4dgs_camera *cam, float t,
                                   const d4dgs_splats *splats, const d4dgs_bins *bins, const float bg[3],
                                   const float *final_T, const uint32_t *n_contrib, const float *dL_dimg,
                                   const float *dL_dflow, float *inst_grads, d4dgs_grads *grads,
                                   d4dgs_stream stream);

/* Fixed-viewpoint multi-timestamp rendering: the parallel rendering of several frames of
 * one camera that the paper reports (Sec. 4, rendering speed), through Alg. 1 with the
 * camera branch taken once.  Frames i = 0..T-1 at times t[i]:
 *   - the camera stage runs once (not at all on a cache hit; cache may be NULL), and the
 *     time stages of up to 16 frames run in one launch, so the splat records are
 *     bit-identical to d4dgs_project at each t[i];
 *   - each frame is then binned, sorted and blended as by d4dgs_bin_sort +
 *     d4dgs_render_fwd (without replay state), with the frames spread over the library's
 *     own streams of the current device, forked from and joined back onto `stream`.
 * t (host) [T]; splats, bins (host arrays of T structs) and workspace, img (host arrays
 * of T device pointers) describe each frame's buffers as for the single-frame calls;
 * every workspace holds workspace_bytes >= d4dgs_workspace_size for its frame.  If a
 * frame's instances exceed its bins capacity, *d_status (device int32, may be NULL) is
 * set to D4DGS_ERR_CAPACITY and that frame renders only the background.  Calls on one
 * device are serialised against each other while they enqueue. */
d4dgs_status d4dgs_render_times(const d4dgs_scene *scene, const d4dgs_camera *cam, int32_t T, const float *t,
                                d4dgs_cam_cache *cache, d4dgs_splats *splats, d4dgs_bins *bins,
                                void *const *workspace, size_t workspace_bytes, const float bg[3],
                                float *const *img, int32_t *d_status, d4dgs_stream stream);

/* ------------------------------------------------------------ scene order ------
 * The binning counts a block of 256 consecutive Gaussians with one device atomic per
 * (block, tile) when the block's Gaussians are close in space, and with one per tile
 * instance otherwise.  These two calls store a scene in an order that keeps Gaussians
 * close in space close in memory: a one-time step at scene load (or after
 * densification), not part of the render path.  The gradients of a reordered scene come
 * in its order; perm maps them back (gradient j belongs to the caller's Gaussian
 * perm[j]). */
typedef struct {
    float *mean, *scale, *quat, *opacity, *t_mean, *t_scale, *velocity, *sh; /* as d4dgs_scene */
} d4dgs_scene_arrays;

/* Bytes of scratch d4dgs_spatial_order needs for n Gaussians (n <= 2^30). */
d4dgs_status d4dgs_spatial_order_workspace_size(int32_t n, size_t *bytes);

/* perm (device, [n] uint32): the Gaussians in ascending 3D Morton (Z-order) code of their
 * means, ties by index.  The code interleaves, per axis a, the 10-bit cell
 * floor((mu_a - min_a) / (max_a - min_a) * 1023) (clamped to [0, 1023], float arithmetic,
 * min / max over the scene's means), x in the lowest bit.  workspace:
 * d4dgs_spatial_order_workspace_size bytes (device).  Asynchronous on stream. */
d4dgs_status d4dgs_spatial_order(const d4dgs_scene *scene, uint32_t *perm, void *workspace, size_t workspace_bytes,
                                 d4dgs_stream stream);

/* dst->x[c][j] = src->x[c][perm[j]] for every parameter array x of the scene (same n and
 * sh_degree).  perm (device) is any permutation of 0..n-1, e.g. from d4dgs_spatial_order.
 * dst's arrays are caller-owned device buffers, none of them one of src's.  Asynchronous. */
d4dgs_status d4dgs_scene_permute(const d4dgs_scene *src, const uint32_t *perm, const d4dgs_scene_arrays *dst,
                                 d4dgs_stream stream);

/* ------------------------------------------------------ without allocation ------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  d4dgs_bin_sort_noalloc is
 * d4dgs_bin_sort with its workspace in a static device array of the library,
 * D4DGS_STATIC_SCRATCH_BYTES (64 MiB) on each GPU the library runs on, held until the
 * process ends; the call allocates nothing (the array's device address is looked up on
 * the first call on a GPU).  Arguments, outputs and the device status word are those of
 * d4dgs_bin_sort, without the workspace.  OUT_OF_MEMORY (nothing enqueued) when
 * d4dgs_workspace_size(n, width, height, bins->capacity) exceeds
 * D4DGS_STATIC_SCRATCH_BYTES (e.g. 300k Gaussians at 1352x1014 with 1.2M instances need
 * about 28 MiB).  All calls on one GPU share its array: calls whose work overlaps on the
 * device (on streams not ordered against each other) race and give wrong results; calls
 * ordered on one stream are safe.  The tile counters that must start at zero are cleared
 * by the call's own first kernel, so what an earlier call left in the array does not
 * matter. */
#define D4DGS_STATIC_SCRATCH_BYTES (64u << 20)
d4dgs_status d4dgs_bin_sort_noalloc(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height,
                                    d4dgs_bins *bins, int32_t *d_status, d4dgs_stream stream);

/* ------------------------------------------------------------------ serving ------
 * A server keeps one scene resident and renders requests (camera, t, resolution) as
 * they arrive.  Requests are admitted in arrival order while fewer than max_inflight are
 * on the GPU and their scratch fits the free part of the arena (scratch_budget_bytes,
 * reserved at creation); the requests admitted together form a batch whose projection
 * runs as one launch over (request x Gaussian), and each request then bins and blends on
 * the least loaded of n_streams streams and completes on its own (an event per request),
 * so requests that arrive while others run overlap them on the device.  A request's
 * image is bitwise the same whether it is rendered alone or in a batch.  submit/poll/
 * wait/stats are thread-safe. */
typedef struct {
    int32_t max_inflight;         /* requests on the GPU at once, e.g. 64 */
    int32_t max_batch;            /* requests per batch, <= max_inflight */
    int64_t scratch_budget_bytes; /* arena size, e.g. 8 GiB */
    int32_t n_streams;            /* e.g. 4 */
    float bg[3];
    int64_t max_instances_per_pixel_x1000; /* initial instance capacity per request =
                                              width * height * this / 1000 (e.g. 1000); raised
                                              to 1.25 x the instances per pixel of the densest
                                              finished request; a request that overflows is
                                              rendered again with room for all */
    int32_t max_queue;            /* requests waiting for admission; 0 = 4 * max_inflight */
} d4dgs_serve_config;

typedef struct {
    int64_t submit_ns, admit_ns, start_ns, done_ns; /* host steady clock */
    int64_t num_instances;
    int32_t status;  /* d4dgs_status of the request */
    int32_t batch_size;
} d4dgs_req_stats;

typedef struct {
    int64_t submitted, completed, rejected, retried;
    int64_t queued, inflight;
    int64_t batches;
    int64_t arena_bytes, arena_peak_bytes;
} d4dgs_serve_stats;

typedef struct d4dgs_server d4dgs_server;

/* The scene must stay valid until destroy. */
d4dgs_status d4dgs_serve_create(const d4dgs_scene *scene, const d4dgs_serve_config *cfg,
                                d4dgs_server **out);
/* Queue a request; never blocks.  out_img (device) [3][height][width] is written
 * before the request is reported done.  BUSY when max_queue requests already wait. */
d4dgs_status d4dgs_serve_submit(d4dgs_server *s, const d4dgs_camera *cam, float t, float *out_img,
                                uint64_t *ticket);
/* *done = 1 once the image is complete (stats filled, the ticket is then released). */
d4dgs_status d4dgs_serve_poll(d4dgs_server *s, uint64_t ticket, int32_t *done, d4dgs_req_stats *st);
/* Blocks until done or timeout_ns passes (TIMEOUT); fills st and releases the ticket.
 * NOT_FOUND if the ticket is unknown or was released meanwhile by another call. */
d4dgs_status d4dgs_serve_wait(d4dgs_server *s, uint64_t ticket, int64_t timeout_ns, d4dgs_req_stats *st);
d4dgs_status d4dgs_serve_stats_get(d4dgs_server *s, d4dgs_serve_stats *st);
/* Cancels the requests not yet admitted, waits for the admitted ones to finish, then
 * frees the arena and streams; every ticket is invalid afterwards. */
d4dgs_status d4dgs_serve_destroy(d4dgs_server *s);

#ifdef __cplusplus
}
#endif
#endif /* D4DGS_H */
