// Continuous-batching render server (d4dgs_serve_*).
//
// One resident scene; requests (camera, t, resolution) arrive from any thread.  A
// scheduler thread
//   1. retires every request whose work has finished (an event per request), frees its
//      scratch, and retries a request whose tile instances overflowed their capacity
//      (with room for all of them);
//   2. while fewer requests run than there are streams, admits the waiting requests in
//      arrival order -- up to max_batch, while fewer than max_inflight are on the GPU and
//      their scratch fits the free part of the arena (a first-fit allocator over one
//      device reservation of scratch_budget_bytes) -- and launches them as one batch.
//      Requests that arrive while the GPU is busy wait and form the next batch, so
//      batches grow with the load.  A submit that finds the GPU below that load launches
//      its request itself, without waking this thread.
// A batch: one projection launch over (request x Gaussian) -- each Gaussian's parameters
// are read once for the whole batch -- that also runs each request's binning count pass;
// then each request, on the least loaded of n_streams streams (waiting for the
// projection), runs both scans in one launch, the scatter, the sort and the blend (the
// fused binning of d4dgs_project_bin) and completes on its own.  The count pass needs tile
// counters that are zero when it starts: each in-flight slot owns a persistent pair of
// counter arrays, zeroed at creation, which every scan leaves at zero; requests with more
// tiles than a slot's counters hold take the separate binning calls.  Every kernel a
// request runs is the one a single-request render runs, with the same inputs, so its
// image is bitwise the same alone or in any mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace d4;

namespace {

constexpr int64_t kMaxCapacity = 0x7fffffff;  // instance capacities stay below 2^31 (the scans' range)
// tiles of a slot's persistent counters: images up to 32,768 16x16 tiles (e.g. 2896 x 2896)
// take the fused binning
constexpr int kSlotTiles = 32768;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, size) with coalescing.
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = al(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = al(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0;
    d4dgs_camera cam{};
    float t = 0.f;
    float *out = nullptr;
    int64_t capacity = 0;
    d4dgs_req_stats st{};
    bool done = false;
    int retries = 0;
    // scratch
    size_t off = 0, bytes = 0;
    int slot = -1;    // in-flight slot: status words, events, tile counters
    int stream = -1;  // stream of the request's work
};

struct Layout {
    size_t rec, count, offset, partial, keys, vals, ranges, order, ninst, ws, total;
    size_t ws_bytes;
};

Layout layout(int n, int W, int H, int64_t cap) {
    Layout L;
    const int tiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    const size_t nn = (size_t)std::max(n, 1);
    size_t p = 0;
    L.rec = p; p += al(nn * 48);
    L.count = p; p += al(nn * 4);
    L.offset = p; p += al(nn * 4);
    L.partial = p; p += al(((nn + kBlock - 1) / kBlock) * 4);
    L.keys = p; p += al((size_t)cap * 8);
    L.vals = p; p += al((size_t)cap * 4);
    L.ranges = p; p += al((size_t)tiles * 8);
    L.order = p; p += al((size_t)tiles * 4);
    L.ninst = p; p += al(16);
    L.ws_bytes = sort_workspace_bytes(n, cap, tiles);
    L.ws = p; p += al(L.ws_bytes);
    L.total = p;
    return L;
}

}  // namespace

struct d4dgs_server {
    d4dgs_scene scene{};
    SceneK sk{};
    d4dgs_serve_config cfg{};
    char *arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;  // requests running per stream
    int device = 0;
    // per in-flight slot: pinned status words {num_instances (int64), status}; the events
    // marking the end of the request's work and, for the first request of a batch, the
    // end of the batch's projection; the grouped and ungrouped tile counters [2][kSlotTiles]
    // (device), zero between requests
    int64_t *pinned = nullptr;
    std::vector<hipEvent_t> ev_done, ev_proj;
    uint32_t *slot_counters = nullptr;
    std::vector<int> free_slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::vector<Req *> running;  // launched, not yet retired
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    d4dgs_serve_stats stats{};
    int64_t last_activity_ns = 0;  // last launch or retirement (for the polling policy)
    // bumped (under mu) whenever a request finishes, so that waiters can poll without mu
    std::atomic<uint64_t> completions{0};
    // the events of the running requests, for polling without mu (rebuilt under mu
    // whenever `running` changes)
    std::vector<hipEvent_t> running_events;
    std::atomic<int64_t> submitted_count{0};  // stats.submitted, readable without mu
    // instances per pixel (x1000) to give a new request: the configured value, raised to
    // 1.25 x the most any finished request needed, so that few requests overflow and retry
    int64_t ipp_x1000 = 0;
    bool submitted_since(int64_t seen) const { return submitted_count.load(std::memory_order_acquire) != seen; }
    void snapshot_running() {
        running_events.clear();
        for (Req *r : running) running_events.push_back(ev_done[r->slot]);
    }

    void run();
    // While fewer requests run than there are streams: admit waiting requests (up to
    // max_batch, within max_inflight, slots and arena memory) as one batch and launch it.
    // Returns whether anything was launched.  mu held; the calling thread's current device
    // must be the server's.
    bool admit_and_launch();
    // the slot's counters for a request that fits them (else all NULL: separate binning);
    // ws: the request's workspace in the arena (its group reservations)
    BinK slot_bin(const Req *r, void *ws) const {
        const CamK ck = make_camk(r->cam);
        const int tiles = ck.TX * ck.TY;
        if (tiles > kSlotTiles || r->slot < 0) return BinK{nullptr, nullptr, nullptr, 0};
        uint32_t *c = slot_counters + (size_t)r->slot * 2 * kSlotTiles;
        return BinK{c, c + kSlotTiles, carve_workspace(ws, scene.n, r->capacity, tiles).grp_off, ck.TX};
    }
    bool retire();
    void launch(std::vector<Req *> &b);
    void finish(Req *r, int status);
    void requeue(Req *r);
};

void d4dgs_server::finish(Req *r, int status) {
    r->st.status = status;
    r->st.done_ns = now_ns();
    r->done = true;
    completions.fetch_add(1, std::memory_order_release);
    if (r->bytes) arena->release(r->off, r->bytes);
    r->bytes = 0;
    if (r->slot >= 0) free_slots.push_back(r->slot);
    r->slot = -1;
    stats.completed++;
}

// back to the front of the queue, as a new admission
void d4dgs_server::requeue(Req *r) {
    arena->release(r->off, r->bytes);
    r->bytes = 0;
    free_slots.push_back(r->slot);
    r->slot = -1;
    r->retries++;
    stats.retried++;
    pending.push_front(r);
}

// A batch: its requests go to the least loaded streams; the projection of the whole batch
// (one launch per kMaxBatch requests, each Gaussian's parameters read once, the count pass
// of each request included) runs on the first request's stream, and the other requests'
// streams wait for it; then each request's scans, scatter, sort, blend and status copies
// run on its own stream, ending with its own event, so that it completes as soon as its
// own work does.
void d4dgs_server::launch(std::vector<Req *> &b) {
    for (Req *r : b) {
        int si = 0;
        for (int k = 1; k < (int)streams.size(); ++k)
            if (stream_load[k] < stream_load[si]) si = k;
        stream_load[si]++;
        r->stream = si;
    }
    const int lead = b[0]->stream;
    hipError_t e = hipSuccess;
    const int64_t t_start = now_ns();
    for (size_t i0 = 0; i0 < b.size() && e == hipSuccess; i0 += kMaxBatch) {
        BatchArgs a{};
        a.nreq = (int)std::min<size_t>(kMaxBatch, b.size() - i0);
        for (int j = 0; j < a.nreq; ++j) {
            Req *r = b[i0 + j];
            const Layout L = layout(scene.n, r->cam.width, r->cam.height, r->capacity);
            char *base = arena_base + r->off;
            a.r[j].cam = make_camk(r->cam);
            a.r[j].t = r->t;
            a.r[j].rec = (float4 *)(base + L.rec);
            a.r[j].count = (uint32_t *)(base + L.count);
            a.r[j].partial = (uint32_t *)(base + L.partial);
            a.r[j].bin = slot_bin(r, base + L.ws);
        }
        e = launch_project_batch(sk, a, streams[lead]);
    }
    bool fork = false;
    for (Req *r : b) fork = fork || r->stream != lead;
    if (e == hipSuccess && fork) e = hipEventRecord(ev_proj[b[0]->slot], streams[lead]);
    for (Req *r : b) {
        if (e != hipSuccess) break;
        hipStream_t st = streams[r->stream];
        if (r->stream != lead) e = hipStreamWaitEvent(st, ev_proj[b[0]->slot], 0);
        if (e != hipSuccess) break;
        r->st.start_ns = t_start;
        r->st.batch_size = (int)b.size();
        const Layout L = layout(scene.n, r->cam.width, r->cam.height, r->capacity);
        char *base = arena_base + r->off;
        const CamK ck = make_camk(r->cam);
        SortWs ws = carve_workspace(base + L.ws, scene.n, r->capacity, ck.TX * ck.TY);
        const BinK bk = slot_bin(r, base + L.ws);
        if (bk.cnt_g) {  // counted by the projection: the slot's counters
            ws.cnt_g = bk.cnt_g;
            ws.cnt_n = bk.cnt_n;
            e = launch_bin_counted((const float4 *)(base + L.rec), (const uint32_t *)(base + L.count),
                                   (uint32_t *)(base + L.offset), (uint32_t *)(base + L.partial), scene.n, ck, ws,
                                   (uint64_t *)(base + L.keys), (uint32_t *)(base + L.vals),
                                   (uint32_t *)(base + L.ranges), (int64_t *)(base + L.ninst), r->capacity, nullptr,
                                   (uint32_t *)(base + L.order), st);
        } else {
            e = launch_bin_sort((const float4 *)(base + L.rec), (const uint32_t *)(base + L.count),
                                (uint32_t *)(base + L.offset), (uint32_t *)(base + L.partial), scene.n, ck, ws,
                                (uint64_t *)(base + L.keys), (uint32_t *)(base + L.vals),
                                (uint32_t *)(base + L.ranges), (int64_t *)(base + L.ninst), r->capacity, nullptr,
                                (uint32_t *)(base + L.order), st);
        }
        if (e == hipSuccess)
            e = launch_blend((const float4 *)(base + L.rec), (const uint32_t *)(base + L.vals),
                             (const uint32_t *)(base + L.ranges), (const uint32_t *)(base + L.order), ck, cfg.bg,
                             r->out, nullptr, nullptr, st);
        if (e == hipSuccess)  // instance total and overflow status back to pinned memory
            e = hipMemcpyAsync(pinned + 2 * r->slot, base + L.ninst, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pinned + 2 * r->slot + 1, ws.misc + 1, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(ev_done[r->slot], st);
    }
    stats.batches++;
    if (e == hipSuccess) {
        running.insert(running.end(), b.begin(), b.end());
        snapshot_running();
        return;
    }
    // a launch failed: wait for whatever was enqueued, then end the batch with the error
    set_error(std::string("serve launch: ") + hipGetErrorString(e));
    for (Req *r : b) (void)hipStreamSynchronize(streams[r->stream]);
    for (Req *r : b) {
        stream_load[r->stream]--;
        finish(r, D4DGS_ERR_HIP);
    }
    cv_done.notify_all();
}

// Retires every request whose work has finished; returns whether any did.
bool d4dgs_server::retire() {
    bool any = false;
    for (size_t i = 0; i < running.size();) {
        Req *r = running[i];
        const hipError_t q = hipEventQuery(ev_done[r->slot]);
        if (q == hipErrorNotReady) {
            ++i;
            continue;
        }
        running.erase(running.begin() + i);
        stream_load[r->stream]--;
        any = true;
        snapshot_running();
        if (q != hipSuccess) {  // the request's work failed
            set_error(std::string("serve request: ") + hipGetErrorString(q));
            finish(r, D4DGS_ERR_HIP);
            continue;
        }
        const int64_t ninst = pinned[2 * r->slot];
        const uint32_t status = (uint32_t)(pinned[2 * r->slot + 1] & 0xffffffff);
        r->st.num_instances = ninst;
        if (status == (uint32_t)D4DGS_ERR_INVALID_ARG && r->retries < 2) {
            // the slot's counters were not zero (only after a failed launch): clear them
            // and render the request again
            const int slot = r->slot;
            const hipError_t ce = hipMemsetAsync(slot_counters + (size_t)slot * 2 * kSlotTiles, 0,
                                                 sizeof(uint32_t) * 2 * kSlotTiles, streams[r->stream]);
            if (ce != hipSuccess || hipStreamSynchronize(streams[r->stream]) != hipSuccess) {
                set_error("serve: clearing a slot's tile counters failed");
                finish(r, D4DGS_ERR_HIP);
            } else {
                requeue(r);
            }
        } else if (status != 0 && status != (uint32_t)D4DGS_ERR_CAPACITY) {
            set_error("serve: binning reported status " + std::to_string(status));
            finish(r, (int)status);
        } else if (status == (uint32_t)D4DGS_ERR_CAPACITY && ninst > kMaxCapacity) {
            // more instances than any bins can hold (capacities stay below 2^31)
            set_error("serve: request has " + std::to_string(ninst) + " tile instances, above 2^31 - 1");
            finish(r, D4DGS_ERR_CAPACITY);
        } else if (status == (uint32_t)D4DGS_ERR_CAPACITY) {
            // retry with room for every instance (rounded up)
            r->capacity = std::min<int64_t>(std::max<int64_t>(2 * r->capacity, ninst + ninst / 4 + 1024), kMaxCapacity);
            requeue(r);
        } else {
            const int64_t px = (int64_t)r->cam.width * r->cam.height;
            ipp_x1000 = std::max<int64_t>(ipp_x1000, (ninst * 1250 + px - 1) / px);
            finish(r, D4DGS_OK);
        }
    }
    return any;
}

bool d4dgs_server::admit_and_launch() {
    bool launched = false;
    while (!pending.empty() && running.size() < streams.size()) {
        std::vector<Req *> b;
        while (!pending.empty() && (int)(running.size() + b.size()) < cfg.max_inflight &&
               (int)b.size() < cfg.max_batch && !free_slots.empty()) {
            Req *r = pending.front();
            const Layout L = layout(scene.n, r->cam.width, r->cam.height, r->capacity);
            if (L.total > arena->size()) {  // can never fit
                pending.pop_front();
                finish(r, D4DGS_ERR_OUT_OF_MEMORY);
                stats.rejected++;
                cv_done.notify_all();
                continue;
            }
            size_t off;
            if (!arena->alloc(L.total, &off)) break;  // wait for memory
            pending.pop_front();
            r->off = off;
            r->bytes = L.total;
            r->slot = free_slots.back();
            free_slots.pop_back();
            if (!r->st.admit_ns) r->st.admit_ns = now_ns();
            b.push_back(r);
        }
        if (b.empty()) break;  // no slot or no memory until a request retires
        launch(b);
        launched = true;
        last_activity_ns = now_ns();
    }
    return launched;
}

void d4dgs_server::run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (retire()) {  // 1. retire finished requests
            last_activity_ns = now_ns();
            cv_done.notify_all();
        }
        if (admit_and_launch()) continue;  // 2. admit waiting requests while a stream is free
        if (stop && pending.empty() && running.empty()) break;
        if (!running.empty()) {
            // poll the GPU without holding mu (submitters and waiters need it): query the
            // running requests' events until one has finished or a request is submitted.
            // Within kSpinNs of the last launch or retirement (a frame takes ~0.1-0.5 ms)
            // the thread yields the CPU between rounds, so a completion is seen within
            // microseconds (a 20 us sleep takes 60-80 us on Linux: timer slack); after
            // that, short sleeps.
            constexpr int64_t kSpinNs = 2000000;
            const bool spin = now_ns() - last_activity_ns < kSpinNs;
            const std::vector<hipEvent_t> evs = running_events;
            const uint64_t seen = stats.submitted;
            lk.unlock();
            for (int round = 0; round < 64; ++round) {
                bool ready = false;
                for (hipEvent_t ev : evs) ready = ready || hipEventQuery(ev) != hipErrorNotReady;
                if (ready || submitted_since(seen)) break;
                if (spin)
                    std::this_thread::yield();
                else
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
            lk.lock();
        } else {
            cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

extern "C" {

d4dgs_status d4dgs_serve_create(const d4dgs_scene *scene, const d4dgs_serve_config *cfg, d4dgs_server **out) {
    if (!scene || !cfg || !out) {
        set_error("serve_create: NULL argument");
        return D4DGS_ERR_INVALID_ARG;
    }
    if (scene->n < 0 || scene->sh_degree < 0 || scene->sh_degree > D4DGS_MAX_SH_DEGREE ||
        (scene->n > 0 && (!scene->mean || !scene->scale || !scene->quat || !scene->opacity || !scene->t_mean ||
                          !scene->t_scale || !scene->velocity || !scene->sh))) {
        set_error("serve_create: invalid scene");
        return D4DGS_ERR_INVALID_ARG;
    }
    if (cfg->max_inflight < 1 || cfg->max_batch < 1 || cfg->n_streams < 1 || cfg->n_streams > 16 ||
        cfg->scratch_budget_bytes < (1 << 20) || cfg->max_instances_per_pixel_x1000 < 1) {
        set_error("serve_create: invalid config");
        return D4DGS_ERR_INVALID_ARG;
    }
    auto s = std::make_unique<d4dgs_server>();
    s->scene = *scene;
    s->sk = make_scenek(*scene);
    s->cfg = *cfg;
    s->cfg.max_batch = std::min(cfg->max_batch, cfg->max_inflight);
    if (s->cfg.max_queue <= 0) s->cfg.max_queue = 4 * cfg->max_inflight;
    hipError_t e = hipMalloc((void **)&s->arena_base, (size_t)cfg->scratch_budget_bytes);
    if (e != hipSuccess) {
        set_error(std::string("serve_create: arena: ") + hipGetErrorString(e));
        return D4DGS_ERR_OUT_OF_MEMORY;
    }
    s->arena = std::make_unique<Arena>((size_t)cfg->scratch_budget_bytes);
    for (int i = 0; i < cfg->n_streams && e == hipSuccess; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    s->stream_load.assign(s->streams.size(), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->pinned, sizeof(int64_t) * 2 * cfg->max_inflight, 0);
    const size_t counter_bytes = sizeof(uint32_t) * 2 * kSlotTiles * (size_t)cfg->max_inflight;
    if (e == hipSuccess) e = hipMalloc((void **)&s->slot_counters, counter_bytes);
    if (e == hipSuccess) e = hipMemset(s->slot_counters, 0, counter_bytes);
    for (int i = 0; i < cfg->max_inflight && e == hipSuccess; ++i) {
        hipEvent_t a = nullptr, b = nullptr;
        e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
        if (a) s->ev_done.push_back(a);
        if (b) s->ev_proj.push_back(b);
    }
    if (e != hipSuccess) {
        for (auto ev : s->ev_done) (void)hipEventDestroy(ev);
        for (auto ev : s->ev_proj) (void)hipEventDestroy(ev);
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        if (s->pinned) (void)hipHostFree(s->pinned);
        if (s->slot_counters) (void)hipFree(s->slot_counters);
        (void)hipFree(s->arena_base);
        set_error(std::string("serve_create: ") + hipGetErrorString(e));
        return D4DGS_ERR_HIP;
    }
    for (int i = cfg->max_inflight - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->stats.arena_bytes = cfg->scratch_budget_bytes;
    d4dgs_server *raw = s.release();
    (void)hipGetDevice(&raw->device);
    raw->th = std::thread([raw] {
        (void)hipSetDevice(raw->device);  // launches and queries on the creator's device
        raw->run();
    });
    *out = raw;
    return D4DGS_OK;
}

d4dgs_status d4dgs_serve_submit(d4dgs_server *s, const d4dgs_camera *cam, float t, float *out_img,
                                uint64_t *ticket) {
    if (!s || !cam || !out_img || !ticket) {
        set_error("serve_submit: NULL argument");
        return D4DGS_ERR_INVALID_ARG;
    }
    if (const char *why = camera_problem(*cam)) {
        set_error(std::string("serve_submit: ") + why);
        return D4DGS_ERR_INVALID_ARG;
    }
    if (!std::isfinite(t)) {
        set_error("serve_submit: t not finite");
        return D4DGS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        set_error("serve_submit: server is shutting down");
        return D4DGS_ERR_INVALID_ARG;
    }
    if ((int64_t)s->pending.size() >= (int64_t)s->cfg.max_queue) {
        set_error("serve_submit: queue full");
        s->stats.rejected++;
        return D4DGS_ERR_BUSY;
    }
    auto r = std::make_unique<Req>();
    r->ticket = s->next_ticket++;
    r->cam = *cam;
    r->t = t;
    r->out = out_img;
    r->capacity = std::max<int64_t>(1 << 16, (int64_t)cam->width * cam->height *
                                                 std::max(s->cfg.max_instances_per_pixel_x1000, s->ipp_x1000) /
                                                 1000);
    r->capacity = std::min<int64_t>(r->capacity, kMaxCapacity);
    r->st.submit_ns = now_ns();
    r->st.status = -1;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->stats.submitted++;
    s->submitted_count.store(s->stats.submitted, std::memory_order_release);
    if (s->running.size() < s->streams.size()) {
        // a stream is free: launch from this thread (on the server's device) rather than
        // wait for the scheduler to wake up
        int dev = -1;
        if (hipGetDevice(&dev) == hipSuccess) {
            const bool other = dev != s->device;
            if (!other || hipSetDevice(s->device) == hipSuccess) {
                s->admit_and_launch();
                if (other) (void)hipSetDevice(dev);
            }
        }
    }
    s->cv_work.notify_one();
    return D4DGS_OK;
}

d4dgs_status d4dgs_serve_poll(d4dgs_server *s, uint64_t ticket, int32_t *done, d4dgs_req_stats *st) {
    if (!s || !done) return D4DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("serve_poll: unknown ticket");
        return D4DGS_ERR_NOT_FOUND;
    }
    *done = it->second->done ? 1 : 0;
    if (it->second->done) {
        if (st) *st = it->second->st;
        s->reqs.erase(it);
    }
    return D4DGS_OK;
}

d4dgs_status d4dgs_serve_wait(d4dgs_server *s, uint64_t ticket, int64_t timeout_ns, d4dgs_req_stats *st) {
    if (!s) return D4DGS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("serve_wait: unknown ticket");
        return D4DGS_ERR_NOT_FOUND;
    }
    // the ticket is looked up again after every wake-up: another thread may have taken it
    auto ready = [s, ticket] {
        auto f = s->reqs.find(ticket);
        return f == s->reqs.end() || f->second->done;
    };
    // a render takes ~0.1-1 ms: poll (yielding the CPU) for up to kSpinNs before blocking,
    // since waking from a condition variable takes tens of microseconds
    constexpr int64_t kSpinNs = 2000000;
    const int64_t t0 = now_ns(), spin_end = t0 + std::min<int64_t>(timeout_ns, kSpinNs);
    bool ok = ready();
    while (!ok && now_ns() < spin_end) {
        // without mu: wait for any request to finish, then look at this one
        const uint64_t c = s->completions.load(std::memory_order_acquire);
        lk.unlock();
        while (s->completions.load(std::memory_order_acquire) == c && now_ns() < spin_end)
            std::this_thread::yield();
        lk.lock();
        ok = ready();
    }
    if (!ok)
        ok = s->cv_done.wait_for(lk, std::chrono::nanoseconds(std::max<int64_t>(0, timeout_ns - (now_ns() - t0))),
                                 ready);
    if (!ok) {
        set_error("serve_wait: timeout");
        return D4DGS_ERR_TIMEOUT;
    }
    it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("serve_wait: ticket taken by another call");
        return D4DGS_ERR_NOT_FOUND;
    }
    if (st) *st = it->second->st;
    s->reqs.erase(it);
    return D4DGS_OK;
}

d4dgs_status d4dgs_serve_stats_get(d4dgs_server *s, d4dgs_serve_stats *st) {
    if (!s || !st) return D4DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->queued = (int64_t)s->pending.size();
    st->inflight = (int64_t)s->running.size();
    st->arena_peak_bytes = (int64_t)s->arena->peak();
    return D4DGS_OK;
}

d4dgs_status d4dgs_serve_destroy(d4dgs_server *s) {
    if (!s) return D4DGS_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // cancel requests that were never admitted
        for (Req *r : s->pending) {
            r->st.status = D4DGS_ERR_NOT_FOUND;
            r->st.done_ns = now_ns();
            r->done = true;
        }
        s->pending.clear();
        s->cv_work.notify_all();
    }
    s->th.join();  // drains in-flight batches
    s->cv_done.notify_all();
    for (auto ev : s->ev_done) (void)hipEventDestroy(ev);
    for (auto ev : s->ev_proj) (void)hipEventDestroy(ev);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    (void)hipHostFree(s->pinned);
    (void)hipFree(s->slot_counters);
    (void)hipFree(s->arena_base);
    delete s;
    return D4DGS_OK;
}

}  // extern "C"
