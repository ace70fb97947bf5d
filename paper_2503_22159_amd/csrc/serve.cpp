// Continuous-batching render server (d4dgs_serve_*).
//
// One resident scene; requests (camera, t, resolution) arrive from any thread.  A
// scheduler thread
//   1. retires finished batches (event query), frees their scratch, retries requests
//      whose tile instances overflowed their capacity (with twice the capacity);
//   2. admits waiting requests in arrival order while fewer than max_inflight are on the
//      GPU and their scratch fits the free part of the arena (first-fit allocator over
//      one device reservation of scratch_budget_bytes);
//   3. launches the admitted group as one batch on the next of n_streams streams: one
//      projection launch over (request x Gaussian) -- each Gaussian's parameters are
//      read once for the whole batch -- then binning/sort and blending per request.
// Requests arriving while earlier batches run are admitted as slots and memory free up;
// their batches overlap on the other streams.  Every kernel a request runs is the one a
// single-request render runs, with the same inputs, so its image is bitwise the same
// alone or in any mix.
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
    int slot = -1;  // pinned status slot
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

struct Batch {
    std::vector<Req *> reqs;
    hipEvent_t ev = nullptr;
    int stream = 0;
};

}  // namespace

struct d4dgs_server {
    d4dgs_scene scene{};
    SceneK sk{};
    d4dgs_serve_config cfg{};
    char *arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    int device = 0;
    // pinned status words, one per in-flight slot: {num_instances (int64), status}
    int64_t *pinned = nullptr;
    std::vector<int> free_slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::vector<Batch> inflight;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    int inflight_reqs = 0;
    bool stop = false;
    std::thread th;
    d4dgs_serve_stats stats{};
    int64_t last_activity_ns = 0;  // last launch or retirement (for the polling policy)

    void run();
    bool retire_one(Batch &b);
    void launch(Batch &b);
    void finish(Req *r, int status);
};

void d4dgs_server::finish(Req *r, int status) {
    r->st.status = status;
    r->st.done_ns = now_ns();
    r->done = true;
    if (r->bytes) arena->release(r->off, r->bytes);
    r->bytes = 0;
    if (r->slot >= 0) free_slots.push_back(r->slot);
    r->slot = -1;
    stats.completed++;
}

void d4dgs_server::launch(Batch &b) {
    const int si = next_stream;
    next_stream = (next_stream + 1) % (int)streams.size();
    b.stream = si;
    hipStream_t st = streams[si];
    hipError_t e = hipSuccess;
    const int64_t t_start = now_ns();
    // batched projection, kMaxBatch requests per launch
    for (size_t i0 = 0; i0 < b.reqs.size() && e == hipSuccess; i0 += kMaxBatch) {
        BatchArgs a{};
        a.nreq = (int)std::min<size_t>(kMaxBatch, b.reqs.size() - i0);
        for (int j = 0; j < a.nreq; ++j) {
            Req *r = b.reqs[i0 + j];
            const Layout L = layout(scene.n, r->cam.width, r->cam.height, r->capacity);
            char *base = arena_base + r->off;
            a.r[j].cam = make_camk(r->cam);
            a.r[j].t = r->t;
            a.r[j].rec = (float4 *)(base + L.rec);
            a.r[j].count = (uint32_t *)(base + L.count);
            a.r[j].partial = (uint32_t *)(base + L.partial);
        }
        e = launch_project_batch(sk, a, st);
    }
    for (Req *r : b.reqs) {
        if (e != hipSuccess) break;
        r->st.start_ns = t_start;
        r->st.batch_size = (int)b.reqs.size();
        const Layout L = layout(scene.n, r->cam.width, r->cam.height, r->capacity);
        char *base = arena_base + r->off;
        const CamK ck = make_camk(r->cam);
        const SortWs ws = carve_workspace(base + L.ws, scene.n, r->capacity, ck.TX * ck.TY);
        e = launch_bin_sort((const float4 *)(base + L.rec), (const uint32_t *)(base + L.count),
                            (uint32_t *)(base + L.offset), (uint32_t *)(base + L.partial), scene.n, ck, ws,
                            (uint64_t *)(base + L.keys), (uint32_t *)(base + L.vals), (uint32_t *)(base + L.ranges),
                            (int64_t *)(base + L.ninst), r->capacity, nullptr, (uint32_t *)(base + L.order), st);
        if (e == hipSuccess)
            e = launch_blend((const float4 *)(base + L.rec), (const uint32_t *)(base + L.vals),
                             (const uint32_t *)(base + L.ranges), (const uint32_t *)(base + L.order), ck, cfg.bg,
                             r->out, nullptr, nullptr, st);
        if (e == hipSuccess)  // instance total and overflow status back to pinned memory
            e = hipMemcpyAsync(pinned + 2 * r->slot, base + L.ninst, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pinned + 2 * r->slot + 1, ws.misc + 1, 4, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b.ev, st);
    if (e != hipSuccess) {
        set_error(std::string("serve launch: ") + hipGetErrorString(e));
        (void)hipStreamSynchronize(st);
        if (b.ev) (void)hipEventDestroy(b.ev);
        b.ev = nullptr;
        for (Req *r : b.reqs) {
            inflight_reqs--;
            finish(r, D4DGS_ERR_HIP);
        }
        b.reqs.clear();
        cv_done.notify_all();
    }
    stats.batches++;
}

// Returns true if the batch finished (and was retired).
bool d4dgs_server::retire_one(Batch &b) {
    if (b.reqs.empty()) return true;
    const hipError_t q = hipEventQuery(b.ev);
    if (q == hipErrorNotReady) return false;
    (void)hipEventDestroy(b.ev);
    if (q != hipSuccess) {  // the batch's work failed: its requests end with the error
        set_error(std::string("serve batch: ") + hipGetErrorString(q));
        for (Req *r : b.reqs) {
            inflight_reqs--;
            finish(r, D4DGS_ERR_HIP);
        }
        return true;
    }
    for (Req *r : b.reqs) {
        const int64_t ninst = pinned[2 * r->slot];
        const uint32_t status = (uint32_t)(pinned[2 * r->slot + 1] & 0xffffffff);
        r->st.num_instances = ninst;
        inflight_reqs--;
        if (status == (uint32_t)D4DGS_ERR_CAPACITY && ninst > kMaxCapacity) {
            // more instances than any bins can hold (capacities stay below 2^31)
            set_error("serve: request has " + std::to_string(ninst) + " tile instances, above 2^31 - 1");
            finish(r, D4DGS_ERR_CAPACITY);
        } else if (status == (uint32_t)D4DGS_ERR_CAPACITY) {
            // retry with room for every instance (rounded up), as a new admission
            arena->release(r->off, r->bytes);
            r->bytes = 0;
            free_slots.push_back(r->slot);
            r->slot = -1;
            r->capacity = std::min<int64_t>(std::max<int64_t>(2 * r->capacity, ninst + ninst / 4 + 1024), kMaxCapacity);
            r->retries++;
            stats.retried++;
            pending.push_front(r);
        } else {
            finish(r, D4DGS_OK);
        }
    }
    return true;
}

void d4dgs_server::run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // 1. retire finished batches
        bool retired = false;
        for (size_t i = 0; i < inflight.size();) {
            if (retire_one(inflight[i])) {
                inflight.erase(inflight.begin() + i);
                retired = true;
            } else {
                ++i;
            }
        }
        if (retired) {
            last_activity_ns = now_ns();
            cv_done.notify_all();
        }
        // 2. admit waiting requests, oldest first
        Batch b;
        while (!pending.empty() && inflight_reqs < cfg.max_inflight && (int)b.reqs.size() < cfg.max_batch &&
               !free_slots.empty()) {
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
            inflight_reqs++;
            b.reqs.push_back(r);
        }
        if (!b.reqs.empty()) {
            launch(b);
            if (!b.reqs.empty()) inflight.push_back(b);
            last_activity_ns = now_ns();
            continue;
        }
        if (stop && pending.empty() && inflight.empty()) break;
        if (!inflight.empty()) {
            // poll the GPU.  Within kSpinNs of the last launch or retirement (a frame takes
            // ~0.1-0.5 ms) the thread spins, yielding the CPU between queries, so a
            // completion is seen within microseconds (a 20 us sleep takes 60-80 us on
            // Linux: timer slack); after that, short sleeps.
            constexpr int64_t kSpinNs = 2000000;
            const bool spin = now_ns() - last_activity_ns < kSpinNs;
            lk.unlock();
            if (spin)
                std::this_thread::yield();
            else
                std::this_thread::sleep_for(std::chrono::microseconds(20));
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
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->pinned, sizeof(int64_t) * 2 * cfg->max_inflight, 0);
    if (e != hipSuccess) {
        for (auto st : s->streams) (void)hipStreamDestroy(st);
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
                                                 s->cfg.max_instances_per_pixel_x1000 / 1000);
    r->capacity = std::min<int64_t>(r->capacity, kMaxCapacity);
    r->st.submit_ns = now_ns();
    r->st.status = -1;
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->stats.submitted++;
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
    const bool ok = s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [s, ticket] {
        auto f = s->reqs.find(ticket);
        return f == s->reqs.end() || f->second->done;
    });
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
    st->inflight = s->inflight_reqs;
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
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    (void)hipHostFree(s->pinned);
    (void)hipFree(s->arena_base);
    delete s;
    return D4DGS_OK;
}

}  // extern "C"
