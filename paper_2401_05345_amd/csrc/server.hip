// Serving runtime: resident scenes with Adam state on the device, and a
// continuous-batching scheduler that turns queued training-step requests
// into batched render + L1 + backward + Adam launches on a few lanes
// (stream + context each), so requests that arrive while others run are
// admitted as soon as a lane and memory free up and their work overlaps.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "gsr_internal.hpp"

using namespace gsr;

namespace {

using Clock = std::chrono::steady_clock;

struct Scene {
    bool alive = false;
    int64_t n = 0;
    int32_t sh_degree = 0;
    int64_t count = 0;      // floats per flat block
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int32_t step = 0;
    bool busy = false;      // a request of this scene is in flight
    int32_t queued = 0;     // requests waiting in the queue
    double pairs_per_px = 0.0; // last observed (tile, Gaussian) pairs per pixel
    double ppp_max = 0.0;      // largest pairs per pixel and largest pair count observed: pairs per pixel
    int64_t pairs_max = 0;     // hold across resolutions for large splats, the count for small ones
    void observe(int64_t pairs, double hw) {
        if (!(hw > 0)) return;
        pairs_per_px = (double)pairs / hw;
        ppp_max = std::max(ppp_max, pairs_per_px);
        pairs_max = std::max(pairs_max, pairs);
    }
    // Pair buffers of a capacity-mode render of this scene at hw pixels.
    int64_t capacity(double hw) const {
        return (int64_t)(1.5 * std::max(ppp_max * hw, (double)pairs_max)) + 65536;
    }
};

struct Pending {
    int64_t id;
    gsr_request req;
    double t_arrival;
    int64_t est_bytes = 0;
};

struct Batch {
    std::vector<Pending> reqs;
    std::vector<int32_t> steps;
    std::vector<Scene *> sc;          // each request's scene (the deque keeps them in place)
    std::vector<gsr_status> status;
    double t_start = 0.0;
};

struct Lane {
    int index = 0;
    hipStream_t stream = nullptr;
    gsr_ctx *ctx = nullptr;
    hipEvent_t done = nullptr;
    float *loss_host = nullptr;   // pinned, GSR_MAX_BATCH sums
    float *loss_dev = nullptr;
    uint32_t *counts_host = nullptr; // pinned, 4 words per view: a capacity-mode render's pairs, visible, overflow
    bool busy = false;
    bool has_batch = false;       // a batch handed over by the scheduler waits for this lane's thread
    Batch batch;
    std::thread waiter;           // runs the lane's batches and stamps their completion
};

template <typename T>
T *offset(T *base, int64_t floats) {
    return base ? base + floats : nullptr;
}

gsr_scene scene_view(const Scene &s, float *block) {
    gsr_scene v{};
    v.n = (int32_t)s.n;
    v.sh_degree = s.sh_degree;
    v.means3d = block;
    v.log_scales = offset(block, 3 * s.n);
    v.quats = offset(block, 6 * s.n);
    v.opacity_logits = offset(block, 10 * s.n);
    v.sh = offset(block, 11 * s.n);
    return v;
}

} // namespace

struct gsr_server {
    int device = 0;
    gsr_server_opts opts{};
    Clock::time_point t0;
    std::string err;
    std::mutex mu;
    std::condition_variable cv;       // scheduler: new work, free lane, stop
    std::condition_variable done_cv;  // drain / remove_scene waiters
    bool stop = false;
    std::deque<Scene> scenes;         // deque: references stay valid as scenes are added
    std::deque<Pending> queue;
    std::vector<gsr_result> results;
    std::vector<Lane *> lanes;
    int64_t next_id = 0, submitted = 0, completed = 0;
    int64_t resident_bytes = 0, inflight_bytes = 0;
    std::thread scheduler;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

gsr_status sfail(gsr_server *s, gsr_status st, const char *fmt, ...) {
    if (s) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = buf;
    }
    return st;
}

int64_t request_bytes(const Scene &sc, const gsr_camera &cam, bool capacity_render) {
    // image, target, dL/dimage, T_final, n_contrib per pixel; projected records, keys, ids,
    // offsets and accumulators per Gaussian; pair keys and ids (with their sort alternates)
    // per (tile, Gaussian) pair: the capacity a capacity-mode render will allocate, else the
    // scene's last pairs-per-pixel ratio.
    const int64_t hw = (int64_t)cam.width * cam.height;
    if (capacity_render && sc.pairs_per_px > 0.0) return 48 * hw + 160 * sc.n + 16 * sc.capacity((double)hw);
    const double ppp = sc.pairs_per_px > 0.0 ? sc.pairs_per_px : 4.0 * (double)sc.n / (double)(hw > 0 ? hw : 1);
    return 48 * hw + 160 * sc.n + 16 * (int64_t)(ppp * (double)hw);
}

// Runs one batch on a lane: everything is enqueued on the lane's stream. The render either
// synchronises once on it (pair counts), or - in capacity mode, when every scene of the batch has
// a pairs-per-pixel estimate - renders into pair buffers sized from that estimate with no host
// synchronisation at all, gating each scene's Adam update on its render's overflow word and
// queueing the read-back of its counts (checked after the batch). Returns whether the batch ran
// in capacity mode. Called by the lane's own thread without the lock, so the scheduler goes on
// admitting work for the other lanes meanwhile.
bool run_batch(gsr_server *S, Lane &L, Batch &b, std::vector<Scene *> &sc, bool allow_capacity) {
    const int k = (int)b.reqs.size();
    gsr_ctx *c = L.ctx;
    hipStream_t st = L.stream;
    gsr_scene scenes[kMaxViews];
    gsr_camera cams[kMaxViews];
    gsr_grads outs[kMaxViews];
    float *imgs[kMaxViews] = {}, *tgts[kMaxViews] = {}, *dls[kMaxViews] = {};
    gsr_fwd *states[kMaxViews] = {};
    std::vector<void *> bufs;
    gsr_status status = GSR_OK;
    const auto alloc = [&](float **p, size_t count) {
        void *q = nullptr;
        if (c->pool->alloc(&q, count * sizeof(float)) != hipSuccess) return false;
        bufs.push_back(q);
        *p = static_cast<float *>(q);
        return true;
    };
    for (int i = 0; i < k && status == GSR_OK; ++i) {
        const Scene &s = *sc[i];
        scenes[i] = scene_view(s, s.p);
        cams[i] = b.reqs[i].req.camera;
        const gsr_scene gv = scene_view(s, s.g);
        outs[i] = gsr_grads{const_cast<float *>(gv.means3d), const_cast<float *>(gv.log_scales),
                            const_cast<float *>(gv.quats), const_cast<float *>(gv.opacity_logits),
                            const_cast<float *>(gv.sh)};
        const size_t n3 = 3 * (size_t)cams[i].width * cams[i].height;
        if (!alloc(&imgs[i], n3) || !alloc(&tgts[i], n3) || !alloc(&dls[i], n3)) status = GSR_ENOMEM;
        else if (launch_uniform(tgts[i], (int64_t)n3, b.reqs[i].req.target_seed, st) != hipSuccess) status = GSR_EHIP;
    }
    if (status == GSR_OK && launch_fill_u32(reinterpret_cast<uint32_t *>(L.loss_dev), 0u, kMaxViews, st) != hipSuccess)
        status = GSR_EHIP;
    bool capacity = allow_capacity && S->opts.capacity_render != 0;
    int64_t caps[kMaxViews] = {};
    for (int i = 0; i < k; ++i) {
        // The scene's pairs per pixel from its last render (written only by the lane that runs
        // its request, and read by the scheduler only while the scene is idle).
        if (!(sc[i]->pairs_per_px > 0.0)) capacity = false;
        caps[i] = sc[i]->capacity((double)cams[i].width * (double)cams[i].height);
    }
    if (status == GSR_OK && capacity) {
        status = render_batch_capacity(c, k, scenes, cams, &S->opts.config, imgs, caps, states);
        // capacities that do not fit in device memory: the batch reads its counts back instead
        if (status == GSR_ENOMEM) {
            capacity = false;
            status = GSR_OK;
        }
    }
    if (status == GSR_OK && !capacity) status = gsr_render_batch(c, k, scenes, cams, &S->opts.config, imgs, states);
    for (int i = 0; i < k && status == GSR_OK; ++i) {
        const int64_t n3 = 3 * (int64_t)cams[i].width * cams[i].height;
        if (launch_l1_sum(imgs[i], tgts[i], n3, L.loss_dev + i, st) != hipSuccess) status = GSR_EHIP;
        else status = gsr_l1_grad(c, imgs[i], tgts[i], n3, dls[i]);
    }
    if (status == GSR_OK)
        status = gsr_backward_batch(c, k, states, dls, outs, 0, &S->opts.config);
    for (int i = 0; i < k && status == GSR_OK; ++i) {
        Scene &s = *sc[i];
        // an overflowed capacity-mode render gives no update (the step runs again)
        if (launch_adam(s.p, s.g, s.m, s.v, s.count, S->opts.lr, S->opts.beta1, S->opts.beta2, S->opts.eps,
                        b.steps[i], st, capacity ? states[i]->totals + 2 : nullptr) != hipSuccess)
            status = GSR_EHIP;
    }
    if (status == GSR_OK &&
        hipMemcpyAsync(L.loss_host, L.loss_dev, k * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
        status = GSR_EHIP;
    for (int i = 0; i < k && status == GSR_OK && capacity; ++i)
        if (hipMemcpyAsync(L.counts_host + 4 * i, states[i]->totals, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           st) != hipSuccess)
            status = GSR_EHIP;
    for (int i = 0; i < k; ++i) {
        if (states[i]) {
            const double hw = (double)cams[i].width * cams[i].height;
            gsr_fwd_stats_t fs{};
            if (!capacity && gsr_fwd_stats(states[i], &fs) == GSR_OK) sc[i]->observe(fs.n_pairs, hw);
            gsr_fwd_release(c, states[i]);
        }
    }
    // The lane's pool hands these buffers only to later work on the same stream.
    for (void *q : bufs) c->pool->release(q);
    if (status != GSR_OK) {
        (void)hipStreamSynchronize(st);
        std::lock_guard<std::mutex> lk(S->mu);
        S->err = c->err;
    }
    for (auto &x : b.status) x = status;
    (void)hipEventRecord(L.done, st);
    return capacity && status == GSR_OK;
}

void scheduler_main(gsr_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        Lane *lane = nullptr;
        Batch b;
        // A request fits if its footprint fits beside the resident scenes and the requests in
        // flight; one that fits nowhere still runs when nothing else is in flight.
        const auto fits = [&](int64_t est, int64_t batch_bytes) {
            const int64_t used = S->resident_bytes + S->inflight_bytes + batch_bytes;
            return used + est <= S->opts.hbm_budget_bytes || (S->inflight_bytes + batch_bytes == 0);
        };
        S->cv.wait(lk, [&] {
            if (S->stop && S->queue.empty()) return true;
            lane = nullptr;
            for (Lane *l : S->lanes)
                if (!l->busy) {
                    lane = l;
                    break;
                }
            if (!lane) return false;
            // The admission scan below starts from the first request whose scene is idle.
            for (const Pending &p : S->queue) {
                const Scene &s = S->scenes[p.req.scene];
                if (!s.busy) return fits(request_bytes(s, p.req.camera, S->opts.capacity_render != 0), 0);
            }
            return false;
        });
        if (S->stop && S->queue.empty()) break;
        // Admission: FIFO scan; a request joins if its scene has nothing in flight (nor an
        // earlier request in this batch) and its footprint fits; the scan stops at the first
        // request that does not fit, so large requests are not starved.
        int64_t batch_bytes = 0;
        for (auto it = S->queue.begin(); it != S->queue.end() && (int)b.reqs.size() < S->opts.max_batch;) {
            Scene &s = S->scenes[it->req.scene];
            if (s.busy) {
                ++it;
                continue;
            }
            const int64_t est = request_bytes(s, it->req.camera, S->opts.capacity_render != 0);
            if (!fits(est, batch_bytes)) break;
            batch_bytes += est;
            it->est_bytes = est;
            s.busy = true;
            s.queued -= 1;
            s.step += 1;
            b.reqs.push_back(*it);
            b.steps.push_back(s.step);
            b.sc.push_back(&s);
            it = S->queue.erase(it);
        }
        if (b.reqs.empty()) continue;
        S->inflight_bytes += batch_bytes;
        lane->busy = true;
        b.status.assign(b.reqs.size(), GSR_OK);
        b.t_start = S->now();
        lane->batch = std::move(b);
        lane->has_batch = true;
        S->cv.notify_all();
    }
}

void lane_main(gsr_server *S, Lane *L) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        S->cv.wait(lk, [&] { return L->has_batch || (S->stop && !L->busy); });
        if (!L->has_batch) break;
        Batch &b = L->batch;
        const hipEvent_t ev = L->done;
        lk.unlock();
        const bool capacity = run_batch(S, *L, b, b.sc, true);
        (void)hipEventSynchronize(ev);
        const size_t k = b.reqs.size();
        std::vector<float> loss(L->loss_host, L->loss_host + k);
        std::vector<int32_t> mode(k, capacity ? 1 : 0);
        if (capacity) {
            // Counts of the capacity-mode renders: pairs-per-pixel estimates for the next ones, and
            // the requests whose pairs overflowed (their Adam update was skipped) run again, exactly.
            Batch again;
            std::vector<size_t> where;
            for (size_t i = 0; i < k; ++i) {
                const uint32_t *h = L->counts_host + 4 * i;
                const gsr_camera &cam = b.reqs[i].req.camera;
                const double hw = (double)cam.width * cam.height;
                b.sc[i]->observe((int64_t)h[0], hw); // the full count, also when it overflowed
                if (h[2] == 0u) continue;
                again.reqs.push_back(b.reqs[i]);
                again.steps.push_back(b.steps[i]);
                again.sc.push_back(b.sc[i]);
                where.push_back(i);
            }
            if (!where.empty()) {
                again.status.assign(where.size(), GSR_OK);
                run_batch(S, *L, again, again.sc, false);
                (void)hipEventSynchronize(ev);
                for (size_t j = 0; j < where.size(); ++j) {
                    b.status[where[j]] = again.status[j];
                    loss[where[j]] = L->loss_host[j];
                    mode[where[j]] = 2;
                }
            }
        }
        const double t_done = S->now();
        lk.lock();
        for (size_t i = 0; i < b.reqs.size(); ++i) {
            const Pending &p = b.reqs[i];
            const gsr_camera &cam = p.req.camera;
            gsr_result r{};
            r.id = p.id;
            r.scene = p.req.scene;
            r.status = b.status[i];
            r.batch_size = (int32_t)b.reqs.size();
            r.lane = L->index;
            r.step = b.steps[i];
            r.loss = b.status[i] == GSR_OK ? loss[i] / (3.0f * (float)cam.width * (float)cam.height) : -1.0f;
            r.render_mode = mode[i];
            r.t_arrival = p.t_arrival;
            r.t_start = b.t_start;
            r.t_done = t_done;
            S->results.push_back(r);
            S->scenes[p.req.scene].busy = false;
            S->inflight_bytes -= p.est_bytes;
            S->completed += 1;
        }
        b = Batch{};
        L->has_batch = false;
        L->busy = false;
        S->cv.notify_all();
        S->done_cv.notify_all();
    }
}

void destroy_lane(Lane *L) {
    if (L->ctx) gsr_ctx_destroy(L->ctx);
    if (L->loss_dev) (void)hipFree(L->loss_dev);
    if (L->loss_host) (void)hipHostFree(L->loss_host);
    if (L->counts_host) (void)hipHostFree(L->counts_host);
    if (L->done) (void)hipEventDestroy(L->done);
    if (L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

bool valid_opts(const gsr_server_opts *o) {
    if (!o) return false;
    if (o->max_batch < 1 || o->max_batch > GSR_MAX_BATCH || o->lanes < 1 || o->lanes > 4) return false;
    if (o->hbm_budget_bytes <= 0) return false;
    if (o->capacity_render != 0 && o->capacity_render != 1) return false;
    if (gsr_validate_config(&o->config, nullptr) != GSR_OK) return false;
    if (!(o->lr > 0.0f) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) || !(o->beta2 >= 0.0f && o->beta2 < 1.0f) ||
        !(o->eps >= 0.0f))
        return false;
    return true;
}

} // namespace

extern "C" {

int64_t gsr_server_scene_bytes(int64_t n, int32_t sh_degree) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3) return -1;
    const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
    return 4 * n * (11 + 3 * K) * (int64_t)sizeof(float);
}

gsr_status gsr_server_create(int device, const gsr_server_opts *opts, gsr_server **out) {
    if (!out) return GSR_EINVAL;
    *out = nullptr;
    if (!valid_opts(opts)) return GSR_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GSR_EHIP;
    if (device < 0 || device >= count) return GSR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return GSR_EHIP;
    gsr_server *S = new (std::nothrow) gsr_server();
    if (!S) return GSR_ENOMEM;
    S->device = device;
    S->opts = *opts;
    S->t0 = Clock::now();
    for (int i = 0; i < opts->lanes; ++i) {
        Lane *L = new (std::nothrow) Lane();
        bool ok = L != nullptr;
        if (ok) {
            L->index = i;
            void *hp = nullptr, *hc = nullptr;
            ok = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&L->done, hipEventDisableTiming) == hipSuccess &&
                 hipHostMalloc(&hp, kMaxViews * sizeof(float), hipHostMallocDefault) == hipSuccess &&
                 hipHostMalloc(&hc, 4 * kMaxViews * sizeof(uint32_t), hipHostMallocDefault) == hipSuccess &&
                 hipMalloc(reinterpret_cast<void **>(&L->loss_dev), kMaxViews * sizeof(float)) == hipSuccess;
            L->loss_host = static_cast<float *>(hp);
            L->counts_host = static_cast<uint32_t *>(hc);
            ok = ok && gsr_ctx_create(&L->ctx, device, L->stream) == GSR_OK;
        }
        if (!ok) {
            if (L) destroy_lane(L);
            for (Lane *l : S->lanes) destroy_lane(l);
            delete S;
            return GSR_EHIP;
        }
        S->lanes.push_back(L);
    }
    for (Lane *L : S->lanes) L->waiter = std::thread(lane_main, S, L);
    S->scheduler = std::thread(scheduler_main, S);
    *out = S;
    return GSR_OK;
}

void gsr_server_destroy(gsr_server *S) {
    if (!S) return;
    gsr_server_drain(S);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->scheduler.joinable()) S->scheduler.join();
    for (Lane *L : S->lanes)
        if (L->waiter.joinable()) L->waiter.join();
    (void)hipSetDevice(S->device);
    for (Lane *L : S->lanes) destroy_lane(L);
    for (Scene &s : S->scenes) {
        if (!s.alive) continue;
        (void)hipFree(s.p);
        (void)hipFree(s.g);
        (void)hipFree(s.m);
        (void)hipFree(s.v);
    }
    delete S;
}

const char *gsr_server_last_error(const gsr_server *S) { return S ? S->err.c_str() : "null server"; }

double gsr_server_now(const gsr_server *S) { return S ? S->now() : 0.0; }

gsr_status gsr_server_add_scene(gsr_server *S, const gsr_scene *init, int32_t *scene_id) {
    if (!S || !scene_id) return GSR_EINVAL;
    if (!init || init->n < 0 || init->sh_degree < 0 || init->sh_degree > 3)
        return sfail(S, GSR_EINVAL, "invalid scene");
    const int64_t bytes = gsr_server_scene_bytes(init->n, init->sh_degree);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->resident_bytes + bytes > S->opts.hbm_budget_bytes) {
            S->err = "scene does not fit the HBM budget";
            return GSR_EBUDGET;
        }
        S->resident_bytes += bytes; // reserved while the copies run
    }
    Scene s;
    s.alive = true;
    s.n = init->n;
    s.sh_degree = init->sh_degree;
    const int64_t K = (int64_t)(s.sh_degree + 1) * (s.sh_degree + 1);
    s.count = s.n * (11 + 3 * K);
    const size_t blk = (size_t)(s.count > 0 ? s.count : 1) * sizeof(float);
    hipError_t e = hipSetDevice(S->device);
    float **blocks[4] = {&s.p, &s.g, &s.m, &s.v};
    for (float **b : blocks)
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(b), blk);
    for (float **b : blocks)
        if (e == hipSuccess) e = hipMemset(*b, 0, blk);
    if (e == hipSuccess) {
        const int64_t seg[5] = {0, 3 * s.n, 6 * s.n, 10 * s.n, 11 * s.n};
        const int64_t len[5] = {3 * s.n, 3 * s.n, 4 * s.n, s.n, 3 * K * s.n};
        const float *src[5] = {init->means3d, init->log_scales, init->quats, init->opacity_logits, init->sh};
        for (int j = 0; j < 5 && e == hipSuccess; ++j)
            if (src[j] && len[j] > 0)
                e = hipMemcpy(s.p + seg[j], src[j], len[j] * sizeof(float), hipMemcpyDeviceToDevice);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (e != hipSuccess) {
        for (float **b : blocks)
            if (*b) (void)hipFree(*b);
        S->resident_bytes -= bytes;
        S->err = std::string("scene upload failed: ") + hipGetErrorString(e);
        return GSR_EHIP;
    }
    S->scenes.push_back(s);
    *scene_id = (int32_t)S->scenes.size() - 1;
    return GSR_OK;
}

gsr_status gsr_server_remove_scene(gsr_server *S, int32_t id) {
    if (!S) return GSR_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (id < 0 || id >= (int32_t)S->scenes.size() || !S->scenes[id].alive) {
        S->err = "unknown scene";
        return GSR_EINVAL;
    }
    S->done_cv.wait(lk, [&] { return S->scenes[id].queued == 0 && !S->scenes[id].busy; });
    Scene &s = S->scenes[id];
    s.alive = false;
    S->resident_bytes -= gsr_server_scene_bytes(s.n, s.sh_degree);
    float *b[4] = {s.p, s.g, s.m, s.v};
    s.p = s.g = s.m = s.v = nullptr;
    lk.unlock();
    (void)hipSetDevice(S->device);
    for (float *q : b) (void)hipFree(q);
    S->cv.notify_all();
    return GSR_OK;
}

gsr_status gsr_server_scene_state(gsr_server *S, int32_t id, gsr_scene *params, gsr_grads *grads, float **adam_m,
                                  float **adam_v, int32_t *step) {
    if (!S) return GSR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (id < 0 || id >= (int32_t)S->scenes.size() || !S->scenes[id].alive) {
        S->err = "unknown scene";
        return GSR_EINVAL;
    }
    const Scene &s = S->scenes[id];
    if (params) *params = scene_view(s, s.p);
    if (grads) {
        const gsr_scene gv = scene_view(s, s.g);
        *grads = gsr_grads{const_cast<float *>(gv.means3d), const_cast<float *>(gv.log_scales),
                           const_cast<float *>(gv.quats), const_cast<float *>(gv.opacity_logits),
                           const_cast<float *>(gv.sh)};
    }
    if (adam_m) *adam_m = s.m;
    if (adam_v) *adam_v = s.v;
    if (step) *step = s.step;
    return GSR_OK;
}

gsr_status gsr_server_set_step(gsr_server *S, int32_t id, int32_t step) {
    if (!S) return GSR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (id < 0 || id >= (int32_t)S->scenes.size() || !S->scenes[id].alive || step < 0) {
        S->err = "unknown scene or negative step";
        return GSR_EINVAL;
    }
    if (S->scenes[id].busy || S->scenes[id].queued) {
        S->err = "scene has requests queued or in flight";
        return GSR_ESTATE;
    }
    S->scenes[id].step = step;
    return GSR_OK;
}

gsr_status gsr_server_scene_io(gsr_server *S, int32_t id, int32_t block, float *host, int32_t to_host) {
    if (!S) return GSR_EINVAL;
    if (!host || block < 0 || block > 3) return sfail(S, GSR_EINVAL, "bad block or null host buffer");
    float *src = nullptr;
    int64_t count = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (id < 0 || id >= (int32_t)S->scenes.size() || !S->scenes[id].alive) {
            S->err = "unknown scene";
            return GSR_EINVAL;
        }
        const Scene &s = S->scenes[id];
        if (s.busy || s.queued) {
            S->err = "scene has requests queued or in flight";
            return GSR_ESTATE;
        }
        float *const b[4] = {s.p, s.g, s.m, s.v};
        src = b[block];
        count = s.count;
    }
    if (count == 0) return GSR_OK;
    hipError_t e = hipSetDevice(S->device);
    if (e == hipSuccess)
        e = to_host ? hipMemcpy(host, src, count * sizeof(float), hipMemcpyDeviceToHost)
                    : hipMemcpy(src, host, count * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return sfail(S, GSR_EHIP, "scene copy failed: %s", hipGetErrorString(e));
    return GSR_OK;
}

gsr_status gsr_server_submit(gsr_server *S, const gsr_request *req, int64_t *id) {
    if (!S || !req) return GSR_EINVAL;
    if (gsr_validate_camera(&req->camera) != GSR_OK) return sfail(S, GSR_EINVAL, "invalid camera");
    if (gsr_validate_config(&S->opts.config, &req->camera) != GSR_OK)
        return sfail(S, GSR_EINVAL, "camera too large for the server's tile size");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        S->err = "server is stopping";
        return GSR_ESTATE;
    }
    if (req->scene < 0 || req->scene >= (int32_t)S->scenes.size() || !S->scenes[req->scene].alive) {
        S->err = "unknown scene";
        return GSR_EINVAL;
    }
    Pending p;
    p.id = S->next_id++;
    p.req = *req;
    p.t_arrival = S->now();
    S->queue.push_back(p);
    S->scenes[req->scene].queued += 1;
    S->submitted += 1;
    if (id) *id = p.id;
    S->cv.notify_all();
    return GSR_OK;
}

gsr_status gsr_server_replay(gsr_server *S, int32_t n, const gsr_request *reqs, const double *arrival_s,
                             int64_t *ids) {
    if (!S || n < 0 || (n > 0 && (!reqs || !arrival_s))) return GSR_EINVAL;
    for (int i = 1; i < n; ++i)
        if (arrival_s[i] < arrival_s[i - 1]) return sfail(S, GSR_EINVAL, "arrival times must ascend");
    const Clock::time_point start = Clock::now();
    for (int i = 0; i < n; ++i) {
        const auto due = start + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
        // Sleep to within 200 us of the arrival, then spin.
        const auto coarse = due - std::chrono::microseconds(200);
        if (Clock::now() < coarse) std::this_thread::sleep_until(coarse);
        while (Clock::now() < due) {
        }
        int64_t id = -1;
        const gsr_status st = gsr_server_submit(S, &reqs[i], &id);
        if (st != GSR_OK) return st;
        if (ids) ids[i] = id;
    }
    return GSR_OK;
}

gsr_status gsr_server_drain(gsr_server *S) {
    if (!S) return GSR_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] { return S->completed == S->submitted; });
    return GSR_OK;
}

gsr_status gsr_server_results(gsr_server *S, gsr_result *out, int32_t max, int32_t *n) {
    if (!S || !n || max < 0 || (max > 0 && !out)) return GSR_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)max, S->results.size());
    for (int32_t i = 0; i < k; ++i) out[i] = S->results[i];
    S->results.erase(S->results.begin(), S->results.begin() + k);
    *n = k;
    return GSR_OK;
}

} // extern "C"
