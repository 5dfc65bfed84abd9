// Host runtime of libgsr: the C ABI of gsr.h, argument checks, a caching
// device-memory pool, and the orchestration of the kernels on the context's
// stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gsr_internal.hpp"

using namespace gsr;

namespace gsr {

Pool::~Pool() {
    for (auto &kv : free_) (void)hipFree(kv.second);
    for (auto &kv : live_) (void)hipFree(kv.first);
}

hipError_t Pool::alloc(void **p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.lower_bound(bytes);
    if (it != free_.end() && it->first <= 2 * bytes + (1u << 20)) {
        *p = it->second;
        live_[it->second] = it->first;
        free_.erase(it);
        return hipSuccess;
    }
    // Large requests get some headroom so a slightly larger one later reuses them.
    size_t cap = bytes >= (64u << 20) ? bytes + bytes / 8 : bytes;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, cap);
    if (e != hipSuccess) {
        // Drop cached blocks and retry once.
        for (auto &kv : free_) {
            (void)hipFree(kv.second);
            reserved_ -= kv.first;
        }
        free_.clear();
        (void)hipGetLastError();
        e = hipMalloc(&q, cap);
        if (e != hipSuccess) return e;
    }
    reserved_ += cap;
    live_[q] = cap;
    *p = q;
    return hipSuccess;
}

void Pool::release(void *p) {
    if (!p) return;
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_.emplace(it->second, p);
    live_.erase(it);
}

DevCamera make_dev_camera(const gsr_camera &c, int tile) {
    DevCamera d{};
    d.width = c.width;
    d.height = c.height;
    d.tile = tile;
    d.grid_x = (c.width + tile - 1) / tile;
    d.grid_y = (c.height + tile - 1) / tile;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.world_to_cam[4 * r + k];
        d.t[r] = c.world_to_cam[4 * r + 3];
    }
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int r = 0; r < 3; ++r) s += (double)d.R[3 * r + k] * (double)d.t[r];
        d.centre[k] = (float)(-s);
    }
    d.znear = c.znear;
    // Guard band of the projection Jacobian: the image extended by 15 % of its size on each side
    // (3DGS's +-1.3 * half-extent / focal when the principal point is at the centre).
    d.lox = (-c.cx - 0.15f * (float)c.width) / c.fx;
    d.hix = ((float)c.width - c.cx + 0.15f * (float)c.width) / c.fx;
    d.loy = (-c.cy - 0.15f * (float)c.height) / c.fy;
    d.hiy = ((float)c.height - c.cy + 0.15f * (float)c.height) / c.fy;
    for (int k = 0; k < 3; ++k) d.bg[k] = c.bg[k];
    return d;
}

} // namespace gsr

namespace {

gsr_status fail(gsr_ctx *ctx, gsr_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define GSR_HIP(ctx, expr)                                                                                          \
    do {                                                                                                            \
        hipError_t e_ = (expr);                                                                                     \
        if (e_ != hipSuccess) return fail(ctx, GSR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
    } while (0)

bool finite(float x) { return std::isfinite(x); }

template <typename T>
gsr_status pool_alloc(gsr_ctx *ctx, gsr_fwd *st, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = ctx->pool->alloc(&q, count * sizeof(T));
    if (e != hipSuccess) return fail(ctx, GSR_ENOMEM, "device allocation of %zu bytes failed: %s", count * sizeof(T),
                                     hipGetErrorString(e));
    if (st) st->owned.push_back(q);
    *p = static_cast<T *>(q);
    return GSR_OK;
}

#define GSR_TRY(x)                                                                                                  \
    do {                                                                                                            \
        gsr_status s_ = (x);                                                                                        \
        if (s_ != GSR_OK) return s_;                                                                                \
    } while (0)

int bits_for(int64_t count) {
    int b = 0;
    while ((int64_t(1) << b) < count) ++b;
    return b;
}

enum { EV_R0 = 0, EV_R1, EV_R2, EV_R3, EV_R4, EV_R5, EV_R6, EV_B0, EV_B1, EV_B2, EV_B3 };

void mark(gsr_ctx *ctx, bool on, int ev) {
    if (on) (void)hipEventRecord(ctx->ev[ev], ctx->stream);
}

} // namespace

// Fixed scratch of the allocation-free backward: the accumulator rows, then the tile order.
// Every GPU holds its own copy at its own address; host code uses only that address (the
// array's name is a host-side stand-in), taken once per device at context creation.
constexpr size_t kNoallocRowBytes = size_t(GSR_NOALLOC_MAX_GAUSSIANS) * GSR_ACC_STRIDE * sizeof(double);
constexpr size_t kNoallocOrderBytes = size_t(GSR_NOALLOC_MAX_TILES) * sizeof(uint2);
static __device__ __align__(256) unsigned char scratch[kNoallocRowBytes + kNoallocOrderBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// With ctx->device current: this device's scratch address, looked up on its first context.
void scratch_init(gsr_ctx *ctx) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= kMaxDevices) {
        ctx->scratch_err = hipErrorInvalidDevice;
        return;
    }
    if (!g_scratch_ptr[ctx->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            ctx->scratch_err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            (void)hipGetLastError();
            return;
        }
        g_scratch_ptr[ctx->device] = p;
    }
    ctx->scratch = g_scratch_ptr[ctx->device];
}

} // namespace

extern "C" {

const char *gsr_version(void) { return "gsr 0.1 gfx950"; }

gsr_status gsr_validate_scene(const gsr_scene *s) {
    if (!s) return GSR_EINVAL;
    if (s->n < 0 || s->sh_degree < 0 || s->sh_degree > 3) return GSR_EINVAL;
    if (s->n > 0 && (!s->means3d || !s->log_scales || !s->quats || !s->opacity_logits || !s->sh)) return GSR_EINVAL;
    return GSR_OK;
}

gsr_status gsr_validate_camera(const gsr_camera *c) {
    if (!c) return GSR_EINVAL;
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384) return GSR_EINVAL;
    if (!finite(c->fx) || !finite(c->fy) || !finite(c->cx) || !finite(c->cy) || !(c->fx > 0) || !(c->fy > 0))
        return GSR_EINVAL;
    for (int i = 0; i < 12; ++i)
        if (!finite(c->world_to_cam[i])) return GSR_EINVAL;
    // Rows of R must be orthonormal (the projection Jacobian assumes a rotation).
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            double d = 0.0;
            for (int k = 0; k < 3; ++k) d += (double)c->world_to_cam[4 * r + k] * c->world_to_cam[4 * q + k];
            if (std::fabs(d - (r == q ? 1.0 : 0.0)) > 1e-4) return GSR_EINVAL;
        }
    if (!finite(c->znear) || !(c->znear > 0)) return GSR_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!finite(c->bg[k])) return GSR_EINVAL;
    return GSR_OK;
}

gsr_status gsr_validate_config(const gsr_config *cf, const gsr_camera *c) {
    if (!cf) return GSR_EINVAL;
    if (cf->tile != 8 && cf->tile != 16 && cf->tile != 32) return GSR_EINVAL;
    if (cf->lds_batch != 64 && cf->lds_batch != 128 && cf->lds_batch != 256) return GSR_EINVAL;
    if (cf->lds_batch > cf->tile * cf->tile) return GSR_EINVAL;
    if (cf->bwd_mode < GSR_BWD_PLAIN_ATOMIC || cf->bwd_mode > GSR_BWD_PLAIN_COMPILER_REDUCE) return GSR_EINVAL;
    // The compiler-reduced kernel is built without the counting instrumentation.
    if (cf->bwd_mode == GSR_BWD_PLAIN_COMPILER_REDUCE && (cf->flags & GSR_FLAG_DEBUG_COUNTERS)) return GSR_EINVAL;
    if (cf->reduce_threshold < 0 || cf->reduce_threshold > 65) return GSR_EINVAL;
    if (cf->flags & ~(GSR_FLAG_DEBUG_COUNTERS | GSR_FLAG_XCD_REMAP | GSR_FLAG_STAGE_TIMING |
                      GSR_FLAG_LANE_SPLIT_ATOMICS | GSR_FLAG_NO_TILE_ORDER | GSR_FLAG_ACC_F32))
        return GSR_EINVAL;
    if (c) {
        const int64_t tiles = (int64_t)((c->width + cf->tile - 1) / cf->tile) * ((c->height + cf->tile - 1) / cf->tile);
        if (tiles > (int64_t(1) << 24)) return GSR_EINVAL;
    }
    return GSR_OK;
}

gsr_status gsr_ctx_create(gsr_ctx **out, int device, void *hip_stream) {
    if (!out) return GSR_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return GSR_EHIP;
    if (device < 0 || device >= count) return GSR_EINVAL;
    gsr_ctx *ctx = new (std::nothrow) gsr_ctx();
    if (!ctx) return GSR_ENOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return GSR_EHIP;
    }
    // NULL is HIP's null stream: the stream a framework's default stream enqueues on, so work
    // stays ordered with the caller's own kernels. The library never creates streams.
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->pool = new (std::nothrow) Pool(device);
    void *hp = nullptr;
    if (!ctx->pool || hipHostMalloc(&hp, 1024, hipHostMallocDefault) != hipSuccess) {
        gsr_ctx_destroy(ctx);
        return GSR_ENOMEM;
    }
    ctx->host_pinned = static_cast<uint32_t *>(hp);
    scratch_init(ctx);
    for (auto &e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            gsr_ctx_destroy(ctx);
            return GSR_EHIP;
        }
    }
    if (hipEventCreateWithFlags(&ctx->ev_counts, hipEventDisableTiming) != hipSuccess) {
        gsr_ctx_destroy(ctx);
        return GSR_EHIP;
    }
    *out = ctx;
    return GSR_OK;
}

void gsr_ctx_destroy(gsr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->ev_counts) (void)hipEventDestroy(ctx->ev_counts);
    delete ctx->pool;
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    delete ctx;
}

const char *gsr_ctx_last_error(const gsr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gsr_status gsr_ctx_set_stream(gsr_ctx *ctx, void *hip_stream) {
    if (!ctx) return GSR_EINVAL;
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    // Drain the old stream first: pooled buffers are only safe to reuse in one stream order.
    GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return GSR_OK;
}

} // extern "C"

namespace {

// Pool buffer that goes back to the pool when the scope ends. The pool hands
// it out again only to later work on the same stream, so releasing it right
// after the launches that use it are enqueued is safe.
struct TempBuf {
    gsr_ctx *ctx = nullptr;
    void *p = nullptr;
    ~TempBuf() {
        if (ctx && p) ctx->pool->release(p);
    }
};

template <typename T>
gsr_status temp_alloc(gsr_ctx *ctx, TempBuf &t, T **p, size_t count) {
    GSR_TRY(pool_alloc(ctx, nullptr, p, count));
    t.ctx = ctx;
    t.p = *p;
    return GSR_OK;
}

ViewDesc desc_of(const gsr_fwd *st, float *image, const float *dl) {
    ViewDesc d{};
    d.cam = st->dcam;
    d.ranges = st->ranges;
    d.ids = st->sorted_pair_id;
    d.rec = st->rec;
    d.image = image;
    d.T_final = st->T_final;
    d.n_contrib = st->n_contrib;
    d.tile_walk = st->tile_walk;
    d.dl_dimage = dl;
    d.acc = st->acc;
    return d;
}

gsr_status check_view(gsr_ctx *ctx, int i, const gsr_scene *scene, const gsr_camera *camera,
                      const gsr_config *config, const float *image) {
    if (gsr_validate_scene(scene) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid scene (view %d)", i);
    if (gsr_validate_camera(camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid camera (view %d)", i);
    if (gsr_validate_config(config, camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid config (view %d)", i);
    if (!image) return fail(ctx, GSR_EINVAL, "image is null (view %d)", i);
    return GSR_OK;
}

// Pair buffers get headroom, so that a later re-render in capacity mode (no host sync) holds
// pair counts up to a quarter (plus 4096) above this render's.
int64_t pair_capacity(int64_t P) { return P + P / 4 + 4096; }

gsr_status alloc_view(gsr_ctx *ctx, gsr_fwd *st) {
    const int64_t n = st->n, nn = n > 0 ? n : 1;
    const int64_t hw = (int64_t)st->camera.width * st->camera.height;
    GSR_TRY(pool_alloc(ctx, st, &st->rec, 3 * nn));
    GSR_TRY(pool_alloc(ctx, st, &st->radius, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->tiles_touched, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->clamp_mask, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->depth_key, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->ids, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->key_alt, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->ids_alt, nn));
    GSR_TRY(pool_alloc(ctx, st, &st->offsets, nn + 1));
    GSR_TRY(pool_alloc(ctx, st, &st->ranges, st->n_tiles));
    GSR_TRY(pool_alloc(ctx, st, &st->T_final, hw));
    GSR_TRY(pool_alloc(ctx, st, &st->n_contrib, hw));
    GSR_TRY(pool_alloc(ctx, st, &st->totals, 8));
    if (n > 1) {
        const size_t hc = radix_hist_count(n);
        GSR_TRY(pool_alloc(ctx, st, &st->dsort_hist, hc));
        GSR_TRY(pool_alloc(ctx, st, &st->dsort_partials, scan_partial_count((int64_t)hc)));
    }
    GSR_TRY(pool_alloc(ctx, st, &st->scan_partials, scan_partial_count(nn) + 8));
    GSR_TRY(pool_alloc(ctx, st, &st->vis_part, visible_partial_count(nn)));
    return GSR_OK;
}

gsr_status alloc_pairs(gsr_ctx *ctx, gsr_fwd *st, int64_t cap) {
    GSR_TRY(pool_alloc(ctx, st, &st->pair_tile, cap));
    GSR_TRY(pool_alloc(ctx, st, &st->pair_id, cap));
    GSR_TRY(pool_alloc(ctx, st, &st->pair_tile_alt, cap));
    GSR_TRY(pool_alloc(ctx, st, &st->pair_id_alt, cap));
    const size_t hc = radix_hist_count(cap);
    GSR_TRY(pool_alloc(ctx, st, &st->tsort_hist, hc));
    GSR_TRY(pool_alloc(ctx, st, &st->tsort_partials, scan_partial_count((int64_t)hc)));
    st->pair_cap = cap;
    return GSR_OK;
}

// a1 and the depth-digit sort for every view.
gsr_status enqueue_project_and_depth_sort(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, bool tm) {
    hipStream_t s = ctx->stream;
    mark(ctx, tm, EV_R0);
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_HIP(ctx, launch_preprocess_fwd(st->scene, st->dcam, st->rec, st->radius, st->tiles_touched, st->depth_key,
                                           st->ids, st->clamp_mask, s));
    }
    mark(ctx, tm, EV_R1);
    // a2/a3 (depth digits): sort Gaussians by fp32 depth; stable, so ties keep index order.
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        int which = 0;
        if (st->n > 1)
            GSR_HIP(ctx, radix_sort_pairs(st->depth_key, st->ids, st->key_alt, st->ids_alt, st->n, 32, st->dsort_hist,
                                          st->dsort_partials, &which, s));
        st->sorted_ids_by_depth = which ? st->ids_alt : st->ids;
    }
    mark(ctx, tm, EV_R2);
    // a2: pair offsets in depth order, their total P and the visible count.
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_HIP(ctx, device_exclusive_scan(st->tiles_touched, st->sorted_ids_by_depth, st->offsets, st->n,
                                           st->totals, st->scan_partials, s));
        GSR_HIP(ctx, launch_count_positive(st->radius, st->n, st->totals + 1, s));
    }
    return GSR_OK;
}

// a5 for every view in one launch (longest list first); it records each tile's deepest
// n_contrib (tile_walk), from which the backward orders its tiles. work: a table of base[nv]
// entries for the launch (nullptr: a pool temp).
gsr_status enqueue_composite_fwd(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, float *const *images,
                                 const gsr_config *config, uint2 *work_buf, bool tm) {
    hipStream_t s = ctx->stream;
    const bool ordered = !(config->flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER));
    ViewBatch vb{};
    vb.n = nv;
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        if (ordered && !st->tile_walk) GSR_TRY(pool_alloc(ctx, st, &st->tile_walk, st->n_tiles));
        if (!ordered) st->tile_walk = nullptr;
        vb.v[v] = desc_of(st, images[v], nullptr);
        vb.base[v + 1] = vb.base[v] + (uint32_t)st->n_tiles;
    }
    {
        TempBuf tb;
        uint2 *work = nullptr;
        if (nv > 1 || ordered) {
            work = work_buf;
            if (!work) GSR_TRY(temp_alloc(ctx, tb, &work, vb.base[nv]));
            GSR_HIP(ctx, launch_order_tiles(vb, ordered ? ORDER_BY_LENGTH : ORDER_IDENTITY, work, s));
        }
        const int remap = (nv == 1 && (config->flags & GSR_FLAG_XCD_REMAP)) ? 1 : 0;
        GSR_HIP(ctx, launch_composite_fwd(vb, config->tile, config->lds_batch, remap, work, s));
    }
    mark(ctx, tm, EV_R6);
    return GSR_OK;
}

// Renders nv validated views. Every stage runs for all views before the
// next; one synchronisation reads back all pair counts; the composite is one
// launch over all (view, tile) pairs.
gsr_status render_views(gsr_ctx *ctx, int nv, const gsr_scene *scenes, const gsr_camera *cameras,
                        const gsr_config *config, float *const *images, gsr_fwd **states_out) {
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_render = tm;
    gsr_fwd *sts[kMaxViews] = {};
    uint32_t *sorted_tile[kMaxViews] = {};
    const auto bail = [&](gsr_status code) {
        for (int v = 0; v < nv; ++v)
            if (sts[v]) gsr_fwd_release(ctx, sts[v]);
        return code;
    };
#define GSR_RT(x)                                                                                                   \
    do {                                                                                                            \
        gsr_status s_ = (x);                                                                                        \
        if (s_ != GSR_OK) return bail(s_);                                                                          \
    } while (0)
#define GSR_RH(expr)                                                                                                \
    do {                                                                                                            \
        hipError_t e_ = (expr);                                                                                     \
        if (e_ != hipSuccess) return bail(fail(ctx, GSR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)));      \
    } while (0)

    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = new (std::nothrow) gsr_fwd();
        if (!st) return bail(fail(ctx, GSR_ENOMEM, "host allocation failed"));
        sts[v] = st;
        st->scene = scenes[v];
        st->camera = cameras[v];
        st->config = *config;
        st->dcam = make_dev_camera(cameras[v], config->tile);
        st->n = scenes[v].n;
        st->n_tiles = (int64_t)st->dcam.grid_x * st->dcam.grid_y;
        GSR_RT(alloc_view(ctx, st));
    }
    mark(ctx, tm, EV_R0);
    // a1: projection
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_RH(launch_preprocess_fwd(st->scene, st->dcam, st->rec, st->radius, st->tiles_touched, st->depth_key,
                                     st->ids, st->clamp_mask, s));
    }
    mark(ctx, tm, EV_R1);
    // Visible Gaussians are compacted (index order) before the depth sort, and the pair count
    // P = sum of tile counts taken; the counts of all views are read back at once.
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_RH(launch_compact_visible(st->radius, st->n, st->depth_key, st->tiles_touched, st->vis_part, st->totals,
                                      st->key_alt, st->ids_alt, s));
        GSR_RH(hipMemcpyAsync(ctx->host_pinned + 6 * v, st->totals, 6 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    GSR_RH(hipEventRecord(ctx->ev_counts, s));
    // a2/a3 (depth digits): stable sort of the visible Gaussians by fp32 depth (ties keep index
    // order). Bits above the highest one in which the smallest and the largest visible key differ
    // are the same in every key and need no pass (for an object seen from outside the exponent
    // byte of every depth is the same). One view whose sort of all n Gaussians needs no scan
    // launches: the sort is enqueued before the host waits for the counts, launched for all n
    // and bounded by the visible count and key range on the device (passes above the varying
    // bits copy), so the GPU sorts while the counts travel. Otherwise, and for several views
    // (which share one wait), each view's sort is sized by its read-back count and key range:
    // at 3M Gaussians / 1080p (0.7M visible) that took 115 us against 144 us for the sort of
    // all n bounded on the device; at 100k / 800x800 the bounded sort took 61 us against 69.
    const bool overlap = nv == 1 && radix_sort_fused(sts[0]->n);
    if (overlap) {
        gsr_fwd *st = sts[0];
        int which = 0;
        GSR_RH(radix_sort_pairs(st->key_alt, st->ids_alt, st->depth_key, st->ids, st->n, 32, st->dsort_hist,
                                st->dsort_partials, &which, s, st->totals + 1, st->totals + 4));
        st->sorted_ids_by_depth = which ? st->ids : st->ids_alt;
    }
    GSR_RH(hipEventSynchronize(ctx->ev_counts));
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        const uint32_t *h = ctx->host_pinned + 6 * v;
        st->P = st->n > 0 ? (int64_t)h[0] : 0;
        st->n_visible = st->n > 0 ? (int64_t)h[1] : 0;
        st->p_known = true;
        if (overlap) continue;
        const uint32_t kmin = ~h[4], kmax = h[5];
        const int bits = kmin < kmax ? 32 - __builtin_clz(kmin ^ kmax) : 0;
        int which = 0;
        if (st->n_visible > 1 && bits > 0)
            GSR_RH(radix_sort_pairs(st->key_alt, st->ids_alt, st->depth_key, st->ids, st->n_visible, bits,
                                    st->dsort_hist, st->dsort_partials, &which, s));
        st->sorted_ids_by_depth = which ? st->ids : st->ids_alt;
    }
    mark(ctx, tm, EV_R2);
    // a2: pair offsets in depth order and the pairs.
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_RH(device_exclusive_scan(st->tiles_touched, st->sorted_ids_by_depth, st->offsets, st->n_visible,
                                     st->totals, st->scan_partials, s));
        GSR_RT(alloc_pairs(ctx, st, pair_capacity(st->P)));
        GSR_RH(launch_emit_pairs(st->n_visible, st->sorted_ids_by_depth, st->offsets, st->rec, st->radius, st->dcam,
                                 st->pair_tile, st->pair_id, st->pair_cap, s));
    }
    mark(ctx, tm, EV_R3);
    // a3 (tile digits): stable sort of the P pairs by tile.
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        int which = 0;
        if (st->P > 1)
            GSR_RH(radix_sort_pairs(st->pair_tile, st->pair_id, st->pair_tile_alt, st->pair_id_alt, st->P,
                                    bits_for(st->n_tiles), st->tsort_hist, st->tsort_partials, &which, s));
        sorted_tile[v] = which ? st->pair_tile_alt : st->pair_tile;
        st->sorted_pair_id = which ? st->pair_id_alt : st->pair_id;
    }
    mark(ctx, tm, EV_R4);
    // a4: per-tile ranges
    for (int v = 0; v < nv; ++v)
        GSR_RH(launch_tile_ranges(sts[v]->P, nullptr, sorted_tile[v], sts[v]->ranges, sts[v]->n_tiles, s));
    mark(ctx, tm, EV_R5);
    GSR_RT(enqueue_composite_fwd(ctx, nv, sts, images, config, nullptr, tm));
#undef GSR_RT
#undef GSR_RH
    for (int v = 0; v < nv; ++v) states_out[v] = sts[v];
    return GSR_OK;
}

// Capacity mode: re-renders existing states (their scenes' current contents, their cameras)
// into their own buffers without any host synchronisation. Each view's tile sort and ranges are
// launched for its whole pair capacity and bounded on the device by its pair count (blocks past
// it exit at once); a view whose pairs exceed the capacity keeps the first pair_cap pairs and
// sets its overflow flag (gsr_fwd_sync reports it).
gsr_status rerender_views(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, float *const *images, const gsr_config *config,
                          uint2 *work_buf, bool tm) {
    hipStream_t s = ctx->stream;
    uint32_t *sorted_tile[kMaxViews] = {};
    for (int v = 0; v < nv; ++v) {
        sts[v]->p_known = false;
        sts[v]->capacity_mode = true;
    }
    GSR_TRY(enqueue_project_and_depth_sort(ctx, nv, sts, tm));
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        GSR_HIP(ctx, launch_emit_pairs(st->n, st->sorted_ids_by_depth, st->offsets, st->rec, st->radius, st->dcam,
                                       st->pair_tile, st->pair_id, st->pair_cap, s));
        GSR_HIP(ctx, launch_pair_overflow(st->totals, st->pair_cap, st->totals + 2, s));
    }
    mark(ctx, tm, EV_R3);
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        int which = 0;
        GSR_HIP(ctx, radix_sort_pairs(st->pair_tile, st->pair_id, st->pair_tile_alt, st->pair_id_alt, st->pair_cap,
                                      bits_for(st->n_tiles), st->tsort_hist, st->tsort_partials, &which, s,
                                      st->totals));
        sorted_tile[v] = which ? st->pair_tile_alt : st->pair_tile;
        st->sorted_pair_id = which ? st->pair_id_alt : st->pair_id;
    }
    mark(ctx, tm, EV_R4);
    for (int v = 0; v < nv; ++v)
        GSR_HIP(ctx, launch_tile_ranges(sts[v]->pair_cap, sts[v]->totals, sorted_tile[v], sts[v]->ranges,
                                        sts[v]->n_tiles, s));
    mark(ctx, tm, EV_R5);
    return enqueue_composite_fwd(ctx, nv, sts, images, config, work_buf, tm);
}

// Renders nv validated views into new states whose pair buffers hold caps[v] pairs, in capacity
// mode: no host synchronisation; a view whose pairs exceed its capacity raises its overflow word
// (totals[2]) and its lists hold only the first caps[v] pairs.
gsr_status render_views_capacity(gsr_ctx *ctx, int nv, const gsr_scene *scenes, const gsr_camera *cameras,
                                 const gsr_config *config, float *const *images, const int64_t *caps,
                                 gsr_fwd **states_out) {
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_render = tm;
    gsr_fwd *sts[kMaxViews] = {};
    gsr_status status = GSR_OK;
    for (int v = 0; v < nv && status == GSR_OK; ++v) {
        status = check_view(ctx, v, &scenes[v], &cameras[v], config, images[v]);
        if (status != GSR_OK) break;
        gsr_fwd *st = new (std::nothrow) gsr_fwd();
        if (!st) {
            status = fail(ctx, GSR_ENOMEM, "host allocation failed");
            break;
        }
        sts[v] = st;
        st->scene = scenes[v];
        st->camera = cameras[v];
        st->config = *config;
        st->dcam = make_dev_camera(cameras[v], config->tile);
        st->n = scenes[v].n;
        st->n_tiles = (int64_t)st->dcam.grid_x * st->dcam.grid_y;
        status = alloc_view(ctx, st);
        if (status == GSR_OK) status = alloc_pairs(ctx, st, caps[v] > 0 ? caps[v] : 1);
    }
    if (status == GSR_OK) status = rerender_views(ctx, nv, sts, images, config, nullptr, tm);
    if (status != GSR_OK) {
        for (int v = 0; v < nv; ++v)
            if (sts[v]) gsr_fwd_release(ctx, sts[v]);
        return status;
    }
    for (int v = 0; v < nv; ++v) states_out[v] = sts[v];
    return GSR_OK;
}

// Backward composite over nv checked states, in two parts so that the second
// can be captured in a graph: bwd_prepare makes every buffer exist (and
// computes a single view's cached tile order once), bwd_enqueue only launches
// kernels (accumulators zeroed by fill kernels, one composite launch over
// every (view, tile) pair).
struct BwdPlan {
    ViewBatch vb{};
    int order_mode = ORDER_IDENTITY;
    uint2 *work = nullptr;   // table the composite reads (nullptr: identity / XCD remap, one view)
    bool build_work = false; // recompute `work` before the composite
    int remap = 0;
    bool own_acc = true;     // accumulators are the states' own rows (not the fixed scratch)
};

gsr_status bwd_prepare(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, const float *const *dls, const gsr_config *cfg,
                       BwdPlan &plan) {
    const bool count = (cfg->flags & GSR_FLAG_DEBUG_COUNTERS) != 0;
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = sts[v];
        if (!st->acc) {
            double *a = nullptr; // rows sized for doubles, so either precision fits
            GSR_TRY(pool_alloc(ctx, st, &a, (size_t)(st->n > 0 ? st->n : 1) * GSR_ACC_STRIDE));
            st->acc = a;
        }
    }
    if (count && !sts[0]->counters) GSR_TRY(pool_alloc(ctx, sts[0], &sts[0]->counters, 80));
    ViewBatch &vb = plan.vb;
    vb = ViewBatch{};
    vb.n = nv;
    bool walks = true;
    for (int v = 0; v < nv; ++v) {
        vb.v[v] = desc_of(sts[v], nullptr, dls[v]);
        vb.base[v + 1] = vb.base[v] + (uint32_t)sts[v]->n_tiles;
        walks = walks && sts[v]->tile_walk != nullptr;
    }
    const bool ordered = !(cfg->flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER));
    plan.order_mode = ordered ? (walks ? ORDER_BY_WALK : ORDER_BY_LENGTH) : ORDER_IDENTITY;
    plan.remap = (nv == 1 && (cfg->flags & GSR_FLAG_XCD_REMAP)) ? 1 : 0;
    plan.work = nullptr;
    plan.build_work = false;
    if (nv == 1) {
        if (ordered) {
            gsr_fwd *st = sts[0];
            if (!st->order_bwd) GSR_TRY(pool_alloc(ctx, st, &st->order_bwd, st->n_tiles));
            plan.work = st->order_bwd;
            plan.build_work = true;
        }
    } else {
        gsr_fwd *lead = sts[0];
        if (lead->batch_work_cap < (int64_t)vb.base[nv]) {
            GSR_TRY(pool_alloc(ctx, lead, &lead->batch_work, vb.base[nv]));
            lead->batch_work_cap = vb.base[nv];
        }
        plan.work = lead->batch_work;
        plan.build_work = true;
    }
    return GSR_OK;
}

gsr_status bwd_enqueue(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, const gsr_config *cfg, const BwdPlan &plan,
                       bool tm) {
    hipStream_t s = ctx->stream;
    const bool count = (cfg->flags & GSR_FLAG_DEBUG_COUNTERS) != 0;
    const bool f64 = (cfg->flags & GSR_FLAG_ACC_F32) == 0;
    for (int v = 0; v < nv; ++v) sts[v]->counters_valid = false;
    mark(ctx, tm, EV_B0);
    // The tiles' order for this backward (longest recorded walk first), built from the walks of
    // the render it follows, is timed with the clearing, so the composite's span is its kernel
    // alone; for one view both go in one launch.
    const bool fused = nv == 1 && plan.build_work;
    for (int v = 0; v < nv; ++v) {
        // The depth-sorted ids start with the visible Gaussians (culled ones carry the largest
        // key): after a render that read its counts back they are exactly those; after a
        // capacity-mode render their count is on the device.
        const gsr_fwd *sv = sts[v];
        const int64_t m = sv->p_known ? sv->n_visible : sv->n;
        const uint32_t *m_dev = sv->p_known ? nullptr : sv->totals + 1;
        if (fused)
            GSR_HIP(ctx, launch_clear_rows_and_order(plan.vb, plan.order_mode, plan.work, sv->sorted_ids_by_depth, m,
                                                     m_dev, plan.vb.v[v].acc, f64, s));
        else
            GSR_HIP(ctx, launch_zero_visible_rows(sv->radius, sv->n, sv->sorted_ids_by_depth, m, m_dev,
                                                  plan.vb.v[v].acc, f64, s));
        if (plan.own_acc) sts[v]->acc_f64 = f64;
    }
    if (count) GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(sts[0]->counters), 0u, 160, s));
    if (plan.build_work && !fused) GSR_HIP(ctx, launch_order_tiles(plan.vb, plan.order_mode, plan.work, s));
    mark(ctx, tm, EV_B1);
    BwdParams p{};
    p.counters = count ? sts[0]->counters : nullptr;
    p.threshold = cfg->reduce_threshold < 1 ? 1 : cfg->reduce_threshold;
    if (cfg->bwd_mode == GSR_BWD_PLAIN_COMPILER_REDUCE)
        GSR_HIP(ctx, launch_composite_bwd_compiler_reduce(plan.vb, cfg->tile, cfg->lds_batch, plan.remap, f64, p,
                                                          plan.work, s));
    else
        GSR_HIP(ctx, launch_composite_bwd(plan.vb, cfg->tile, cfg->lds_batch, plan.remap, cfg->bwd_mode, count,
                                          (cfg->flags & GSR_FLAG_LANE_SPLIT_ATOMICS) != 0, f64, p, plan.work, s));
    mark(ctx, tm, EV_B2);
    sts[0]->counters_valid = count;
    return GSR_OK;
}

gsr_status bwd_views(gsr_ctx *ctx, int nv, gsr_fwd *const *sts, const float *const *dls, const gsr_config *cfg,
                     bool tm) {
    BwdPlan plan;
    GSR_TRY(bwd_prepare(ctx, nv, sts, dls, cfg, plan));
    return bwd_enqueue(ctx, nv, sts, cfg, plan, tm);
}

// The plan of a single-view backward whose accumulators and (when the state caches none) tile
// order are in the fixed scratch: makes no buffer.
void bwd_plan_scratch(gsr_ctx *ctx, gsr_fwd *st, const float *dl, const gsr_config *cfg, BwdPlan &plan) {
    ViewBatch &vb = plan.vb;
    vb = ViewBatch{};
    vb.n = 1;
    vb.v[0] = desc_of(st, nullptr, dl);
    vb.v[0].acc = ctx->scratch;
    vb.base[1] = (uint32_t)st->n_tiles;
    const bool ordered = !(cfg->flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER));
    plan.order_mode = ordered ? (st->tile_walk ? ORDER_BY_WALK : ORDER_BY_LENGTH) : ORDER_IDENTITY;
    plan.remap = (cfg->flags & GSR_FLAG_XCD_REMAP) ? 1 : 0;
    plan.work = nullptr;
    plan.build_work = false;
    plan.own_acc = false;
    if (ordered) {
        plan.work = st->order_bwd ? st->order_bwd
                                  : reinterpret_cast<uint2 *>(static_cast<unsigned char *>(ctx->scratch) +
                                                              kNoallocRowBytes);
        plan.build_work = true;
    }
}

gsr_status check_bwd_args(gsr_ctx *ctx, gsr_fwd *st, const float *dl, const gsr_config **cfg) {
    if (!st) return fail(ctx, GSR_EINVAL, "state is null");
    if (!dl) return fail(ctx, GSR_EINVAL, "dl_dimage is null");
    if (!*cfg) *cfg = &st->config;
    if ((*cfg)->tile != st->config.tile) return fail(ctx, GSR_EINVAL, "backward tile differs from the render's");
    if (gsr_validate_config(*cfg, &st->camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid config");
    return GSR_OK;
}

gsr_status check_grads(gsr_ctx *ctx, const gsr_fwd *st, const gsr_grads *out) {
    if (!out) return fail(ctx, GSR_EINVAL, "grads is null");
    if (st->n > 0 && (!out->means3d || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh))
        return fail(ctx, GSR_EINVAL, "a gradient pointer is null");
    return GSR_OK;
}

// 0: no pointer shared, 1: all five equal, -1: some but not all.
int grads_alias(const gsr_grads &a, const gsr_grads &b) {
    const int eq = (a.means3d == b.means3d) + (a.log_scales == b.log_scales) + (a.quats == b.quats) +
                   (a.opacity_logits == b.opacity_logits) + (a.sh == b.sh);
    return eq == 5 ? 1 : (eq == 0 ? 0 : -1);
}

} // namespace

namespace gsr {
gsr_status render_batch_capacity(gsr_ctx *ctx, int nv, const gsr_scene *scenes, const gsr_camera *cameras,
                                 const gsr_config *config, float *const *images, const int64_t *caps,
                                 gsr_fwd **states_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (nv < 1 || nv > GSR_MAX_BATCH) return fail(ctx, GSR_EINVAL, "n_views %d outside 1..16", nv);
    if (!scenes || !cameras || !images || !caps || !states_out || !config)
        return fail(ctx, GSR_EINVAL, "null array argument");
    for (int v = 0; v < nv; ++v) states_out[v] = nullptr;
    return render_views_capacity(ctx, nv, scenes, cameras, config, images, caps, states_out);
}
} // namespace gsr

extern "C" {

gsr_status gsr_render(gsr_ctx *ctx, const gsr_scene *scene, const gsr_camera *camera, const gsr_config *config,
                      float *image_chw, gsr_fwd **state_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!state_out) return fail(ctx, GSR_EINVAL, "state_out is null");
    *state_out = nullptr;
    GSR_TRY(check_view(ctx, 0, scene, camera, config, image_chw));
    return render_views(ctx, 1, scene, camera, config, &image_chw, state_out);
}

gsr_status gsr_render_batch(gsr_ctx *ctx, int32_t n_views, const gsr_scene *scenes, const gsr_camera *cameras,
                            const gsr_config *config, float *const *images_chw, gsr_fwd **states_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (n_views < 1 || n_views > GSR_MAX_BATCH) return fail(ctx, GSR_EINVAL, "n_views %d outside 1..16", n_views);
    if (!scenes || !cameras || !images_chw || !states_out) return fail(ctx, GSR_EINVAL, "null array argument");
    for (int v = 0; v < n_views; ++v) states_out[v] = nullptr;
    for (int v = 0; v < n_views; ++v) GSR_TRY(check_view(ctx, v, &scenes[v], &cameras[v], config, images_chw[v]));
    return render_views(ctx, n_views, scenes, cameras, config, images_chw, states_out);
}

gsr_status gsr_backward_composite(gsr_ctx *ctx, gsr_fwd *st, const float *dl_dimage_chw, const gsr_config *config) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    GSR_TRY(check_bwd_args(ctx, st, dl_dimage_chw, &config));
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_bwd = false;
    return bwd_views(ctx, 1, &st, &dl_dimage_chw, config, tm);
}

gsr_status gsr_backward_params(gsr_ctx *ctx, gsr_fwd *st, const gsr_grads *out, int accumulate) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st) return fail(ctx, GSR_EINVAL, "state is null");
    GSR_TRY(check_grads(ctx, st, out));
    if (!st->acc) return fail(ctx, GSR_ESTATE, "no backward composite has run on this state");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, st->acc, st->acc_f64, *out, accumulate ? 1 : 0,
                                       ctx->stream));
    return GSR_OK;
}

gsr_status gsr_backward(gsr_ctx *ctx, gsr_fwd *st, const float *dl_dimage_chw, const gsr_grads *out, int accumulate,
                        const gsr_config *config) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    GSR_TRY(check_bwd_args(ctx, st, dl_dimage_chw, &config));
    GSR_TRY(check_grads(ctx, st, out));
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    GSR_TRY(bwd_views(ctx, 1, &st, &dl_dimage_chw, config, tm));
    GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, st->acc, st->acc_f64, *out, accumulate ? 1 : 0,
                                       ctx->stream));
    mark(ctx, tm, EV_B3);
    ctx->timing_bwd = tm;
    return GSR_OK;
}

gsr_status gsr_backward_noalloc(gsr_ctx *ctx, gsr_fwd *st, const float *dl_dimage_chw, const gsr_grads *out,
                                int accumulate, const gsr_config *config) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    GSR_TRY(check_bwd_args(ctx, st, dl_dimage_chw, &config));
    GSR_TRY(check_grads(ctx, st, out));
    if (config->flags & GSR_FLAG_DEBUG_COUNTERS)
        return fail(ctx, GSR_EINVAL, "debug counters need an allocated buffer (use gsr_backward)");
    if (st->n > GSR_NOALLOC_MAX_GAUSSIANS)
        return fail(ctx, GSR_EINVAL, "%lld Gaussians exceed the allocation-free backward's %d",
                    (long long)st->n, GSR_NOALLOC_MAX_GAUSSIANS);
    if (st->n_tiles > GSR_NOALLOC_MAX_TILES)
        return fail(ctx, GSR_EINVAL, "%lld tiles exceed the allocation-free backward's %d", (long long)st->n_tiles,
                    GSR_NOALLOC_MAX_TILES);
    if (!ctx->scratch)
        return fail(ctx, GSR_EHIP, "scratch address of device %d unavailable: %s", ctx->device,
                    hipGetErrorString(ctx->scratch_err));
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    BwdPlan plan;
    bwd_plan_scratch(ctx, st, dl_dimage_chw, config, plan);
    GSR_TRY(bwd_enqueue(ctx, 1, &st, config, plan, tm));
    const bool f64 = (config->flags & GSR_FLAG_ACC_F32) == 0;
    GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, ctx->scratch, f64, *out, accumulate ? 1 : 0,
                                       ctx->stream));
    mark(ctx, tm, EV_B3);
    ctx->timing_bwd = tm;
    return GSR_OK;
}

} // extern "C"

namespace {

// Argument checks shared by the batched backward and its graph capture. adds[v]: view v's
// per-Gaussian part adds to its outputs (accumulate, or outputs shared with an earlier view).
gsr_status check_batch_bwd(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states, const float *const *dls,
                           const gsr_grads *outs, int accumulate, const gsr_config **config, int *adds) {
    if (n_views < 1 || n_views > GSR_MAX_BATCH) return fail(ctx, GSR_EINVAL, "n_views %d outside 1..16", n_views);
    if (!states || !dls || !outs) return fail(ctx, GSR_EINVAL, "null array argument");
    if (!states[0]) return fail(ctx, GSR_EINVAL, "state 0 is null");
    if (!*config) *config = &states[0]->config;
    for (int v = 0; v < n_views; ++v) {
        const gsr_config *c = *config;
        GSR_TRY(check_bwd_args(ctx, states[v], dls[v], &c));
        GSR_TRY(check_grads(ctx, states[v], &outs[v]));
        adds[v] = accumulate ? 1 : 0;
        for (int u = 0; u < v; ++u) {
            if (states[u] == states[v]) return fail(ctx, GSR_EINVAL, "views %d and %d share a state", u, v);
            const int al = grads_alias(outs[u], outs[v]);
            if (al < 0) return fail(ctx, GSR_EINVAL, "outputs of views %d and %d partly overlap", u, v);
            if (al > 0) adds[v] = 1;
        }
    }
    return GSR_OK;
}

gsr_status enqueue_params(gsr_ctx *ctx, int nv, gsr_fwd *const *states, const gsr_grads *outs, const int *adds) {
    for (int v = 0; v < nv; ++v) {
        gsr_fwd *st = states[v];
        GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, st->acc, st->acc_f64, outs[v], adds[v],
                                           ctx->stream));
    }
    return GSR_OK;
}

} // namespace

struct gsr_graph {
    int device = 0;
    gsr_ctx *ctx = nullptr;          // the capturing context; its pool owns `owned`
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> owned;       // buffers only the replays use (work tables, loss scratch)
};

extern "C" {

gsr_status gsr_backward_batch(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states,
                              const float *const *dl_dimages_chw, const gsr_grads *outs, int accumulate,
                              const gsr_config *config) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    int adds[kMaxViews] = {};
    GSR_TRY(check_batch_bwd(ctx, n_views, states, dl_dimages_chw, outs, accumulate, &config, adds));
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    GSR_TRY(bwd_views(ctx, n_views, states, dl_dimages_chw, config, tm));
    GSR_TRY(enqueue_params(ctx, n_views, states, outs, adds));
    mark(ctx, tm, EV_B3);
    ctx->timing_bwd = tm;
    return GSR_OK;
}

} // extern "C"

namespace {

// Records `body` (which only enqueues kernels on ctx->stream) into a graph. When the context
// is on the null stream the capture runs on a temporary stream of default priority.
template <typename F>
gsr_status capture_graph(gsr_ctx *ctx, gsr_graph *gr, F &&body) {
    hipStream_t saved = ctx->stream, cs = ctx->stream;
    const bool own = cs == nullptr;
    if (own) GSR_HIP(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    gsr_status st = GSR_OK;
    if (e == hipSuccess) {
        ctx->stream = cs;
        st = body();
        ctx->stream = saved;
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cs, &g) : e;
    if (own) (void)hipStreamDestroy(cs);
    if (st != GSR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e2 != hipSuccess) return fail(ctx, GSR_EHIP, "stream capture failed: %s", hipGetErrorString(e2));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(ctx, GSR_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    gr->device = ctx->device;
    gr->ctx = ctx;
    gr->graph = g;
    gr->exec = ex;
    return GSR_OK;
}

template <typename T>
gsr_status graph_alloc(gsr_ctx *ctx, gsr_graph *gr, T **p, size_t count) {
    GSR_TRY(pool_alloc(ctx, nullptr, p, count));
    gr->owned.push_back(*p);
    return GSR_OK;
}

void free_graph(gsr_ctx *ctx, gsr_graph *gr) {
    for (void *p : gr->owned) ctx->pool->release(p);
    delete gr;
}

} // namespace

extern "C" {

gsr_status gsr_graph_capture_backward(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states,
                                      const float *const *dl_dimages_chw, const gsr_grads *outs, int accumulate,
                                      const gsr_config *config, gsr_graph **graph_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!graph_out) return fail(ctx, GSR_EINVAL, "graph_out is null");
    *graph_out = nullptr;
    int adds[kMaxViews] = {};
    GSR_TRY(check_batch_bwd(ctx, n_views, states, dl_dimages_chw, outs, accumulate, &config, adds));
    gsr_config cfg = *config;
    cfg.flags &= ~GSR_FLAG_STAGE_TIMING;
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    // Every buffer is allocated (and a single view's tile order computed) before the capture,
    // so the captured work is kernels only.
    BwdPlan plan;
    GSR_TRY(bwd_prepare(ctx, n_views, states, dl_dimages_chw, &cfg, plan));
    gsr_graph *gr = new (std::nothrow) gsr_graph();
    if (!gr) return fail(ctx, GSR_ENOMEM, "host allocation failed");
    const gsr_status st = capture_graph(ctx, gr, [&] {
        GSR_TRY(bwd_enqueue(ctx, n_views, states, &cfg, plan, false));
        return enqueue_params(ctx, n_views, states, outs, adds);
    });
    if (st != GSR_OK) {
        free_graph(ctx, gr);
        return st;
    }
    *graph_out = gr;
    return GSR_OK;
}

gsr_status gsr_rerender_batch(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states, float *const *images_chw,
                              const gsr_config *config) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (n_views < 1 || n_views > GSR_MAX_BATCH) return fail(ctx, GSR_EINVAL, "n_views %d outside 1..16", n_views);
    if (!states || !images_chw) return fail(ctx, GSR_EINVAL, "null array argument");
    if (!states[0]) return fail(ctx, GSR_EINVAL, "state 0 is null");
    if (!config) config = &states[0]->config;
    for (int v = 0; v < n_views; ++v) {
        if (!states[v] || !images_chw[v]) return fail(ctx, GSR_EINVAL, "null state or image (view %d)", v);
        if (states[v]->config.tile != config->tile) return fail(ctx, GSR_EINVAL, "tile differs from the render's");
        if (gsr_validate_config(config, &states[v]->camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid config");
        for (int u = 0; u < v; ++u)
            if (states[u] == states[v]) return fail(ctx, GSR_EINVAL, "views %d and %d share a state", u, v);
    }
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_render = tm;
    return rerender_views(ctx, n_views, states, images_chw, config, nullptr, tm);
}

gsr_status gsr_fwd_sync(gsr_ctx *ctx, gsr_fwd *st, int64_t *n_pairs, int32_t *overflowed) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st) return fail(ctx, GSR_EINVAL, "state is null");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    int32_t over = 0;
    // After a capacity-mode render (or graph replays of one) the device holds the counts.
    if (!st->p_known || st->capacity_mode) {
        GSR_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, st->totals, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
        GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
        st->P = st->n > 0 ? (int64_t)ctx->host_pinned[0] : 0;
        st->n_visible = st->n > 0 ? (int64_t)ctx->host_pinned[1] : 0;
        over = ctx->host_pinned[2] != 0u;
        if (over) st->P = st->pair_cap; // the lists hold the first pair_cap pairs only
        st->p_known = true;
        st->overflowed = over != 0;
    } else {
        over = st->overflowed ? 1 : 0;
    }
    if (n_pairs) *n_pairs = st->P;
    if (overflowed) *overflowed = over;
    return GSR_OK;
}

gsr_status gsr_graph_capture_step(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states, float *const *images_chw,
                                  const float *const *targets_chw, float loss_lambda, float *const *dl_dimages_chw,
                                  const gsr_grads *outs, int accumulate, const gsr_config *config,
                                  gsr_graph **graph_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!graph_out) return fail(ctx, GSR_EINVAL, "graph_out is null");
    *graph_out = nullptr;
    if (!images_chw || !targets_chw || !dl_dimages_chw) return fail(ctx, GSR_EINVAL, "null array argument");
    if (!(loss_lambda >= 0.0f && loss_lambda <= 1.0f)) return fail(ctx, GSR_EINVAL, "lambda outside [0, 1]");
    int adds[kMaxViews] = {};
    GSR_TRY(check_batch_bwd(ctx, n_views, states, dl_dimages_chw, outs, accumulate, &config, adds));
    for (int v = 0; v < n_views; ++v)
        if (!images_chw[v] || !targets_chw[v]) return fail(ctx, GSR_EINVAL, "null image or target (view %d)", v);
    gsr_config cfg = *config;
    cfg.flags &= ~GSR_FLAG_STAGE_TIMING;
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    gsr_graph *gr = new (std::nothrow) gsr_graph();
    if (!gr) return fail(ctx, GSR_ENOMEM, "host allocation failed");
    const auto bail = [&](gsr_status code) {
        free_graph(ctx, gr);
        return code;
    };
    // Eager preparation: every buffer the replays touch exists before the capture.
    const bool ordered = !(cfg.flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER));
    int64_t tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        gsr_fwd *st = states[v];
        if (ordered && !st->tile_walk) {
            const gsr_status e = pool_alloc(ctx, st, &st->tile_walk, st->n_tiles);
            if (e != GSR_OK) return bail(e);
        }
        if (ordered && n_views == 1 && !st->order_bwd) {
            const gsr_status e = pool_alloc(ctx, st, &st->order_bwd, st->n_tiles);
            if (e != GSR_OK) return bail(e);
        }
        tiles += st->n_tiles;
    }
    uint2 *fwd_work = nullptr;
    if (n_views > 1 || ordered) {
        const gsr_status e = graph_alloc(ctx, gr, &fwd_work, tiles);
        if (e != GSR_OK) return bail(e);
    }
    float *scratch[kMaxViews][4] = {};
    if (loss_lambda > 0.0f)
        for (int v = 0; v < n_views; ++v) {
            const size_t n3 = 3 * (size_t)states[v]->camera.width * states[v]->camera.height;
            for (int k = 0; k < 3; ++k) {
                const gsr_status e = graph_alloc(ctx, gr, &scratch[v][k], n3);
                if (e != GSR_OK) return bail(e);
            }
            const gsr_status e = graph_alloc(ctx, gr, &scratch[v][3], 2);  // loss value not produced
            if (e != GSR_OK) return bail(e);
        }
    const float *dls_c[kMaxViews];
    for (int v = 0; v < n_views; ++v) dls_c[v] = dl_dimages_chw[v];
    BwdPlan plan;
    {
        const gsr_status e = bwd_prepare(ctx, n_views, states, dls_c, &cfg, plan);
        if (e != GSR_OK) return bail(e);
    }
    const gsr_status st = capture_graph(ctx, gr, [&] {
        GSR_TRY(rerender_views(ctx, n_views, states, images_chw, &cfg, fwd_work, false));
        for (int v = 0; v < n_views; ++v) {
            const gsr_camera &c = states[v]->camera;
            if (loss_lambda > 0.0f) {
                GSR_HIP(ctx, launch_l1_dssim_grad(images_chw[v], targets_chw[v], 3, c.width, c.height, loss_lambda,
                                                  scratch[v][0], scratch[v][1], scratch[v][2], scratch[v][3],
                                                  dl_dimages_chw[v], nullptr, ctx->stream));
            } else {
                GSR_HIP(ctx, launch_l1_grad(images_chw[v], targets_chw[v], 3 * (int64_t)c.width * c.height,
                                            dl_dimages_chw[v], ctx->stream));
            }
        }
        // The rerender refreshed the lists and walks the plan's view table points at.
        for (int v = 0; v < n_views; ++v) plan.vb.v[v] = desc_of(states[v], nullptr, dls_c[v]);
        GSR_TRY(bwd_enqueue(ctx, n_views, states, &cfg, plan, false));
        return enqueue_params(ctx, n_views, states, outs, adds);
    });
    if (st != GSR_OK) return bail(st);
    *graph_out = gr;
    return GSR_OK;
}

gsr_status gsr_graph_launch(gsr_ctx *ctx, gsr_graph *graph) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!graph) return fail(ctx, GSR_EINVAL, "graph is null");
    if (graph->device != ctx->device) return fail(ctx, GSR_EINVAL, "graph was captured on another device");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, hipGraphLaunch(graph->exec, ctx->stream));
    return GSR_OK;
}

void gsr_graph_destroy(gsr_ctx *ctx, gsr_graph *graph) {
    if (!graph) return;
    (void)hipSetDevice(graph->device);
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    if (graph->ctx)
        for (void *p : graph->owned) graph->ctx->pool->release(p);
    delete graph;
}

gsr_status gsr_fwd_release(gsr_ctx *ctx, gsr_fwd *st) {
    if (!ctx || !st) return GSR_EINVAL;
    for (void *p : st->owned) ctx->pool->release(p);
    delete st;
    return GSR_OK;
}

gsr_status gsr_fwd_stats(const gsr_fwd *st, gsr_fwd_stats_t *out) {
    if (!st || !out) return GSR_EINVAL;
    out->n = st->n;
    out->n_visible = st->p_known ? st->n_visible : -1;
    out->n_pairs = st->p_known ? st->P : -1;
    out->grid_x = st->dcam.grid_x;
    out->grid_y = st->dcam.grid_y;
    out->tile = st->config.tile;
    return GSR_OK;
}

gsr_status gsr_fwd_export(gsr_ctx *ctx, const gsr_fwd *st, const gsr_fwd_export_t *d) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st || !d) return fail(ctx, GSR_EINVAL, "null argument");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t n = st->n, hw = (int64_t)st->camera.width * st->camera.height;
    if (n > 0) {
        GSR_HIP(ctx, launch_export_rec(st->radius, st->rec, n, d->mean2d, d->conic_opacity, d->rgb, d->depth, s));
        if (d->radius) GSR_HIP(ctx, hipMemcpyAsync(d->radius, st->radius, n * 4, hipMemcpyDeviceToDevice, s));
        if (d->tiles_touched)
            GSR_HIP(ctx, hipMemcpyAsync(d->tiles_touched, st->tiles_touched, n * 4, hipMemcpyDeviceToDevice, s));
        if (d->clamp_mask) GSR_HIP(ctx, hipMemcpyAsync(d->clamp_mask, st->clamp_mask, n, hipMemcpyDeviceToDevice, s));
        if (d->acc) {
            if (!st->acc) return fail(ctx, GSR_ESTATE, "no backward has run on this state");
            GSR_HIP(ctx, launch_export_acc(st->radius, st->rec, n, st->acc, st->acc_f64, d->acc, s));
        }
    }
    if (d->sorted_ids && !st->p_known)
        return fail(ctx, GSR_ESTATE, "pair count unknown after a capacity-mode render: call gsr_fwd_sync");
    if (d->sorted_ids && st->P > 0)
        GSR_HIP(ctx, hipMemcpyAsync(d->sorted_ids, st->sorted_pair_id, st->P * 4, hipMemcpyDeviceToDevice, s));
    if (d->ranges)
        GSR_HIP(ctx, hipMemcpyAsync(d->ranges, st->ranges, st->n_tiles * 8, hipMemcpyDeviceToDevice, s));
    if (d->T_final) GSR_HIP(ctx, hipMemcpyAsync(d->T_final, st->T_final, hw * 4, hipMemcpyDeviceToDevice, s));
    if (d->n_contrib) GSR_HIP(ctx, hipMemcpyAsync(d->n_contrib, st->n_contrib, hw * 4, hipMemcpyDeviceToDevice, s));
    return GSR_OK;
}

gsr_status gsr_bwd_counters(gsr_ctx *ctx, const gsr_fwd *st, gsr_bwd_counters_t *out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st || !out) return fail(ctx, GSR_EINVAL, "null argument");
    if (!st->counters_valid || !st->counters)
        return fail(ctx, GSR_ESTATE, "the last backward did not run with GSR_FLAG_DEBUG_COUNTERS");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    unsigned long long h[75];
    GSR_HIP(ctx, hipMemcpyAsync(h, st->counters, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    out->evaluated = h[0];
    out->active = h[1];
    out->wave_entries = h[2];
    out->reduced = h[3];
    out->plain_lanes = h[4];
    out->lane_atomics = h[5];
    out->atomic_instrs = h[6];
    for (int i = 0; i < 65; ++i) out->hist[i] = h[7 + i];
    out->visited = h[72];
    out->max_wave_visits = h[73];
    out->walked = h[74];
    return GSR_OK;
}

gsr_status gsr_ctx_stage_times(gsr_ctx *ctx, gsr_stage_times_t *out) {
    if (!ctx || !out) return GSR_EINVAL;
    ctx->err.clear();
    std::memset(out, 0, sizeof(*out));
    if (!ctx->timing_render && !ctx->timing_bwd) return fail(ctx, GSR_ESTATE, "no timed call");
    const auto el = [&](int a, int b, float *dst) -> hipError_t {
        hipError_t e = hipEventSynchronize(ctx->ev[b]);
        if (e != hipSuccess) return e;
        return hipEventElapsedTime(dst, ctx->ev[a], ctx->ev[b]);
    };
    if (ctx->timing_render) {
        GSR_HIP(ctx, el(EV_R0, EV_R1, &out->preprocess));
        GSR_HIP(ctx, el(EV_R1, EV_R2, &out->depth_sort));
        GSR_HIP(ctx, el(EV_R2, EV_R3, &out->scan_emit));
        GSR_HIP(ctx, el(EV_R3, EV_R4, &out->tile_sort));
        GSR_HIP(ctx, el(EV_R4, EV_R5, &out->ranges));
        GSR_HIP(ctx, el(EV_R5, EV_R6, &out->composite_fwd));
    }
    if (ctx->timing_bwd) {
        GSR_HIP(ctx, el(EV_B0, EV_B1, &out->zero_acc));
        GSR_HIP(ctx, el(EV_B1, EV_B2, &out->composite_bwd));
        GSR_HIP(ctx, el(EV_B2, EV_B3, &out->preprocess_bwd));
    }
    return GSR_OK;
}

gsr_status gsr_l1_grad(gsr_ctx *ctx, const float *image, const float *target, int64_t count, float *dl_dimage) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (count < 0 || (count > 0 && (!image || !target || !dl_dimage))) return fail(ctx, GSR_EINVAL, "bad arguments");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, launch_l1_grad(image, target, count, dl_dimage, ctx->stream));
    return GSR_OK;
}

gsr_status gsr_l1_dssim_grad(gsr_ctx *ctx, const float *image, const float *target, int32_t height, int32_t width,
                             float lambda, float *dl_dimage, float *loss) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (height < 1 || width < 1 || height > 16384 || width > 16384 || !image || !target || !dl_dimage)
        return fail(ctx, GSR_EINVAL, "bad arguments");
    if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(ctx, GSR_EINVAL, "lambda outside [0, 1]");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    const size_t n = 3 * (size_t)height * width;
    TempBuf t0, t1, t2, t3;
    float *dmu = nullptr, *dexx = nullptr, *dexy = nullptr, *sums = nullptr;
    GSR_TRY(temp_alloc(ctx, t0, &dmu, n));
    GSR_TRY(temp_alloc(ctx, t1, &dexx, n));
    GSR_TRY(temp_alloc(ctx, t2, &dexy, n));
    GSR_TRY(temp_alloc(ctx, t3, &sums, dssim_partial_count(3, width, height)));
    GSR_HIP(ctx, launch_l1_dssim_grad(image, target, 3, width, height, lambda, dmu, dexx, dexy, sums, dl_dimage, loss,
                                      ctx->stream));
    return GSR_OK;
}

gsr_status gsr_microbench(gsr_ctx *ctx, int32_t kind, int64_t bytes, int32_t reps, double *ms_per_launch,
                          double *ops_per_launch) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (kind < GSR_MB_COPY || kind > GSR_MB_GATHER48) return fail(ctx, GSR_EINVAL, "bad kind");
    if (bytes < (1 << 20) || bytes > (int64_t(1) << 32) || (bytes & (bytes - 1)))
        return fail(ctx, GSR_EINVAL, "bytes must be a power of two in [1 MiB, 4 GiB]");
    if (reps < 1 || reps > 100 || !ms_per_launch || !ops_per_launch) return fail(ctx, GSR_EINVAL, "bad arguments");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    TempBuf t;
    uint8_t *buf = nullptr;
    GSR_TRY(temp_alloc(ctx, t, &buf, (size_t)bytes));
    GSR_HIP(ctx, hipMemsetAsync(buf, 0, (size_t)bytes, ctx->stream));
    int64_t ops = 0;
    GSR_HIP(ctx, launch_microbench(kind, buf, bytes, &ops, ctx->stream)); // untimed
    std::vector<hipEvent_t> ev(reps + 1, nullptr);
    gsr_status rc = GSR_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(ctx, GSR_EHIP, "hipEventCreate failed");
    std::vector<double> ms;
    if (rc == GSR_OK && hipEventRecord(ev[0], ctx->stream) != hipSuccess) rc = fail(ctx, GSR_EHIP, "event record");
    for (int r = 0; r < reps && rc == GSR_OK; ++r) {
        if (launch_microbench(kind, buf, bytes, &ops, ctx->stream) != hipSuccess ||
            hipEventRecord(ev[r + 1], ctx->stream) != hipSuccess)
            rc = fail(ctx, GSR_EHIP, "launch failed");
    }
    if (rc == GSR_OK && hipEventSynchronize(ev[reps]) != hipSuccess) rc = fail(ctx, GSR_EHIP, "synchronize failed");
    for (int r = 0; r < reps && rc == GSR_OK; ++r) {
        float m = 0.0f;
        if (hipEventElapsedTime(&m, ev[r], ev[r + 1]) != hipSuccess) rc = fail(ctx, GSR_EHIP, "elapsed time");
        ms.push_back(m);
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != GSR_OK) return rc;
    std::sort(ms.begin(), ms.end());
    *ms_per_launch = ms[ms.size() / 2];
    *ops_per_launch = (double)ops;
    return GSR_OK;
}

gsr_status gsr_wave_reduce_selftest(gsr_ctx *ctx, const float *vals, const uint8_t *active, int32_t n_waves,
                                    int32_t mode, int32_t threshold, int32_t lane_split, float *sums,
                                    uint64_t *lane_atomics) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (n_waves < 0 || n_waves > (1 << 24) || (n_waves > 0 && (!vals || !active)) || !sums || !lane_atomics)
        return fail(ctx, GSR_EINVAL, "bad arguments");
    if (mode != GSR_BWD_PLAIN_ATOMIC && mode != GSR_BWD_WAVE_REDUCE && mode != GSR_BWD_SERIAL_REDUCE)
        return fail(ctx, GSR_EINVAL, "bad mode");
    if (threshold < 0 || threshold > 65) return fail(ctx, GSR_EINVAL, "bad threshold");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(sums), 0u, 9, ctx->stream));
    GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(lane_atomics), 0u, 2, ctx->stream));
    GSR_HIP(ctx, launch_wave_reduce_selftest(vals, active, n_waves, mode, threshold < 1 ? 1 : threshold, lane_split,
                                             sums, reinterpret_cast<unsigned long long *>(lane_atomics),
                                             ctx->stream));
    return GSR_OK;
}

} // extern "C"

namespace {

gsr_status check_space(gsr_ctx *ctx, const gsr_tune_space *sp) {
    if (!sp) return fail(ctx, GSR_EINVAL, "tune space is null");
    if (sp->n_tiles < 1 || sp->n_tiles > 3 || sp->n_batches < 1 || sp->n_batches > 3 || sp->n_thresholds < 1 ||
        sp->n_thresholds > 12 || sp->reps < 1 || sp->reps > 100)
        return fail(ctx, GSR_EINVAL, "tune space sizes out of range");
    for (int i = 0; i < sp->n_tiles; ++i)
        if (sp->tiles[i] != 8 && sp->tiles[i] != 16 && sp->tiles[i] != 32)
            return fail(ctx, GSR_EINVAL, "tile %d not in {8,16,32}", sp->tiles[i]);
    for (int i = 0; i < sp->n_batches; ++i)
        if (sp->batches[i] != 64 && sp->batches[i] != 128 && sp->batches[i] != 256)
            return fail(ctx, GSR_EINVAL, "lds batch %d not in {64,128,256}", sp->batches[i]);
    for (int i = 0; i < sp->n_thresholds; ++i)
        if (sp->thresholds[i] < 1 || sp->thresholds[i] > 65)
            return fail(ctx, GSR_EINVAL, "threshold %d outside 1..65", sp->thresholds[i]);
    bool any = false;
    for (int i = 0; i < sp->n_tiles; ++i)
        for (int j = 0; j < sp->n_batches; ++j) any = any || sp->batches[j] <= sp->tiles[i] * sp->tiles[i];
    if (!any) return fail(ctx, GSR_EINVAL, "no (tile, lds batch) pair with batch <= tile*tile");
    return GSR_OK;
}

float median_of(std::vector<float> v) {
    std::sort(v.begin(), v.end());
    return v[v.size() / 2];
}

// Pool buffers and events of one tuning run, returned when it ends.
struct TuneScratch {
    gsr_ctx *ctx;
    std::vector<void *> bufs;
    hipEvent_t ev[2] = {nullptr, nullptr};
    gsr_fwd *sts[kMaxViews] = {};
    int nv = 0;
    explicit TuneScratch(gsr_ctx *c) : ctx(c) {}
    void release_states() {
        for (int v = 0; v < nv; ++v)
            if (sts[v]) gsr_fwd_release(ctx, sts[v]);
        for (auto &p : sts) p = nullptr;
    }
    ~TuneScratch() {
        release_states();
        for (void *p : bufs) ctx->pool->release(p);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    template <typename T>
    gsr_status alloc(T **p, size_t count) {
        GSR_TRY(pool_alloc(ctx, nullptr, p, count));
        bufs.push_back(*p);
        return GSR_OK;
    }
};

} // namespace

struct gsr_tuner {
    gsr_tune_space space{};
    int32_t every = 1;
    int64_t iter = 0;
    gsr_config best{};
};

extern "C" {

gsr_status gsr_autotune(gsr_ctx *ctx, int32_t n_views, const gsr_scene *scenes, const gsr_camera *cameras,
                        const float *const *dl_dimages_chw, const gsr_tune_space *space, gsr_config *best,
                        gsr_tune_entry *entries, int32_t max_entries, int32_t *n_entries) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (n_views < 1 || n_views > GSR_MAX_BATCH) return fail(ctx, GSR_EINVAL, "n_views %d outside 1..16", n_views);
    if (!scenes || !cameras || !best) return fail(ctx, GSR_EINVAL, "null argument");
    if (max_entries < 0 || (max_entries > 0 && !entries)) return fail(ctx, GSR_EINVAL, "bad entries buffer");
    GSR_TRY(check_space(ctx, space));
    const int32_t flags = space->flags & ~(GSR_FLAG_STAGE_TIMING | GSR_FLAG_DEBUG_COUNTERS);
    for (int v = 0; v < n_views; ++v) {
        if (gsr_validate_scene(&scenes[v]) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid scene (view %d)", v);
        if (gsr_validate_camera(&cameras[v]) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid camera (view %d)", v);
        for (int i = 0; i < space->n_tiles; ++i) {
            const gsr_config c{space->tiles[i], 64, GSR_BWD_WAVE_REDUCE, 1, flags};
            if (gsr_validate_config(&c, &cameras[v]) != GSR_OK)
                return fail(ctx, GSR_EINVAL, "tune flags or tile %d invalid for view %d", space->tiles[i], v);
        }
    }
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    TuneScratch sc(ctx);
    sc.nv = n_views;
    for (auto &e : sc.ev) GSR_HIP(ctx, hipEventCreate(&e));
    // Scratch images, gradient images and outputs (views of one scene share outputs, which
    // sums their gradients as a training step over the batch would).
    float *images[kMaxViews] = {};
    const float *dls[kMaxViews] = {};
    gsr_grads outs[kMaxViews] = {};
    int adds[kMaxViews] = {};
    for (int v = 0; v < n_views; ++v) {
        const size_t hw = (size_t)cameras[v].width * cameras[v].height;
        GSR_TRY(sc.alloc(&images[v], 3 * hw));
        if (dl_dimages_chw && dl_dimages_chw[v]) {
            dls[v] = dl_dimages_chw[v];
        } else {
            float *d = nullptr;
            GSR_TRY(sc.alloc(&d, 3 * hw));
            const float c = 1e-3f;
            uint32_t bits;
            std::memcpy(&bits, &c, 4);
            GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(d), bits, 3 * hw, s));
            dls[v] = d;
        }
        int shared = -1;
        for (int u = 0; u < v; ++u)
            if (scenes[u].means3d == scenes[v].means3d && scenes[u].n == scenes[v].n &&
                scenes[u].sh_degree == scenes[v].sh_degree)
                shared = u;
        if (shared >= 0) {
            outs[v] = outs[shared];
            adds[v] = 1;
            continue;
        }
        const size_t n = scenes[v].n > 0 ? scenes[v].n : 1, K = (size_t)(scenes[v].sh_degree + 1) * (scenes[v].sh_degree + 1);
        GSR_TRY(sc.alloc(&outs[v].means3d, 3 * n));
        GSR_TRY(sc.alloc(&outs[v].log_scales, 3 * n));
        GSR_TRY(sc.alloc(&outs[v].quats, 4 * n));
        GSR_TRY(sc.alloc(&outs[v].opacity_logits, n));
        GSR_TRY(sc.alloc(&outs[v].sh, 3 * K * n));
    }
    const auto timed = [&](float *ms, auto &&work) -> gsr_status {
        GSR_HIP(ctx, hipEventRecord(sc.ev[0], s));
        GSR_TRY(work());
        GSR_HIP(ctx, hipEventRecord(sc.ev[1], s));
        GSR_HIP(ctx, hipEventSynchronize(sc.ev[1]));
        GSR_HIP(ctx, hipEventElapsedTime(ms, sc.ev[0], sc.ev[1]));
        return GSR_OK;
    };
    int32_t count = 0;
    float best_ms = 0.0f;
    bool have = false;
    for (int ti = 0; ti < space->n_tiles; ++ti) {
        for (int bi = 0; bi < space->n_batches; ++bi) {
            const int tile = space->tiles[ti], lb = space->batches[bi];
            if (lb > tile * tile) continue;
            gsr_config cfg{tile, lb, GSR_BWD_WAVE_REDUCE, 1, flags};
            // One untimed run first: it fills the pool for this tile size.
            std::vector<float> rt;
            for (int r = 0; r <= space->reps; ++r) {
                sc.release_states();
                float ms = 0.0f;
                GSR_TRY(timed(&ms, [&] { return render_views(ctx, n_views, scenes, cameras, &cfg, images, sc.sts); }));
                if (r > 0) rt.push_back(ms);
            }
            const float render_ms = median_of(rt);
            for (int hi = 0; hi < space->n_thresholds; ++hi) {
                cfg.reduce_threshold = space->thresholds[hi];
                std::vector<float> bt;
                for (int r = 0; r <= space->reps; ++r) {
                    float ms = 0.0f;
                    GSR_TRY(timed(&ms, [&] {
                        GSR_TRY(bwd_views(ctx, n_views, sc.sts, dls, &cfg, false));
                        return enqueue_params(ctx, n_views, sc.sts, outs, adds);
                    }));
                    if (r > 0) bt.push_back(ms);
                }
                const float bwd_ms = median_of(bt);
                if (count < max_entries) entries[count] = gsr_tune_entry{cfg, render_ms, bwd_ms};
                ++count;
                if (!have || render_ms + bwd_ms < best_ms) {
                    have = true;
                    best_ms = render_ms + bwd_ms;
                    *best = cfg;
                }
            }
        }
    }
    if (n_entries) *n_entries = count < max_entries ? count : max_entries;
    return GSR_OK;
}

gsr_status gsr_tuner_create(const gsr_tune_space *space, int32_t every, gsr_tuner **out) {
    if (!out) return GSR_EINVAL;
    *out = nullptr;
    if (every < 1 || check_space(nullptr, space) != GSR_OK) return GSR_EINVAL;
    gsr_tuner *t = new (std::nothrow) gsr_tuner();
    if (!t) return GSR_ENOMEM;
    t->space = *space;
    t->every = every;
    *out = t;
    return GSR_OK;
}

gsr_status gsr_tuner_next(gsr_ctx *ctx, gsr_tuner *tuner, int32_t n_views, const gsr_scene *scenes,
                          const gsr_camera *cameras, const float *const *dl_dimages_chw, gsr_config *config_out,
                          int32_t *retuned) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!tuner || !config_out) return fail(ctx, GSR_EINVAL, "null argument");
    int32_t did = 0;
    if (tuner->iter % tuner->every == 0) {
        GSR_TRY(gsr_autotune(ctx, n_views, scenes, cameras, dl_dimages_chw, &tuner->space, &tuner->best, nullptr, 0,
                             nullptr));
        did = 1;
    }
    ++tuner->iter;
    *config_out = tuner->best;
    if (retuned) *retuned = did;
    return GSR_OK;
}

void gsr_tuner_destroy(gsr_tuner *tuner) { delete tuner; }

} // extern "C"

