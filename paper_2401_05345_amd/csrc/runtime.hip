// Host runtime of libgsr: the C ABI of gsr.h, argument checks, a caching
// device-memory pool, and the orchestration of the kernels on the context's
// stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

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
    d.limx = 1.3f * (0.5f * (float)c.width) / c.fx;
    d.limy = 1.3f * (0.5f * (float)c.height) / c.fy;
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
    if (cf->bwd_mode != GSR_BWD_PLAIN_ATOMIC && cf->bwd_mode != GSR_BWD_WAVE_REDUCE) return GSR_EINVAL;
    if (cf->reduce_threshold < 0 || cf->reduce_threshold > 65) return GSR_EINVAL;
    if (cf->flags & ~(GSR_FLAG_DEBUG_COUNTERS | GSR_FLAG_XCD_REMAP | GSR_FLAG_STAGE_TIMING |
                      GSR_FLAG_LANE_SPLIT_ATOMICS | GSR_FLAG_NO_TILE_ORDER))
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
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return GSR_EHIP;
        }
        ctx->own_stream = true;
    }
    ctx->pool = new (std::nothrow) Pool(device);
    void *hp = nullptr;
    if (!ctx->pool || hipHostMalloc(&hp, 256, hipHostMallocDefault) != hipSuccess) {
        gsr_ctx_destroy(ctx);
        return GSR_ENOMEM;
    }
    ctx->host_pinned = static_cast<uint32_t *>(hp);
    for (auto &e : ctx->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            gsr_ctx_destroy(ctx);
            return GSR_EHIP;
        }
    }
    *out = ctx;
    return GSR_OK;
}

void gsr_ctx_destroy(gsr_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx->pool;
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char *gsr_ctx_last_error(const gsr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gsr_status gsr_ctx_set_stream(gsr_ctx *ctx, void *hip_stream) {
    if (!ctx) return GSR_EINVAL;
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->own_stream) {
        if (hip_stream) {
            (void)hipStreamDestroy(ctx->stream);
            ctx->own_stream = false;
            ctx->stream = static_cast<hipStream_t>(hip_stream);
        }
    } else if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        GSR_HIP(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    return GSR_OK;
}

gsr_status gsr_render(gsr_ctx *ctx, const gsr_scene *scene, const gsr_camera *camera, const gsr_config *config,
                      float *image_chw, gsr_fwd **state_out) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!state_out) return fail(ctx, GSR_EINVAL, "state_out is null");
    *state_out = nullptr;
    if (gsr_validate_scene(scene) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid scene");
    if (gsr_validate_camera(camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid camera");
    if (gsr_validate_config(config, camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid config");
    if (!image_chw) return fail(ctx, GSR_EINVAL, "image is null");
    GSR_HIP(ctx, hipSetDevice(ctx->device));

    gsr_fwd *st = new (std::nothrow) gsr_fwd();
    if (!st) return fail(ctx, GSR_ENOMEM, "host allocation failed");
    st->scene = *scene;
    st->camera = *camera;
    st->config = *config;
    st->dcam = make_dev_camera(*camera, config->tile);
    st->n = scene->n;
    st->n_tiles = (int64_t)st->dcam.grid_x * st->dcam.grid_y;
    const int64_t n = st->n;
    const int64_t hw = (int64_t)camera->width * camera->height;
    hipStream_t s = ctx->stream;
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_render = tm;
    auto bail = [&](gsr_status code) {
        gsr_fwd_release(ctx, st);
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

    const int64_t nn = n > 0 ? n : 1;
    GSR_RT(pool_alloc(ctx, st, &st->rec, 3 * nn));
    GSR_RT(pool_alloc(ctx, st, &st->radius, nn));
    GSR_RT(pool_alloc(ctx, st, &st->tiles_touched, nn));
    GSR_RT(pool_alloc(ctx, st, &st->clamp_mask, nn));
    GSR_RT(pool_alloc(ctx, st, &st->depth_key, nn));
    GSR_RT(pool_alloc(ctx, st, &st->ids, nn));
    GSR_RT(pool_alloc(ctx, st, &st->key_alt, nn));
    GSR_RT(pool_alloc(ctx, st, &st->ids_alt, nn));
    GSR_RT(pool_alloc(ctx, st, &st->offsets, nn + 1));
    GSR_RT(pool_alloc(ctx, st, &st->ranges, st->n_tiles));
    GSR_RT(pool_alloc(ctx, st, &st->T_final, hw));
    GSR_RT(pool_alloc(ctx, st, &st->n_contrib, hw));

    uint32_t *hist = nullptr, *partials = nullptr, *total = nullptr;
    GSR_RT(pool_alloc(ctx, st, &total, 4));

    mark(ctx, tm, EV_R0);
    // a1: projection
    GSR_RH(launch_preprocess_fwd(*scene, st->dcam, st->rec, st->radius, st->tiles_touched, st->depth_key, st->ids,
                                 st->clamp_mask, s));
    mark(ctx, tm, EV_R1);
    // a2/a3 (depth digits): sort Gaussians by fp32 depth; stable, so ties keep index order.
    int which = 0;
    if (n > 1) {
        const size_t hc = radix_hist_count(n), pc = scan_partial_count((int64_t)hc);
        GSR_RT(pool_alloc(ctx, st, &hist, hc));
        GSR_RT(pool_alloc(ctx, st, &partials, pc));
        GSR_RH(radix_sort_pairs(st->depth_key, st->ids, st->key_alt, st->ids_alt, n, 32, hist, partials, &which, s));
    }
    st->sorted_ids_by_depth = which ? st->ids_alt : st->ids;
    mark(ctx, tm, EV_R2);
    // a2: pair offsets in depth order, total P read back to size the pair buffers.
    {
        uint32_t *sp = nullptr;
        GSR_RT(pool_alloc(ctx, st, &sp, scan_partial_count(nn) + 8));
        GSR_RH(device_exclusive_scan(st->tiles_touched, st->sorted_ids_by_depth, st->offsets, n, total, sp, s));
        GSR_RH(launch_count_positive(st->radius, n, total + 1, s));
        GSR_RH(hipMemcpyAsync(ctx->host_pinned, total, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        GSR_RH(hipStreamSynchronize(s));
        st->P = n > 0 ? (int64_t)ctx->host_pinned[0] : 0;
        st->n_visible = n > 0 ? (int64_t)ctx->host_pinned[1] : 0;
    }
    const int64_t P = st->P;
    const int64_t PP = P > 0 ? P : 1;
    GSR_RT(pool_alloc(ctx, st, &st->pair_tile, PP));
    GSR_RT(pool_alloc(ctx, st, &st->pair_id, PP));
    GSR_RT(pool_alloc(ctx, st, &st->pair_tile_alt, PP));
    GSR_RT(pool_alloc(ctx, st, &st->pair_id_alt, PP));
    GSR_RH(launch_emit_pairs(n, st->sorted_ids_by_depth, st->offsets, st->rec, st->radius, st->dcam, st->pair_tile,
                             st->pair_id, s));
    mark(ctx, tm, EV_R3);
    // a3 (tile digits): stable sort of the pairs by tile.
    which = 0;
    if (P > 1) {
        const size_t hc = radix_hist_count(P), pc = scan_partial_count((int64_t)hc);
        uint32_t *h2 = nullptr, *p2 = nullptr;
        GSR_RT(pool_alloc(ctx, st, &h2, hc));
        GSR_RT(pool_alloc(ctx, st, &p2, pc));
        GSR_RH(radix_sort_pairs(st->pair_tile, st->pair_id, st->pair_tile_alt, st->pair_id_alt, P,
                                bits_for(st->n_tiles), h2, p2, &which, s));
    }
    uint32_t *sorted_tile = which ? st->pair_tile_alt : st->pair_tile;
    st->sorted_pair_id = which ? st->pair_id_alt : st->pair_id;
    mark(ctx, tm, EV_R4);
    // a4: per-tile ranges
    GSR_RH(launch_tile_ranges(P, sorted_tile, st->ranges, st->n_tiles, s));
    mark(ctx, tm, EV_R5);
    // a5: forward composite, tiles launched longest list first; it records each tile's
    // deepest n_contrib, which orders the backward's tiles the same way.
    const bool ordered = !(config->flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER));
    if (ordered) {
        GSR_RT(pool_alloc(ctx, st, &st->order_fwd, st->n_tiles));
        GSR_RT(pool_alloc(ctx, st, &st->order_bwd, st->n_tiles));
        GSR_RT(pool_alloc(ctx, st, &st->tile_walk, st->n_tiles));
        GSR_RH(launch_order_tiles(nullptr, st->ranges, st->n_tiles, st->order_fwd, s));
    }
    FwdArgs fa{st->ranges, st->sorted_pair_id, st->rec, image_chw, st->T_final, st->n_contrib,
               ordered ? st->order_fwd : nullptr, ordered ? st->tile_walk : nullptr};
    GSR_RH(launch_composite_fwd(st->dcam, config->lds_batch, (config->flags & GSR_FLAG_XCD_REMAP) ? 1 : 0, fa, s));
    if (ordered) GSR_RH(launch_order_tiles(st->tile_walk, nullptr, st->n_tiles, st->order_bwd, s));
    mark(ctx, tm, EV_R6);
#undef GSR_RT
#undef GSR_RH
    *state_out = st;
    return GSR_OK;
}

static gsr_status bwd_composite(gsr_ctx *ctx, gsr_fwd *st, const float *dl, const gsr_config *cfg, bool tm) {
    const int64_t n = st->n;
    const int64_t nn = n > 0 ? n : 1;
    hipStream_t s = ctx->stream;
    if (!st->acc) GSR_TRY(pool_alloc(ctx, st, &st->acc, (size_t)nn * GSR_ACC_STRIDE));
    const bool count = (cfg->flags & GSR_FLAG_DEBUG_COUNTERS) != 0;
    if (count && !st->counters) GSR_TRY(pool_alloc(ctx, st, &st->counters, 80));
    mark(ctx, tm, EV_B0);
    GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(st->acc), 0u, nn * GSR_ACC_STRIDE, s));
    if (count) GSR_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(st->counters), 0u, 160, s));
    mark(ctx, tm, EV_B1);
    BwdArgs a{};
    a.ranges = st->ranges;
    a.sorted_ids = st->sorted_pair_id;
    a.rec = st->rec;
    a.dl_dimage = dl;
    a.T_final = st->T_final;
    a.n_contrib = st->n_contrib;
    a.acc = st->acc;
    a.counters = st->counters;
    a.threshold = cfg->reduce_threshold < 1 ? 1 : cfg->reduce_threshold;
    a.order = (cfg->flags & (GSR_FLAG_XCD_REMAP | GSR_FLAG_NO_TILE_ORDER)) ? nullptr : st->order_bwd;
    GSR_HIP(ctx, launch_composite_bwd(st->dcam, cfg->lds_batch, (cfg->flags & GSR_FLAG_XCD_REMAP) ? 1 : 0,
                                      cfg->bwd_mode, count, (cfg->flags & GSR_FLAG_LANE_SPLIT_ATOMICS) != 0, a, s));
    mark(ctx, tm, EV_B2);
    st->counters_valid = count;
    return GSR_OK;
}

static gsr_status check_bwd_args(gsr_ctx *ctx, gsr_fwd *st, const float *dl, const gsr_config **cfg) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st) return fail(ctx, GSR_EINVAL, "state is null");
    if (!dl) return fail(ctx, GSR_EINVAL, "dl_dimage is null");
    if (!*cfg) *cfg = &st->config;
    if ((*cfg)->tile != st->config.tile) return fail(ctx, GSR_EINVAL, "backward tile differs from the render's");
    if (gsr_validate_config(*cfg, &st->camera) != GSR_OK) return fail(ctx, GSR_EINVAL, "invalid config");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    return GSR_OK;
}

static gsr_status check_grads(gsr_ctx *ctx, const gsr_fwd *st, const gsr_grads *out) {
    if (!out) return fail(ctx, GSR_EINVAL, "grads is null");
    if (st->n > 0 && (!out->means3d || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh))
        return fail(ctx, GSR_EINVAL, "a gradient pointer is null");
    return GSR_OK;
}

gsr_status gsr_backward_composite(gsr_ctx *ctx, gsr_fwd *st, const float *dl_dimage_chw, const gsr_config *config) {
    GSR_TRY(check_bwd_args(ctx, st, dl_dimage_chw, &config));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    ctx->timing_bwd = false;
    return bwd_composite(ctx, st, dl_dimage_chw, config, tm);
}

gsr_status gsr_backward_params(gsr_ctx *ctx, gsr_fwd *st, const gsr_grads *out, int accumulate) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (!st) return fail(ctx, GSR_EINVAL, "state is null");
    GSR_TRY(check_grads(ctx, st, out));
    if (!st->acc) return fail(ctx, GSR_ESTATE, "no backward composite has run on this state");
    GSR_HIP(ctx, hipSetDevice(ctx->device));
    GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, st->acc, *out, accumulate ? 1 : 0,
                                       ctx->stream));
    return GSR_OK;
}

gsr_status gsr_backward(gsr_ctx *ctx, gsr_fwd *st, const float *dl_dimage_chw, const gsr_grads *out, int accumulate,
                        const gsr_config *config) {
    GSR_TRY(check_bwd_args(ctx, st, dl_dimage_chw, &config));
    GSR_TRY(check_grads(ctx, st, out));
    const bool tm = (config->flags & GSR_FLAG_STAGE_TIMING) != 0;
    GSR_TRY(bwd_composite(ctx, st, dl_dimage_chw, config, tm));
    GSR_HIP(ctx, launch_preprocess_bwd(st->scene, st->dcam, st->radius, st->acc, *out, accumulate ? 1 : 0,
                                       ctx->stream));
    mark(ctx, tm, EV_B3);
    ctx->timing_bwd = tm;
    return GSR_OK;
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
    out->n_visible = st->n_visible;
    out->n_pairs = st->P;
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
    const auto cp = [&](void *dst, const void *src, size_t bytes, size_t spitch, size_t dpitch, size_t width,
                        size_t rows) -> hipError_t {
        if (!dst || rows == 0) return hipSuccess;
        if (spitch == dpitch && spitch == width) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
        return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, hipMemcpyDeviceToDevice, s);
    };
    if (n > 0) {
        // rec rows are 48 bytes: (u, v, A, B) (C, o, r, g) (b, depth, ., .)
        const float *rec = reinterpret_cast<const float *>(st->rec);
        GSR_HIP(ctx, cp(d->mean2d, rec, 0, 48, 8, 8, n));
        if (d->conic_opacity) {
            GSR_HIP(ctx, hipMemcpy2DAsync(d->conic_opacity, 16, rec + 2, 48, 8, n, hipMemcpyDeviceToDevice, s));
            GSR_HIP(ctx, hipMemcpy2DAsync(d->conic_opacity + 2, 16, rec + 4, 48, 8, n, hipMemcpyDeviceToDevice, s));
        }
        if (d->rgb) {
            GSR_HIP(ctx, hipMemcpy2DAsync(d->rgb, 12, rec + 6, 48, 8, n, hipMemcpyDeviceToDevice, s));
            GSR_HIP(ctx, hipMemcpy2DAsync(d->rgb + 2, 12, rec + 8, 48, 4, n, hipMemcpyDeviceToDevice, s));
        }
        GSR_HIP(ctx, cp(d->depth, rec + 9, 0, 48, 4, 4, n));
        if (d->radius) GSR_HIP(ctx, hipMemcpyAsync(d->radius, st->radius, n * 4, hipMemcpyDeviceToDevice, s));
        if (d->tiles_touched)
            GSR_HIP(ctx, hipMemcpyAsync(d->tiles_touched, st->tiles_touched, n * 4, hipMemcpyDeviceToDevice, s));
        if (d->clamp_mask) GSR_HIP(ctx, hipMemcpyAsync(d->clamp_mask, st->clamp_mask, n, hipMemcpyDeviceToDevice, s));
        if (d->acc) {
            if (!st->acc) return fail(ctx, GSR_ESTATE, "no backward has run on this state");
            GSR_HIP(ctx, hipMemcpyAsync(d->acc, st->acc, n * GSR_ACC_STRIDE * 4, hipMemcpyDeviceToDevice, s));
        }
    }
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
    unsigned long long h[72];
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

gsr_status gsr_wave_reduce_selftest(gsr_ctx *ctx, const float *vals, const uint8_t *active, int32_t n_waves,
                                    int32_t mode, int32_t threshold, int32_t lane_split, float *sums,
                                    uint64_t *lane_atomics) {
    if (!ctx) return GSR_EINVAL;
    ctx->err.clear();
    if (n_waves < 0 || n_waves > (1 << 24) || (n_waves > 0 && (!vals || !active)) || !sums || !lane_atomics)
        return fail(ctx, GSR_EINVAL, "bad arguments");
    if (mode != GSR_BWD_PLAIN_ATOMIC && mode != GSR_BWD_WAVE_REDUCE) return fail(ctx, GSR_EINVAL, "bad mode");
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
