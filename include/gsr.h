/*
 * gsr.h - 3D Gaussian Splatting render and backward pass for AMD MI355X
 * (gfx950), with a per-wavefront choice between a register (cross-lane)
 * reduction plus one lane's atomics and plain per-lane global atomics.
 *
 * The calls follow the problem the paper (DISTWAR, arXiv 2401.05345) states
 * for raster-based differentiable rendering: render a view of a set of
 * learnable primitives, then propagate dL/dimage back to every parameter of
 * every primitive that influenced the image (Background, the differentiable
 * rendering training pipeline and the rasterisation pipeline figure; its
 * steps 1-7). The backward accumulation is the paper's gradient-computation
 * kernel (Motivation, outline of the gradient computation step); the
 * per-wave reduction with a balancing threshold is its SW-B primitive
 * (Detailed Design, "Butterfly Reduction (SW-B)", and Approach, "Scheduling
 * Atomic Updates Between Core and L2"). The rendering math is the published
 * 3D Gaussian Splatting method the paper instruments.
 *
 * Conventions
 *  - Every array pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *    tensor on the context's device) unless marked [host].
 *  - All arrays are dense, row-major, fp32 unless stated; no strides.
 *  - Every call that launches work enqueues it on the context's stream and
 *    returns without waiting, except where "synchronises" is stated.
 *  - No call throws; every call returns a gsr_status. On failure the
 *    context's message (gsr_ctx_last_error) says why. Arguments are checked
 *    on the host before anything is enqueued; on GSR_EINVAL nothing ran.
 *  - A context is used by one host thread at a time.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSR_OK = 0,
    GSR_EINVAL = -1,  /* bad argument; nothing was enqueued */
    GSR_ENOMEM = -2,  /* device or pinned-host allocation failed */
    GSR_EHIP = -3,    /* a HIP runtime call failed; message carries hipGetErrorString */
    GSR_ESTATE = -4,  /* object used in a wrong state (e.g. counters never collected) */
    GSR_EBUDGET = -5  /* a scene does not fit the server's HBM budget */
} gsr_status;

typedef enum {
    GSR_BWD_PLAIN_ATOMIC = 0, /* every active lane issues its own 9 atomic adds */
    GSR_BWD_WAVE_REDUCE = 1,  /* wave reduction + one lane's atomics when active lanes >= threshold */
    GSR_BWD_SERIAL_REDUCE = 2, /* ablation: the sums built one active lane at a time (readlane loop, the
                                  paper's serialised SW-S form) when active lanes >= threshold; lanes 0..8 issue */
    GSR_BWD_BLOCK_REDUCE = 3, /* extension: waves at or above the threshold reduce into LDS; the
                                 block issues one atomic per (tile, Gaussian, value) after each LDS batch */
    GSR_BWD_PLAIN_COMPILER_REDUCE = 4 /* ablation: the plain-atomic kernel's source compiled with the
                                 compiler's own rewrite of atomics to one address (LLVM's atomic
                                 optimizer, DPP strategy): each of the nine adds becomes a reduction over
                                 the active lanes and one lane's atomic. The threshold is ignored and
                                 GSR_FLAG_DEBUG_COUNTERS is rejected (GSR_EINVAL) for this mode */
} gsr_bwd_mode;

enum {
    GSR_FLAG_DEBUG_COUNTERS = 1, /* backward counts wave-entries, active lanes and issued atomics */
    GSR_FLAG_XCD_REMAP = 2,      /* composite kernels map consecutive blocks of one XCD to neighbouring tiles */
    GSR_FLAG_STAGE_TIMING = 4,   /* record HIP events around each stage (gsr_ctx_stage_times) */
    GSR_FLAG_LANE_SPLIT_ATOMICS = 8, /* reduce path: nine lanes each issue one of the 9 sums in one instruction */
    GSR_FLAG_NO_TILE_ORDER = 16,     /* launch tiles in index order instead of longest-work first */
    GSR_FLAG_ACC_F32 = 32            /* fp32 backward accumulators (the paper's setting). Without it the
                                        per-wave sums, kept in fp32 registers, are added into fp64
                                        accumulator rows (one 128-byte row per Gaussian): the result no
                                        longer depends on the order of the atomic adds. */
};

/* Number of floats reserved per Gaussian in the backward accumulators:
 * (dL/du, dL/dv, dL/dA, dL/dB, dL/dC, dL/do, dL/dr, dL/dg, dL/db, pad...). */
#define GSR_ACC_STRIDE 16

/* Learnable scene. n >= 0; sh_degree 0..3, K = (sh_degree+1)^2 coefficients.
 *  means3d [n,3], log_scales [n,3], quats [n,4] as (w,x,y,z) (need not be
 *  unit length; normalised inside, gradients go through the normalisation),
 *  opacity_logits [n], sh [n,K,3] (coefficient k = l*l + l + m, channel last). */
typedef struct {
    int32_t n;
    int32_t sh_degree;
    const float *means3d;
    const float *log_scales;
    const float *quats;
    const float *opacity_logits;
    const float *sh;
} gsr_scene;

/* Pinhole camera, OpenCV axes (+x right, +y down, +z forward). Pixel (x,y)
 * is sampled at (x+0.5, y+0.5). world_to_cam [host] is the row-major 3x4
 * [R|t]; R must be a rotation. Points with fp32 camera depth <= znear are
 * culled. bg is the background colour. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float world_to_cam[12];
    float znear;
    float bg[3];
} gsr_camera;

/* tile: 8, 16 or 32 (pixels per tile side; one workgroup of tile*tile
 * threads per tile). lds_batch: 64, 128 or 256 Gaussian records staged in
 * LDS per round, <= tile*tile. bwd_mode: gsr_bwd_mode. reduce_threshold
 * 0..65: in GSR_BWD_WAVE_REDUCE a wave reduces iff its active-lane count is
 * >= max(threshold, 1); 65 never reduces (same atomics as plain). flags:
 * GSR_FLAG_* bits. */
typedef struct {
    int32_t tile;
    int32_t lds_batch;
    int32_t bwd_mode;
    int32_t reduce_threshold;
    int32_t flags;
} gsr_config;

/* Caller-owned gradient outputs, same shapes as the scene's arrays. */
typedef struct {
    float *means3d;
    float *log_scales;
    float *quats;
    float *opacity_logits;
    float *sh;
} gsr_grads;

typedef struct gsr_ctx gsr_ctx;
typedef struct gsr_fwd gsr_fwd;

/* Host-visible facts about a forward state (filled by a synchronising call). */
typedef struct {
    int64_t n;            /* Gaussians */
    int64_t n_visible;    /* Gaussians with radius > 0 */
    int64_t n_pairs;      /* P: (tile, Gaussian) pairs in the sorted lists */
    int32_t grid_x, grid_y;
    int32_t tile;
} gsr_fwd_stats_t;

/* Destinations for gsr_fwd_export; every pointer is a caller-owned device
 * buffer or NULL to skip it. Sizes: n Gaussians, P pairs, G = grid_x*grid_y
 * tiles, HW pixels.
 *  mean2d [n,2], conic_opacity [n,4] (A,B,C,o), rgb [n,3], depth [n],
 *  radius [n] int32 (0 = culled), tiles_touched [n] uint32,
 *  clamp_mask [n] uint8 (bit c: colour channel c clamped at 0),
 *  sorted_ids [P] uint32 (Gaussian per list entry, tile-major then depth),
 *  ranges [G,2] uint32 half-open [start,end) into sorted_ids,
 *  T_final [HW], n_contrib [HW] uint32 (1-based list position of the last
 *  composited entry, 0 = none), acc [n,GSR_ACC_STRIDE] (the last backward's
 *  accumulators as fp32 gradients in the column order of GSR_ACC_STRIDE,
 *  whatever their precision; rows of culled Gaussians read 0. The composite
 *  accumulates moments of each pixel's dL/do over the pixel offsets, which
 *  the export turns into mean and conic gradients with the state's current
 *  opacities and conics). */
typedef struct {
    float *mean2d;
    float *conic_opacity;
    float *rgb;
    float *depth;
    int32_t *radius;
    uint32_t *tiles_touched;
    uint8_t *clamp_mask;
    uint32_t *sorted_ids;
    uint32_t *ranges;
    float *T_final;
    uint32_t *n_contrib;
    float *acc;
} gsr_fwd_export_t;

/* Debug counters of the last backward run with GSR_FLAG_DEBUG_COUNTERS.
 *  evaluated     E: (pixel, entry) pairs walked with entry <= n_contrib
 *  active        A: pairs that contributed (the paper's participating threads)
 *  wave_entries  (wave, entry) steps with at least one active lane
 *  reduced       W_R: wave-entries that took the reduction path
 *  plain_lanes   A_<: active lanes of wave-entries that issued per-lane atomics
 *  lane_atomics  atomic lane-operations issued (each lane of each atomic instruction)
 *  atomic_instrs atomic instructions issued
 *  hist[c]       wave-entries with c active lanes, c = 0..64 (c = 0 not counted)
 *  visited       (wave, entry) steps the walk took: entries a wave's visit
 *                masks kept, active lanes or not (>= wave_entries)
 *  max_wave_visits  the most entries one wave visited (the longest walk)
 *  walked        P_walk: list entries staged, summed over tiles (each tile's
 *                block walks to its deepest pixel's n_contrib) */
typedef struct {
    uint64_t evaluated, active, wave_entries, reduced, plain_lanes, lane_atomics, atomic_instrs;
    uint64_t hist[65];
    uint64_t visited, max_wave_visits, walked;
} gsr_bwd_counters_t;

/* Milliseconds of the stages of the last gsr_render / gsr_backward with
 * GSR_FLAG_STAGE_TIMING (HIP events on the context stream). zero_acc covers
 * the clearing of the accumulator rows and the building of the backward's
 * tile order; composite_bwd the backward composite launch alone. */
typedef struct {
    float preprocess, depth_sort, scan_emit, tile_sort, ranges, composite_fwd;
    float zero_acc, composite_bwd, preprocess_bwd;
} gsr_stage_times_t;

/* Create a context on `device`. hip_stream: the hipStream_t to enqueue on;
 * NULL means HIP's null stream (where a framework's default stream runs, so
 * the library's work is ordered with the caller's). The library enqueues on
 * no other stream (the one exception: a graph capture from a context on the
 * null stream records on a temporary stream). Returns GSR_EINVAL for a bad
 * device, GSR_EHIP on runtime failure. */
gsr_status gsr_ctx_create(gsr_ctx **out, int device, void *hip_stream);

/* Destroy a context and free all library-owned device memory. Waits for the
 * stream to drain. Forward states must be released before. */
void gsr_ctx_destroy(gsr_ctx *ctx);

/* Message describing the last failure on this context ("" if none). The
 * string is owned by the context and valid until the next call on it. */
const char *gsr_ctx_last_error(const gsr_ctx *ctx);

/* Replace the stream the context enqueues on (NULL = HIP's null stream).
 * Synchronises the old stream first (pooled buffers are reused in one
 * stream order). */
gsr_status gsr_ctx_set_stream(gsr_ctx *ctx, void *hip_stream);

/* Forward pass (3DGS rasterisation: per-Gaussian projection, tile binning
 * with a device radix sort on (tile, depth), front-to-back composite).
 * Defined by: the rendering of the primitives into a 2D image (Background,
 * "Differentiable Rendering for Rasterization Pipelines", steps 1-2 of the
 * rasterisation pipeline figure; the forward pass of the training pipeline
 * figure), which also produces the per-pixel primitive lists the gradient
 * kernel consumes (Motivation, "Atomic Reduction Bottleneck").
 * image_chw [3,H,W] is written. *state_out receives a library-owned state
 * holding the projected Gaussians, the sorted lists, per-tile ranges and
 * per-pixel T_final / n_contrib; it borrows the scene's arrays, which must
 * stay valid and unchanged until gsr_fwd_release. Synchronises once (the
 * number of pairs is read back to size the sort buffers). n = 0 is valid:
 * the image is bg. */
gsr_status gsr_render(gsr_ctx *ctx, const gsr_scene *scene, const gsr_camera *camera,
                      const gsr_config *config, float *image_chw, gsr_fwd **state_out);

/* Backward pass for a forward state: walks every tile list in reverse,
 * accumulates the nine per-Gaussian gradients (2D mean, conic, opacity,
 * colour) with the configured reduction mode, then turns them into
 * gradients of the raw parameters. Defined by: the loss backpropagated to
 * the gradients of every parameter of each primitive that influences the
 * image (Background, rasterisation pipeline figure, steps 4-6). The
 * accumulation is the gradient computation kernel (Motivation, "Atomic
 * Reduction Bottleneck": one thread per pixel walks its list, conditions
 * decide participation, participants add atomically); the wave reduction
 * and its balancing threshold are Approach, "Key Components" (butterfly
 * reduction; scheduling between core and L2) and Detailed Design (SW-B). dl_dimage_chw [3,H,W]. out: caller-owned
 * gradients; accumulate = 0 overwrites, 1 adds. Culled Gaussians get 0 (or
 * keep their value when accumulating). May be called several times per
 * state, with any mode/threshold in `config` (NULL = the render config). */
gsr_status gsr_backward(gsr_ctx *ctx, gsr_fwd *state, const float *dl_dimage_chw,
                        const gsr_grads *out, int accumulate, const gsr_config *config);

/* Only the composite part of the backward: fills the state's accumulators
 * (exported as `acc`). Same arguments as gsr_backward. Defined by: the
 * gradient computation kernel alone (Motivation, "Atomic Reduction
 * Bottleneck"), the step the paper measures. */
gsr_status gsr_backward_composite(gsr_ctx *ctx, gsr_fwd *state, const float *dl_dimage_chw,
                                  const gsr_config *config);

/* Only the per-Gaussian part: raw-parameter gradients from the state's
 * accumulators of the last gsr_backward_composite. Defined by: step 6 of the
 * rasterisation pipeline figure (gradients for all the parameters of each
 * primitive), through the 3D Gaussian Splatting projection. Writes every
 * Gaussian's rows of the five outputs (zeros for culled Gaussians when
 * accumulate = 0); outputs need no alignment (16-byte aligned ones are
 * written with wider stores). */
gsr_status gsr_backward_params(gsr_ctx *ctx, gsr_fwd *state, const gsr_grads *out, int accumulate);

/* Largest state gsr_backward_noalloc takes: Gaussians, and tiles of the view. */
#define GSR_NOALLOC_MAX_GAUSSIANS 524288
#define GSR_NOALLOC_MAX_TILES 65536

/* gsr_backward without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, kernels and results as gsr_backward;
 * the per-Gaussian accumulator rows (and, when the state has none cached, the
 * backward's tile order) live in a fixed scratch area that the library holds
 * on each GPU it runs on until the process ends: 64 MiB of rows
 * (GSR_NOALLOC_MAX_GAUSSIANS x GSR_ACC_STRIDE doubles) plus 512 KiB of tile
 * order. The rows the kernels add into are cleared at the start of every
 * call; the area keeps the last call's sums afterwards.
 * Errors: GSR_EINVAL (before anything is enqueued) when the state has more
 * than GSR_NOALLOC_MAX_GAUSSIANS Gaussians or GSR_NOALLOC_MAX_TILES tiles, or
 * when config asks for GSR_FLAG_DEBUG_COUNTERS (their buffer is allocated);
 * GSR_EHIP when the scratch area's address could not be obtained at context
 * creation. Every call on one GPU shares that GPU's area: calls that overlap
 * on one GPU (two streams or two host threads) race and must be serialised by
 * the caller. The sums stay in the shared area, so gsr_backward_params and
 * the `acc` export of this state do not see them. */
gsr_status gsr_backward_noalloc(gsr_ctx *ctx, gsr_fwd *state, const float *dl_dimage_chw,
                                const gsr_grads *out, int accumulate, const gsr_config *config);

/* Most views one batched call takes. */
#define GSR_MAX_BATCH 16

/* Forward pass over n_views (1..GSR_MAX_BATCH) views at once (the training
 * loop repeats the forward pass for images from different view points:
 * Background, "Differentiable Rendering for 3D Scene Reconstruction"): scenes[i] seen
 * by cameras[i] into images_chw[i] [3,H_i,W_i], states_out[i] receiving view
 * i's state (as gsr_render). Views may share a scene and may differ in
 * resolution and Gaussian count; one config (tile, LDS batch, flags) serves
 * all. Every stage runs for all views before the next, the pair counts of
 * all views are read back with ONE synchronisation, and the composite is one
 * launch over every (view, tile) pair of the batch, longest tile first
 * (GSR_FLAG_NO_TILE_ORDER: view-major index order; GSR_FLAG_XCD_REMAP has no
 * effect on a batch of more than one view). Results equal gsr_render's for
 * each view. On failure no state is returned. */
gsr_status gsr_render_batch(gsr_ctx *ctx, int32_t n_views, const gsr_scene *scenes, const gsr_camera *cameras,
                            const gsr_config *config, float *const *images_chw, gsr_fwd **states_out);

/* Backward pass over n_views (1..GSR_MAX_BATCH) forward states at once (from
 * gsr_render or gsr_render_batch, all rendered with config->tile): one
 * composite launch over every (view, tile) pair, then each view's
 * per-Gaussian part. dl_dimages_chw[i] [3,H_i,W_i]; outs[i] view i's
 * gradient outputs. Views whose outs are identical (all five pointers
 * equal) are summed: the first of them writes (or adds, when accumulate is
 * 1), later ones add. outs that share some but not all pointers are
 * rejected (GSR_EINVAL). With GSR_FLAG_DEBUG_COUNTERS the counters of the
 * whole launch are kept on states[0]. config NULL = states[0]'s render
 * config. */
gsr_status gsr_backward_batch(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states,
                              const float *const *dl_dimages_chw, const gsr_grads *outs, int accumulate,
                              const gsr_config *config);

/* A batched backward captured in a HIP graph: the kernels gsr_backward_batch
 * would enqueue for these states, dL/dimage buffers, outputs, accumulate flag
 * and config, replayed by gsr_graph_launch without host work per kernel. The
 * graph holds the addresses given here: write new dL/dimage values into the
 * same buffers between launches. The states must stay alive (not released)
 * until the graph is destroyed, and the scenes unchanged in shape. Every
 * buffer the replay touches is allocated during this call; the capture
 * itself holds kernel launches only (fills, not memsets). When the context's
 * stream is the null stream the capture uses a temporary stream of default
 * priority. GSR_FLAG_STAGE_TIMING is ignored. Nothing is executed by the
 * capture except a single view's one-time tile ordering. */
typedef struct gsr_graph gsr_graph;
gsr_status gsr_graph_capture_backward(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states,
                                      const float *const *dl_dimages_chw, const gsr_grads *outs, int accumulate,
                                      const gsr_config *config, gsr_graph **graph_out);

/* Enqueue one replay of a captured graph on the context's stream. */
gsr_status gsr_graph_launch(gsr_ctx *ctx, gsr_graph *graph);

/* Wait for the context's stream, then free the graph. */
void gsr_graph_destroy(gsr_ctx *ctx, gsr_graph *graph);

/* Autotuner (the paper's rule: time one gradient-kernel iteration per
 * candidate, keep the fastest, repeat periodically; Detailed Design,
 * "Determining Balancing Threshold", and Approach, the balancing threshold
 * as a hyperparameter tuned per workload). Candidates are every
 * valid (tile, lds_batch) pair of the space (lds_batch <= tile*tile) times
 * every threshold; each is timed as one batched render plus one batched
 * backward of the given views with HIP events (median of `reps` runs), with
 * bwd_mode GSR_BWD_WAVE_REDUCE and `flags` (GSR_FLAG_STAGE_TIMING and
 * GSR_FLAG_DEBUG_COUNTERS are dropped). */
typedef struct {
    int32_t n_tiles, tiles[3];           /* subset of {8, 16, 32} */
    int32_t n_batches, batches[3];       /* subset of {64, 128, 256} */
    int32_t n_thresholds, thresholds[12]; /* 1..65 */
    int32_t reps;                        /* >= 1 */
    int32_t flags;
} gsr_tune_space;

typedef struct {
    gsr_config config;
    float render_ms, backward_ms;        /* medians over reps, whole batch */
} gsr_tune_entry;

/* Time every candidate of `space` on n_views (1..GSR_MAX_BATCH) views
 * (scenes[i] seen by cameras[i]; dl_dimages_chw[i] [3,H_i,W_i] or NULL for a
 * constant gradient image) and write the fastest (render + backward) to
 * *best. entries (may be NULL) receives up to max_entries timed candidates,
 * *n_entries (may be NULL) their count. Images and gradient outputs are
 * scratch buffers of the context's pool. Synchronises. */
gsr_status gsr_autotune(gsr_ctx *ctx, int32_t n_views, const gsr_scene *scenes, const gsr_camera *cameras,
                        const float *const *dl_dimages_chw, const gsr_tune_space *space, gsr_config *best,
                        gsr_tune_entry *entries, int32_t max_entries, int32_t *n_entries);

/* Periodic re-tuning: gsr_tuner_next returns the config to use for this
 * iteration, running gsr_autotune on the given views first on iteration 0
 * and then every `every` iterations (the paper re-tunes every 2000). */
typedef struct gsr_tuner gsr_tuner;
gsr_status gsr_tuner_create(const gsr_tune_space *space, int32_t every, gsr_tuner **out);
gsr_status gsr_tuner_next(gsr_ctx *ctx, gsr_tuner *tuner, int32_t n_views, const gsr_scene *scenes,
                          const gsr_camera *cameras, const float *const *dl_dimages_chw, gsr_config *config_out,
                          int32_t *retuned);
void gsr_tuner_destroy(gsr_tuner *tuner);

/* ---------------------------------------------------------------------
 * Serving: training-step requests (render + L1 loss + backward + Adam step,
 * step 7 of the paper's training pipeline figure) against resident scenes,
 * with continuous batching. A scheduler thread admits queued requests into
 * a batch as soon as a lane (a stream with its own context) is free: at
 * most max_batch requests, at most one in flight per scene (each request is
 * one optimiser step, so a scene's steps stay in arrival order and every
 * result equals what the request computes alone), and only while the
 * requests' estimated HBM footprint fits beside the resident scenes in the
 * budget. Batches on different lanes overlap on the device; a completion
 * thread per lane stamps finished requests.
 *
 * Resident state per scene (server-owned device memory): parameters,
 * gradients, Adam first and second moments, each one flat fp32 block of
 * n*(11 + 3K) floats laid out means3d [n,3] | log_scales [n,3] | quats
 * [n,4] | opacity_logits [n] | sh [n,K,3].
 * ------------------------------------------------------------------- */
typedef struct gsr_server gsr_server;

typedef struct {
    int64_t hbm_budget_bytes; /* resident scenes + in-flight request estimates */
    int32_t max_batch;        /* 1..GSR_MAX_BATCH requests per batch */
    int32_t lanes;            /* 1..4 streams batches rotate over */
    gsr_config config;        /* render/backward configuration of every batch */
    float lr, beta1, beta2, eps;
    int32_t capacity_render;  /* 1: a batch whose scenes have been rendered before renders with pair
                                 buffers of 1.5 x max(largest pairs per pixel seen x pixels, largest
                                 pair count seen) + 65536 per view (memory only: the sorts are
                                 bounded by the device-side count) and runs render, loss, backward
                                 and Adam without any host
                                 synchronisation; a request whose pairs overflow skips its Adam
                                 update on the device and is run again with the counts read back
                                 (gsr_result.render_mode). 0: every batch's render reads its counts
                                 back */
} gsr_server_opts;

/* One request: a step of scene `scene` seen by `camera` against a target
 * image drawn on the device, U[0,1) per value from SplitMix64 seeded with
 * target_seed (value i of the [3,H,W] image uses counter i). */
typedef struct {
    int32_t scene;
    gsr_camera camera;
    uint64_t target_seed;
} gsr_request;

typedef struct {
    int64_t id;                  /* from gsr_server_submit, in submission order */
    int32_t scene;
    int32_t status;              /* gsr_status of the step */
    int32_t batch_size, lane;    /* the batch that carried it */
    int32_t step;                /* the scene's optimiser step count after this request */
    float loss;                  /* mean |image - target| of the render before the step */
    double t_arrival, t_start, t_done; /* seconds on the server clock (gsr_server_now) */
    int32_t render_mode;         /* 0: the render read its pair counts back; 1: capacity mode (no host
                                    synchronisation); 2: its capacity-mode render overflowed and the
                                    step ran again with the counts read back */
} gsr_result;

/* Resident bytes of a scene of n Gaussians at sh_degree (four flat blocks). */
int64_t gsr_server_scene_bytes(int64_t n, int32_t sh_degree);

gsr_status gsr_server_create(int device, const gsr_server_opts *opts, gsr_server **out);
/* Drains every submitted request, stops the threads, frees everything. */
void gsr_server_destroy(gsr_server *server);
const char *gsr_server_last_error(const gsr_server *server);
/* Seconds since the server was created (steady clock). */
double gsr_server_now(const gsr_server *server);

/* Make a scene resident: its arrays (device pointers, or NULL for zeros,
 * e.g. to fill them later through gsr_server_scene_state) are copied into
 * server memory, Adam moments zeroed, step 0. GSR_EBUDGET if the resident
 * bytes would exceed the budget. Synchronises. */
gsr_status gsr_server_add_scene(gsr_server *server, const gsr_scene *init, int32_t *scene_id);
/* Waits for the scene's queued and in-flight requests, then frees it. */
gsr_status gsr_server_remove_scene(gsr_server *server, int32_t scene_id);
/* Device pointers of a resident scene's four flat blocks (valid until it is
 * removed; touch them only while no request for it is queued or in flight)
 * and its step count. Any output may be NULL. */
gsr_status gsr_server_scene_state(gsr_server *server, int32_t scene_id, gsr_scene *params, gsr_grads *grads,
                                  float **adam_m, float **adam_v, int32_t *step);
gsr_status gsr_server_set_step(gsr_server *server, int32_t scene_id, int32_t step);
/* Copy one flat block of a resident scene (block 0 parameters, 1 gradients,
 * 2 Adam m, 3 Adam v; n*(11+3K) floats) to (to_host = 1) or from (0) the
 * [host] buffer `host`, for checkpoints. Fails with GSR_ESTATE while a
 * request for the scene is queued or in flight. Synchronises. */
gsr_status gsr_server_scene_io(gsr_server *server, int32_t scene_id, int32_t block, float *host, int32_t to_host);

/* Queue a request (thread-safe); *id receives its id. Requests for unknown
 * scenes or with invalid cameras are rejected here. */
gsr_status gsr_server_submit(gsr_server *server, const gsr_request *req, int64_t *id);
/* Submit n requests at arrival_s[i] seconds after this call starts (an
 * open-loop load generator; ascending times), returning once the last is
 * submitted. ids (may be NULL) receives their ids. */
gsr_status gsr_server_replay(gsr_server *server, int32_t n, const gsr_request *reqs, const double *arrival_s,
                             int64_t *ids);
/* Wait until every submitted request has completed. */
gsr_status gsr_server_drain(gsr_server *server);
/* Move up to max completed results (completion order) into out. */
gsr_status gsr_server_results(gsr_server *server, gsr_result *out, int32_t max, int32_t *n);

/* Capacity mode: re-render n_views (1..GSR_MAX_BATCH) existing states
 * (each state's scene arrays, read again - their contents may have changed,
 * their sizes not - and its camera) into images_chw[i] without any host
 * synchronisation, reusing the states' buffers. Each state's pair buffers
 * hold pair_capacity = P + P/4 + 4096 entries of the P of the gsr_render
 * that created it; the tile sort and the ranges are launched for the whole
 * capacity and bounded on the device by the current pair count. A view whose pairs
 * exceed the capacity loses the excess and sets an overflow flag
 * (gsr_fwd_sync). config NULL = states[0]'s render config; its tile must
 * equal the render's. Afterwards the state's pair count is unknown on the
 * host (gsr_fwd_stats reports -1) until gsr_fwd_sync. */
gsr_status gsr_rerender_batch(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states, float *const *images_chw,
                              const gsr_config *config);

/* Read back a state's pair count after capacity-mode renders or graph
 * replays of them (synchronises; reads the device's count every time once a
 * state has been re-rendered in capacity mode). *overflowed = 1 when the last render's pairs exceeded
 * the capacity: its image and gradients are then incomplete, and the view
 * must be rendered again with gsr_render. Either output may be NULL. */
gsr_status gsr_fwd_sync(gsr_ctx *ctx, gsr_fwd *state, int64_t *n_pairs, int32_t *overflowed);

/* A whole batched training step captured in a HIP graph: capacity-mode
 * re-render of the states into images_chw, the loss gradient against
 * targets_chw into dl_dimages_chw ((1 - loss_lambda) L1 + loss_lambda
 * D-SSIM as gsr_l1_dssim_grad; loss_lambda = 0 is L1), and the batched
 * backward into outs (same rules as gsr_backward_batch). Replays read the
 * scenes' arrays, the cameras and the targets at capture time's addresses;
 * update parameters in place between replays (e.g. an optimiser step) and
 * check gsr_fwd_sync for overflow when the geometry changes a lot. Buffers
 * only the replays use belong to the graph; states, images, targets,
 * dL/dimage buffers, outputs and the context must outlive it. */
gsr_status gsr_graph_capture_step(gsr_ctx *ctx, int32_t n_views, gsr_fwd *const *states, float *const *images_chw,
                                  const float *const *targets_chw, float loss_lambda, float *const *dl_dimages_chw,
                                  const gsr_grads *outs, int accumulate, const gsr_config *config,
                                  gsr_graph **graph_out);

/* Release a forward state (its buffers return to the context's pool after
 * the stream reaches this point). */
gsr_status gsr_fwd_release(gsr_ctx *ctx, gsr_fwd *state);

/* Host-side facts about a state; does not touch the device. */
gsr_status gsr_fwd_stats(const gsr_fwd *state, gsr_fwd_stats_t *out);

/* Copy intermediate results to caller buffers (device-to-device, async). */
gsr_status gsr_fwd_export(gsr_ctx *ctx, const gsr_fwd *state, const gsr_fwd_export_t *dst);

/* Read the debug counters of the last backward (synchronises). GSR_ESTATE if
 * that backward did not run with GSR_FLAG_DEBUG_COUNTERS. */
gsr_status gsr_bwd_counters(gsr_ctx *ctx, const gsr_fwd *state, gsr_bwd_counters_t *out);

/* Stage times of the last render/backward with GSR_FLAG_STAGE_TIMING
 * (synchronises on the events). */
gsr_status gsr_ctx_stage_times(gsr_ctx *ctx, gsr_stage_times_t *out);

/* L1 loss gradient (harness step, outside the timed backward; the loss as
 * the difference of rendered and reference RGB values, Background, "3D Scene
 * Reconstruction"):
 * dl_dimage = sign(image - target) / count over `count` floats, sign(0) = 0. */
gsr_status gsr_l1_grad(gsr_ctx *ctx, const float *image, const float *target, int64_t count, float *dl_dimage);

/* Loss of the object-scene workload and its gradient (harness step, outside
 * the timed backward): L = (1 - lambda) * mean|image - target| + lambda *
 * (1 - SSIM(image, target)), SSIM with an 11x11 normalised Gaussian window
 * (sigma 1.5) as a zero-padded same-size convolution per channel, C1 =
 * 0.01^2, C2 = 0.03^2, averaged over the 3HW values. image, target,
 * dl_dimage [3,H,W]; loss (device, may be NULL) receives L. lambda in [0, 1]
 * (0.2 in 3D Gaussian Splatting). */
gsr_status gsr_l1_dssim_grad(gsr_ctx *ctx, const float *image, const float *target, int32_t height, int32_t width,
                             float lambda, float *dl_dimage, float *loss);

/* The paper's primitive exposed as a callable (Approach, "Key Components":
 * SW-B is a function call inserted in GPU code). Runs the per-wave
 * reduce-or-atomic primitive on synthetic data: wave w,
 * lane l contributes vals[(w*64+l)*9 + k] to sums[k] (k < 9) when
 * active[w*64+l] != 0. mode (plain, wave or serial reduce; not block) and
 * threshold as in gsr_config. lane_atomics[0]
 * receives the number of atomic lane-operations issued. sums [9] and
 * lane_atomics [1] are zeroed by the call. */
gsr_status gsr_wave_reduce_selftest(gsr_ctx *ctx, const float *vals, const uint8_t *active, int32_t n_waves,
                                    int32_t mode, int32_t threshold, int32_t lane_split,
                                    float *sums, uint64_t *lane_atomics);

/* Measurement utility (not part of rendering): one memory-operation
 * pattern of the backward composite, timed alone, to measure the roofs the
 * kernels are held against (no atomic rate is published for this GPU, so
 * it is measured).
 *   GSR_MB_COPY                   float4 copy of bytes/2 into the other half
 *                                 (ops = bytes read + written: HBM bandwidth)
 *   GSR_MB_ATOMIC_F32_DISTINCT    no-return fp32 adds, every lane its own
 *                                 address, lanes of a wave on consecutive
 *                                 elements (ops = lane-operations)
 *   GSR_MB_ATOMIC_F64_DISTINCT    the same with fp64
 *   GSR_MB_ATOMIC_F32_SAME_ADDRESS all 64 lanes of a wave add to one float
 *                                 (the plain kernel's pattern; ops = lane-ops)
 *   GSR_MB_ATOMIC_F32_ONE_LANE    lane 0 of each wave adds (one reduced sum
 *                                 per instruction; ops = lane-ops)
 *   GSR_MB_ATOMIC_F64_NINE_LANES  lanes 0..8 add to nine consecutive doubles
 *                                 (the reduced kernel's nine-lane issue)
 *   GSR_MB_WRITE                  non-temporal 16-byte stores over `bytes`
 *                                 (ops = bytes written)
 *   GSR_MB_READ                   16-byte loads over `bytes` less 16
 *                                 (ops = bytes read)
 *   GSR_MB_COPY_NT                as GSR_MB_COPY with non-temporal loads and
 *                                 stores, eight 16-byte chunks in flight
 *   GSR_MB_GATHER48               every 48-byte record of the largest power
 *                                 of two of them that fits read once, in a
 *                                 scattered (permuted) order (ops = bytes read)
 * The atomic patterns sweep a working set of `bytes` (128-byte slots for the
 * last three of them) with 8192 workgroups of 256 threads, 64 operations each.
 * bytes: a power of two in [1 MiB, 4 GiB], allocated and cleared by the call
 * from the context's pool. Runs one untimed launch, then `reps` (1..100)
 * timed ones on the context's stream and synchronises; ms_per_launch and
 * ops_per_launch (host) receive the median launch time and the operation
 * count of one launch. */
enum {
    GSR_MB_COPY = 0,
    GSR_MB_ATOMIC_F32_DISTINCT = 1,
    GSR_MB_ATOMIC_F64_DISTINCT = 2,
    GSR_MB_ATOMIC_F32_SAME_ADDRESS = 3,
    GSR_MB_ATOMIC_F32_ONE_LANE = 4,
    GSR_MB_ATOMIC_F64_NINE_LANES = 5,
    GSR_MB_WRITE = 6,
    GSR_MB_READ = 7,
    GSR_MB_COPY_NT = 8,
    GSR_MB_GATHER48 = 9
};
gsr_status gsr_microbench(gsr_ctx *ctx, int32_t kind, int64_t bytes, int32_t reps, double *ms_per_launch,
                          double *ops_per_launch);

/* Host-only argument checks (no device needed); GSR_OK or GSR_EINVAL. */
gsr_status gsr_validate_scene(const gsr_scene *scene);
gsr_status gsr_validate_camera(const gsr_camera *camera);
gsr_status gsr_validate_config(const gsr_config *config, const gsr_camera *camera);

/* Library version string, e.g. "gsr 0.1 gfx950". */
const char *gsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
