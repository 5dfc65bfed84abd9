// Internal declarations shared by the HIP translation units of libgsr.
// Device layouts (all in HBM, one allocation each, from the context pool):
//   rec        [n][3] float4  (u, v, A, B) (C, o, r, g) (b, id bits, 2 ln(255 o), depth): the
//              record each list entry gathers in the composite kernels
//   radius     [n] int32, tiles_touched [n] uint32, clamp_mask [n] uint8
//   depth_key  [n] uint32 (fp32 depth bits, 0xffffffff when culled), ids [n]
//   offsets    [n] uint32 exclusive scan of tiles_touched in depth order
//   pair_tile / pair_id [P] uint32 (+ alternates for the radix sort)
//   ranges     [tiles] uint2, T_final [HW] f32, n_contrib [HW] uint32
//   acc        [n][GSR_ACC_STRIDE] f32 or f64 backward accumulators: five moments of the
//              pixels' dL/do over the pixel offsets, dL/do, dL/drgb
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "gsr.h"

namespace gsr {

// Camera as the kernels take it (by value).
struct DevCamera {
    int width, height, tile, grid_x, grid_y;
    float fx, fy, cx, cy;
    float R[9];        // world -> camera rotation, row-major
    float t[3];
    float centre[3];   // camera centre in world space, -R^T t
    float znear;
    float lox, hix, loy, hiy; // guard band of the projection Jacobian's x/z and y/z
    float bg[3];
};

DevCamera make_dev_camera(const gsr_camera &c, int tile);

// Caching device allocator: buffers return to per-size free lists and are
// reused by later requests on the same (single) stream, so no hipFree or
// hipMalloc runs in steady state.
class Pool {
public:
    explicit Pool(int device) : device_(device) {}
    ~Pool();
    hipError_t alloc(void **p, size_t bytes);
    void release(void *p);
    size_t reserved() const { return reserved_; }
private:
    int device_;
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live_;
    size_t reserved_ = 0;
};

// ----- kernel launchers (defined in the .hip files) -----

// a1: per-Gaussian projection (sh_degree 0..3).
hipError_t launch_preprocess_fwd(const gsr_scene &s, const DevCamera &cam, float4 *rec, int32_t *radius,
                                 uint32_t *tiles_touched, uint32_t *depth_key, uint32_t *ids, uint8_t *clamp_mask,
                                 hipStream_t st);

// a7: raw-parameter gradients from the accumulators (float or, acc_f64, double rows). Writes
// every row (zeros for culled Gaussians), or with accumulate = 1 adds to the visible rows only.
hipError_t launch_preprocess_bwd(const gsr_scene &s, const DevCamera &cam, const int32_t *radius, const void *acc,
                                 bool acc_f64, const gsr_grads &out, int accumulate, hipStream_t st);

// Zero the accumulator rows of Gaussians with radius > 0 (the only rows the composite writes):
// those listed in visible_ids[0, n_visible) when the list is given (the first *n_visible_dev of
// them when that device-side count is given), else found from radius.
hipError_t launch_zero_visible_rows(const int32_t *radius, int64_t n, const uint32_t *visible_ids, int64_t n_visible,
                                    const uint32_t *n_visible_dev, void *acc, bool acc_f64, hipStream_t st);
// Accumulator rows as fp32 gradients [n][GSR_ACC_STRIDE] (dL/du, dL/dv, dL/dA, dL/dB, dL/dC,
// dL/do, dL/drgb: the moments converted with the record's opacity and conic), culled rows as
// zeros.
hipError_t launch_export_acc(const int32_t *radius, const float4 *rec, int64_t n, const void *acc, bool acc_f64,
                             float *dst, hipStream_t st);
// mean2d [n,2], conic_opacity [n,4] (A, B, C, o), rgb [n,3], depth [n] out of the records, zeros
// for culled Gaussians (radius 0); any output may be null.
hipError_t launch_export_rec(const int32_t *radius, const float4 *rec, int64_t n, float *mean2d,
                             float *conic_opacity, float *rgb, float *depth, hipStream_t st);

// Exclusive scan of n uint32 values (in[gather[i]] when gather != nullptr; out may equal in when
// gather is nullptr, and must alias neither in nor gather when it is not). total (device, may be
// nullptr) receives the sum. Scratch sized by scan_partial_count.
size_t scan_partial_count(int64_t n);
hipError_t device_exclusive_scan(const uint32_t *in, const uint32_t *gather, uint32_t *out, int64_t n,
                                 uint32_t *total, uint32_t *partials, hipStream_t st);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits). Buffers
// ping-pong between (k0,v0) and (k1,v1); returns the index (0/1) holding the
// result in *which. With n_dev the item count is read on the device (at most n,
// which sizes the launches); with range_dev = (max ~key, max key) on the device,
// passes above the keys' highest varying bit copy instead of sorting.
size_t radix_hist_count(int64_t n);
// Whether a sort of n items runs without a separate scan launch per pass (few blocks, each
// deriving its offsets from the histogram table itself).
bool radix_sort_fused(int64_t n);
hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits,
                            uint32_t *hist, uint32_t *partials, int *which, hipStream_t st,
                            const uint32_t *n_dev = nullptr, const uint32_t *range_dev = nullptr);

// a2: expand each depth-ordered Gaussian into its (tile, id) pairs; pairs at positions >= cap
// are dropped.
hipError_t launch_emit_pairs(int64_t n, const uint32_t *sorted_ids, const uint32_t *offsets, const float4 *rec,
                             const int32_t *radius, const DevCamera &cam, uint32_t *pair_tile, uint32_t *pair_id,
                             int64_t cap, hipStream_t st);

// Capacity mode: overflow[0] = (*total > cap).
hipError_t launch_pair_overflow(const uint32_t *total, int64_t cap, uint32_t *overflow, hipStream_t st);

// a4: per-tile [start, end) ranges of the first P tile-sorted pairs, every tile written (empty
// ones as [i, i)); P_dev (nullable) bounds P with a device-side count.
hipError_t launch_tile_ranges(int64_t P, const uint32_t *P_dev, const uint32_t *sorted_tile, uint2 *ranges,
                              int64_t n_tiles, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t st);

// out[0] = number of r[i] > 0.
hipError_t launch_count_positive(const int32_t *r, int64_t n, uint32_t *out, hipStream_t st);

// flags[i] = (r[i] > 0); and the compaction of the flagged (key[i], i) to positions pos[i].
// Visible Gaussians (r > 0) in index order: key_out/id_out[0, n_visible) = (key[i], i);
// totals[0] = sum of tiles[i] over them (the pair count P), totals[1] = n_visible, totals[4] =
// max of ~key and totals[5] = max of key over them (0, 0 when none). part: visible_partial_count(n)
// entries of scratch.
size_t visible_partial_count(int64_t n);
hipError_t launch_compact_visible(const int32_t *r, int64_t n, const uint32_t *key, const uint32_t *tiles,
                                  uint4 *part, uint32_t *totals, uint32_t *key_out, uint32_t *id_out,
                                  hipStream_t st);

// One view of a composite launch. A launch covers up to kMaxViews views (same
// tile size and LDS batch): the views travel by value in the kernel
// arguments and a work table gives each workgroup its (view, tile).
constexpr int kMaxViews = 16;
struct ViewDesc {
    DevCamera cam;
    const uint2 *ranges;
    const uint32_t *ids;      // tile-sorted Gaussian ids
    const float4 *rec;
    float *image;             // forward outputs
    float *T_final;
    uint32_t *n_contrib;
    uint32_t *tile_walk;      // optional forward output: deepest n_contrib per tile
    const float *dl_dimage;   // backward input / output
    void *acc;                // [n][GSR_ACC_STRIDE] float or double rows
};
struct ViewBatch {
    ViewDesc v[kMaxViews];
    uint32_t base[kMaxViews + 1]; // base[i]: index of view i's first tile in the batch's tile numbering
    int n;
};
enum { ORDER_IDENTITY = 0, ORDER_BY_LENGTH = 1, ORDER_BY_WALK = 2 };

// a5: forward composite. work: per-workgroup (view, tile), base[n] entries; nullptr = one
// view, tiles in index order (or XCD remap).
hipError_t launch_composite_fwd(const ViewBatch &vb, int tile, int lds_batch, int remap, const uint2 *work,
                                hipStream_t st);

// The batch's (view, tile) pairs, base[n] of them: in index order (ORDER_IDENTITY) or by
// decreasing work (list length, or each view's tile_walk).
hipError_t launch_order_tiles(const ViewBatch &vb, int mode, uint2 *work, hipStream_t st);
// One view (vb.n == 1): the tile order as launch_order_tiles and, in the same launch, the
// accumulator rows of the m listed Gaussians (m_dev: the count on the device, nullable) cleared.
hipError_t launch_clear_rows_and_order(const ViewBatch &vb, int mode, uint2 *work, const uint32_t *ids, int64_t m,
                                       const uint32_t *m_dev, void *acc, bool acc_f64, hipStream_t st);

// a6: backward composite.
struct BwdParams {
    unsigned long long *counters; // [7 + 65 + 2] when counting (one set for the launch)
    int threshold;                // effective: reduce iff active >= threshold (>= 1)
};
hipError_t launch_composite_bwd(const ViewBatch &vb, int tile, int lds_batch, int remap, int mode, bool count,
                                bool lane_split, bool acc_f64, const BwdParams &p, const uint2 *work,
                                hipStream_t st);
// The plain-atomic a6 built with the compiler's atomic optimizer (k_composite_compiler_reduce.hip).
hipError_t launch_composite_bwd_compiler_reduce(const ViewBatch &vb, int tile, int lds_batch, int remap,
                                                bool acc_f64, const BwdParams &p, const uint2 *work, hipStream_t st);

hipError_t launch_l1_grad(const float *image, const float *target, int64_t count, float *out, hipStream_t st);

// Training-step kernels (k_train.hip): Adam on a flat block (step >= 1; no update when `skip` is
// given and *skip != 0 on the device), a SplitMix64 U[0,1) fill, and sum |a-b| added into *out.
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st, const uint32_t *skip = nullptr);
hipError_t launch_uniform(float *out, int64_t count, uint64_t seed, hipStream_t st);
hipError_t launch_l1_sum(const float *a, const float *b, int64_t count, float *out, hipStream_t st);

// (1 - lambda) L1 + lambda (1 - SSIM) of C-channel W x H images (k_loss.hip): dL/dimage into
// out, the loss into *loss when loss != nullptr. dmu/dexx/dexy: C*W*H scratch floats each,
// sums: dssim_partial_count(C, W, H) scratch floats (used only when loss != nullptr).
size_t dssim_partial_count(int C, int W, int H);
hipError_t launch_l1_dssim_grad(const float *img, const float *ref, int C, int W, int H, float lambda, float *dmu,
                                float *dexx, float *dexy, float *sums, float *out, float *loss, hipStream_t st);
// Micro-benchmark kernels (k_micro.hip): one launch of pattern `kind` (GSR_MB_*) over a
// working set of `bytes` (a power of two >= 1 MiB); *ops = its operation count.
hipError_t launch_microbench(int kind, void *buf, int64_t bytes, int64_t *ops, hipStream_t st);
hipError_t launch_wave_reduce_selftest(const float *vals, const uint8_t *active, int n_waves, int mode,
                                       int threshold, int lane_split, float *sums, unsigned long long *lane_atomics,
                                       hipStream_t st);

// Batched render into new states in capacity mode (pair buffers of caps[v] pairs, no host
// synchronisation; a view whose pairs exceed its capacity raises its overflow word, totals[2]).
gsr_status render_batch_capacity(gsr_ctx *ctx, int nv, const gsr_scene *scenes, const gsr_camera *cameras,
                                 const gsr_config *config, float *const *images, const int64_t *caps,
                                 gsr_fwd **states_out);

} // namespace gsr

// ----- opaque API objects -----

struct gsr_ctx {
    int device = 0;
    hipStream_t stream = nullptr; // nullptr = HIP's null stream
    std::string err;
    gsr::Pool *pool = nullptr;
    uint32_t *host_pinned = nullptr; // small readback area
    hipEvent_t ev[12] = {};
    hipEvent_t ev_counts = nullptr;  // counts of a render read back (no timing)
    bool timing_render = false, timing_bwd = false;
    void *scratch = nullptr;         // this device's fixed scratch area (gsr_backward_noalloc)
    hipError_t scratch_err = hipSuccess;
};

struct gsr_fwd {
    gsr_scene scene{};
    gsr_camera camera{};
    gsr_config config{};
    gsr::DevCamera dcam{};
    int64_t n = 0, n_visible = -1, P = 0, n_tiles = 0;
    float4 *rec = nullptr;
    int32_t *radius = nullptr;
    uint32_t *tiles_touched = nullptr;
    uint8_t *clamp_mask = nullptr;
    uint32_t *depth_key = nullptr, *ids = nullptr, *key_alt = nullptr, *ids_alt = nullptr;
    uint32_t *sorted_ids_by_depth = nullptr; // points into ids or ids_alt
    uint32_t *offsets = nullptr;
    uint32_t *pair_tile = nullptr, *pair_id = nullptr, *pair_tile_alt = nullptr, *pair_id_alt = nullptr;
    uint32_t *sorted_pair_id = nullptr; // points into pair_id or pair_id_alt
    int64_t pair_cap = 0;               // entries of each pair buffer
    bool p_known = true;                // P and n_visible hold this render's values
    bool overflowed = false;            // the last capacity-mode render dropped pairs
    bool capacity_mode = false;         // re-rendered in capacity mode (counts live on the device)
    // Scratch kept for re-renders without reallocation (capacity mode, graph capture).
    uint32_t *totals = nullptr;         // [0] P, [1] n_visible, [2] overflow flag, [4..5] depth-key range
    uint32_t *dsort_hist = nullptr, *dsort_partials = nullptr, *scan_partials = nullptr;
    uint32_t *tsort_hist = nullptr, *tsort_partials = nullptr;
    uint4 *vis_part = nullptr;          // per-block statistics of the visible-Gaussian compaction
    uint2 *ranges = nullptr;
    uint32_t *tile_walk = nullptr; // deepest n_contrib per tile (ordered renders)
    uint2 *order_bwd = nullptr;    // table a single-view backward orders its tiles in (rebuilt by each)
    uint2 *batch_work = nullptr;   // (view, tile) table of a batched backward led by this state
    int64_t batch_work_cap = 0;
    float *T_final = nullptr;
    uint32_t *n_contrib = nullptr;
    void *acc = nullptr;                // n rows of GSR_ACC_STRIDE values, room for doubles
    bool acc_f64 = false;               // precision of the last backward composite's accumulators
    unsigned long long *counters = nullptr;
    bool counters_valid = false;
    std::vector<void *> owned; // every pool buffer of this state
};
