// Composite kernels of the 3DGS pipeline on gfx950 (fp32), one workgroup of
// TILE*TILE threads per screen tile, one thread per pixel, each 64-lane
// wavefront covering an 8x8 pixel block.
//   a5 composite_fwd: front-to-back blending over the tile's depth-ordered
//      list, Gaussian records staged through LDS in batches; stores
//      T_final and n_contrib so the backward can recompute instead of store.
//   a6 composite_bwd: the paper's gradient-computation kernel (Motivation,
//      outline of the gradient computation step): each pixel walks the same
//      list in reverse and adds its contribution to nine per-Gaussian
//      gradients. All lanes of a wave walk the same entry in lockstep, so the
//      address is wave-uniform by construction (the paper's observation that
//      almost every warp updates a single primitive), and lanes that skip an
//      entry carry zeros instead of leaving the loop (the SW-B kernel
//      transformation of Detailed Design, "Butterfly Reduction"). The update
//      is either nine plain atomic adds per active lane, or - when the
//      wave's active-lane count reaches the balancing threshold (Approach,
//      "Scheduling Atomic Updates Between Core and L2") - a cross-lane reduction
//      over the 64 lanes and one lane's (or nine lanes') atomics.
#include "device_common.hpp"

namespace gsr {
namespace {

__device__ __forceinline__ int tile_for_block(int b, int n_tiles, int remap) {
    if (!remap) return b;
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous band of tiles so neighbouring tiles (which share Gaussians)
    // update accumulator lines through the same L2.
    const int per = (n_tiles + 7) / 8;
    return (b & 7) * per + (b >> 3);
}

__host__ __device__ __forceinline__ int grid_for_tiles(int n_tiles, int remap) {
    return remap ? ((n_tiles + 7) / 8) * 8 : n_tiles;
}

// Accumulator add in the accumulator's precision (fp32 or fp64 rows).
__device__ __forceinline__ void atomic_acc(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_acc(double *p, float v) { unsafeAtomicAdd(p, (double)v); }

// Per-wave update of the nine values of one Gaussian. Every lane of the wave
// must call it (uniform control flow). Returns the atomic lane-operations
// this lane issued.
template <int MODE, bool SPLIT, typename AccT>
__device__ __forceinline__ uint32_t emit9(bool active, uint64_t m, float (&v)[9], AccT *dst, int threshold, int lane,
                                          uint64_t &reduced_mask_out) {
    // m: the wave's ballot of active
    uint32_t issued = 0;
    reduced_mask_out = 0;
    if (MODE == GSR_BWD_PLAIN_ATOMIC) {
        if (active) {
#pragma unroll
            for (int k = 0; k < 9; ++k) atomic_acc(dst + k, v[k]);
            issued = 9;
        }
        return issued;
    }
    const int cnt = __popcll(m);
    if (MODE == GSR_BWD_SERIAL_REDUCE) {
        if (cnt >= threshold) {
            // Serialised leader: the nine sums are built one active lane at a time from that
            // lane's registers (a uniform loop of readlanes over the ballot), then lanes 0..8
            // issue them as one instruction.
            reduced_mask_out = m;
            float s[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) s[k] = 0.0f;
            for (uint64_t rest = m; rest; rest &= rest - 1) {
                const int l = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(rest));
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    s[k] += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[k]), l));
            }
            float mine = s[0];
#pragma unroll
            for (int k = 1; k < 9; ++k) mine = lane == k ? s[k] : mine;
            if (lane < 9) {
                atomic_acc(dst + lane, mine);
                issued = 1;
            }
        } else if (active) {
#pragma unroll
            for (int k = 0; k < 9; ++k) atomic_acc(dst + k, v[k]);
            issued = 9;
        }
        return issued;
    }
    // The sparse case is issued first, as straight-line code under the lane mask: the reduction
    // is then the last use of v, and its lane swaps (which overwrite their operands) need no
    // copies of the nine values.
    const bool sparse = cnt < threshold;
    if (sparse && active) {
#pragma unroll
        for (int k = 0; k < 9; ++k) atomic_acc(dst + k, v[k]);
        issued = 9;
    }
    if (sparse) return issued;
    reduced_mask_out = m; // threshold >= 1, so cnt > 0 here
    if (SPLIT) {
        float mine = wave_sum9_scatter(v, lane);
        // The last exchange's add stays with its exchange (one DPP add at full exec) instead of
        // sinking into the issuing lanes' branch as a separate move, clear and add.
        asm volatile("" : "+v"(mine));
        if (sum9_issues(lane)) {
            atomic_acc(dst + sum9_slot(lane), mine);
            issued = 1;
        }
        return issued;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = wave_sum_to_lane63(v[k]);
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < 9; ++k) atomic_acc(dst + k, v[k]);
        issued = 9;
    }
    return issued;
}

// Entries of a staged LDS batch this wave has to visit, as wave-uniform bit
// masks (bit j % 64 of mask[j / 64] for entry j < limit). A lane of the wave
// can pass entry j only if the splat's quadratic form (log2(e)/2) d^T K d (K
// the conic, d the offset from its centre; the staged units) is at most
// log2(255 o) at that lane's sample point. The test takes the minimum of the
// form over the square spanned by the wave's 8x8 sample points (the pixel
// centres, qc +- 3.5 in each axis): zero when the centre lies inside, else
// the least of the four edge minima (each a clamped one-dimensional
// quadratic). Being a minimum over a superset of the sample points, with an
// absolute slack of 1e-3, it never drops an entry some lane passes. (The
// square widened by half a pixel more kept 7 % more entries that no lane
// takes.) Lane l tests entries l, l+64, ... so the walk loops need no
// per-entry test and skip the rest with scalar bit scans.
__device__ __forceinline__ float edge_min(float d, float lo, float hi, float kd, float kcross, float ko) {
    // min over e in [lo, hi] of kd d^2 + 2 kcross d e + ko e^2 (ko > 0)
    // (an approximate minimiser moves the value only to second order, far inside the slack)
    const float e = fminf(fmaxf(-kcross * d * __builtin_amdgcn_rcpf(ko), lo), hi);
    return fmaf(kd * d, d, fmaf(2.0f * kcross * d, e, ko * e * e));
}

template <int BATCH>
__device__ __forceinline__ void wave_visit_masks(const float4 *s0, const float4 *s1, const float4 *s2, int limit,
                                                 float qcx, float qcy, int lane, uint64_t (&mask)[BATCH / 64]) {
#pragma unroll
    for (int q = 0; q < BATCH / 64; ++q) {
        const int j = q * 64 + lane;
        bool vis = false;
        if (j < limit) {
            const float4 r = s0[j];
            // the staged form is -log2(e)/2 (d^T K d): (ka, kb, kc) = its negation as (A, B, C)
            const float ka = -r.z, kb = -0.5f * r.w, kc = -s1[j].x, reach = s2[j].z;
            // square [qc - 3.5, qc + 3.5]^2 relative to the splat centre
            const float lx = qcx - 3.5f - r.x, hx = qcx + 3.5f - r.x;
            const float ly = qcy - 3.5f - r.y, hy = qcy + 3.5f - r.y;
            const bool inside = lx <= 0.0f && hx >= 0.0f && ly <= 0.0f && hy >= 0.0f;
            float fmin = 0.0f;
            if (!(ka > 0.0f && kc > 0.0f && ka * kc - kb * kb > 0.0f)) {
                fmin = 0.0f; // not positive definite (numerically): keep the entry
            } else if (!inside) {
                fmin = fminf(fminf(edge_min(lx, ly, hy, ka, kb, kc), edge_min(hx, ly, hy, ka, kb, kc)),
                             fminf(edge_min(ly, lx, hx, kc, kb, ka), edge_min(hy, lx, hx, kc, kb, ka)));
            }
            vis = reach > 0.0f && fmin <= reach + 1e-3f;
        }
        mask[q] = __ballot(vis);
    }
}

// The workgroup's (view, tile): from the work table, else view 0 with the
// identity or XCD-banded tile order. Returns false for padding workgroups.
__device__ __forceinline__ bool block_work(const ViewBatch &vb, int remap, const uint2 *work, int &view, int &tile) {
    if (work) {
        const uint2 w = work[blockIdx.x];
        view = __builtin_amdgcn_readfirstlane((int)w.x);
        tile = __builtin_amdgcn_readfirstlane((int)w.y);
        return true;
    }
    const int n_tiles = vb.v[0].cam.grid_x * vb.v[0].cam.grid_y;
    view = 0;
    tile = tile_for_block(blockIdx.x, n_tiles, remap);
    return tile < n_tiles;
}

template <int TILE, int BATCH>
__global__ __launch_bounds__(TILE *TILE) void composite_fwd_kernel(ViewBatch vb, int remap,
                                                                   const uint2 *__restrict__ work) {
    constexpr int NT = TILE * TILE;
    constexpr int QX = TILE / 8;
    __shared__ float4 s0[BATCH], s1[BATCH], s2[BATCH];
    __shared__ uint32_t s_deepest;
    int view, tile;
    if (!block_work(vb, remap, work, view, tile)) return;
    const ViewDesc &f = vb.v[view];
    const DevCamera &cam = f.cam;
    const uint2 *__restrict__ ranges = f.ranges;
    const uint32_t *__restrict__ ids = f.ids;
    const float4 *__restrict__ rec = f.rec;
    if (threadIdx.x == 0) s_deepest = 0;
    __syncthreads();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qx0 = (tile % cam.grid_x) * TILE + (wave % QX) * 8;
    const int qy0 = (tile / cam.grid_x) * TILE + (wave / QX) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const float qcx = (float)qx0 + 4.0f, qcy = (float)qy0 + 4.0f; // centre of the wave's 8x8 sample points
    const uint2 rg = ranges[tile];
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    // The next batch's records are loaded while this batch is walked (and the list ids of the
    // batch after it), so staging a batch does not wait for memory.
    const bool stager = tid < BATCH;
    float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0; // raw records of the next batch
    uint32_t id_next = 0;                                              // list ids one batch further
    if (stager && rg.x + tid < rg.y) {
        const size_t g = 3 * (size_t)ids[rg.x + tid];
        n0 = rec[g];
        n1 = rec[g + 1];
        n2 = rec[g + 2];
    }
    if (stager && rg.x + BATCH + tid < rg.y) id_next = ids[rg.x + BATCH + tid];
    for (uint32_t start = rg.x; start < rg.y; start += BATCH) {
        if (__syncthreads_count(done) == NT) break;
        if (stager && start + tid < rg.y) {
            prescale_record(n0, n1, n2);
            s0[tid] = n0;
            s1[tid] = n1;
            s2[tid] = n2;
        }
        __syncthreads();
        if (stager && start + BATCH + tid < rg.y) {
            const size_t g = 3 * (size_t)id_next;
            n0 = rec[g];
            n1 = rec[g + 1];
            n2 = rec[g + 2];
        }
        if (stager && start + 2 * BATCH + tid < rg.y) id_next = ids[start + 2 * BATCH + tid];
        const int cnt = min(BATCH, (int)(rg.y - start));
        uint64_t vis[BATCH / 64];
        wave_visit_masks<BATCH>(s0, s1, s2, cnt, qcx, qcy, lane, vis);
        // One entry for the whole wave: lanes that have stopped (or skip it) run the same
        // arithmetic with their updates masked off, so the walk is a uniform loop.
        const auto blend = [&](int j, const float4 &a, const float4 &b, const float4 &c, bool valid) {
            const SplatEval e = eval_splat(fpx, fpy, a.x, a.y, a.z, a.w, b.x, b.y);
            const bool take = valid && e.pass && !done;
            const float Tn = T * (1.0f - e.alpha);
            const bool stop = take && Tn < kTStop;
            const bool use = take && !stop;
            done = done || stop;
            const float w = use ? e.alpha * T : 0.0f;
            c0 = fmaf(w, b.z, c0);
            c1 = fmaf(w, b.w, c1);
            c2 = fmaf(w, c.x, c2);
            T = use ? Tn : T;
            last = use ? start - rg.x + (uint32_t)j + 1 : last;
        };
#pragma unroll
        for (int q = 0; q < BATCH / 64; ++q) {
            uint64_t mq = vis[q];
            // Visited entries two at a time: both records are read before the first is blended
            // (an odd last entry is paired with itself, the copy masked off).
            while (mq && __ballot(!done)) {
                const int j1 = q * 64 + __builtin_ctzll(mq);
                mq &= mq - 1;
                const bool two = mq != 0;
                const int j2 = two ? q * 64 + __builtin_ctzll(mq) : j1;
                mq = two ? mq & (mq - 1) : mq;
                const float4 a1 = s0[j1], b1 = s1[j1], e1 = s2[j1];
                const float4 a2 = s0[j2], b2 = s1[j2], e2 = s2[j2];
                blend(j1, a1, b1, e1, true);
                blend(j2, a2, b2, e2, two);
            }
        }
    }
    if (inside) {
        const size_t hw = (size_t)cam.width * cam.height;
        const size_t pix = (size_t)py * cam.width + px;
        f.image[pix] = fmaf(T, cam.bg[0], c0);
        f.image[hw + pix] = fmaf(T, cam.bg[1], c1);
        f.image[2 * hw + pix] = fmaf(T, cam.bg[2], c2);
        f.T_final[pix] = T;
        f.n_contrib[pix] = last;
    }
    if (f.tile_walk) {
        // Deepest n_contrib of the tile: the backward's walk length, used to order its blocks.
        const uint32_t w = wave_max_u32(last);
        if (lane == 0) atomicMax(&s_deepest, w);
        __syncthreads();
        if (threadIdx.x == 0) f.tile_walk[tile] = s_deepest;
    }
}

enum { CNT_EVAL = 0, CNT_ACTIVE, CNT_WAVE_ENTRIES, CNT_REDUCED, CNT_PLAIN_LANES, CNT_LANE_ATOMICS, CNT_INSTRS, CNT_HIST };
// after the 65 histogram slots: visited wave-entries (every entry a wave's visit masks keep)
// and the most entries any one wave visited
// and the list entries the blocks staged (each block walks to its deepest pixel's n_contrib)
constexpr int CNT_VISITED = CNT_HIST + 65, CNT_MAX_WAVE_VISITS = CNT_HIST + 66, CNT_WALKED = CNT_HIST + 67,
              CNT_SLOTS = CNT_HIST + 68;

template <int TILE, int BATCH, int MODE, bool COUNT, bool SPLIT, typename AccT>
__global__ __launch_bounds__(TILE *TILE) void composite_bwd_kernel(ViewBatch vb, int remap,
                                                                   const uint2 *__restrict__ work, BwdParams p) {
    constexpr int QX = TILE / 8;
    __shared__ float4 s0[BATCH], s1[BATCH], s2[BATCH];
    __shared__ uint32_t s_walk;
    __shared__ unsigned long long s_cnt[COUNT ? CNT_SLOTS : 1];
    // Block pre-reduction: the reduced sums of every wave land in LDS per batch entry, and the
    // block issues one atomic per (tile, Gaussian, value) when the batch is done.
    constexpr bool BLOCK = MODE == GSR_BWD_BLOCK_REDUCE;
    __shared__ float s_acc[BLOCK ? BATCH * 9 : 1];
    __shared__ uint32_t s_touch[BLOCK ? BATCH : 1];
    int view, tile;
    if (!block_work(vb, remap, work, view, tile)) return;
    const ViewDesc &a = vb.v[view];
    const DevCamera &cam = a.cam;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qx0 = (tile % cam.grid_x) * TILE + (wave % QX) * 8;
    const int qy0 = (tile / cam.grid_x) * TILE + (wave / QX) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const float qcx = (float)qx0 + 4.0f, qcy = (float)qy0 + 4.0f;
    const size_t hw = (size_t)cam.width * cam.height;
    const size_t pix = inside ? (size_t)py * cam.width + px : 0;
    float T = inside ? a.T_final[pix] : 1.0f;
    const uint32_t nc = inside ? a.n_contrib[pix] : 0u;
    const float G0 = inside ? a.dl_dimage[pix] : 0.0f;
    const float G1 = inside ? a.dl_dimage[hw + pix] : 0.0f;
    const float G2 = inside ? a.dl_dimage[2 * hw + pix] : 0.0f;
    // Colour behind the current entry, projected on this pixel's dL/dpixel: the recursion
    // Q <- Q + alpha (c - Q) of the three channels carried as one number S = Q . dL/dpixel.
    float S = cam.bg[0] * G0 + cam.bg[1] * G1 + cam.bg[2] * G2;
    const uint2 rg = a.ranges[tile];
    // The view's pointers in registers: read through the descriptor, they would be loaded again
    // after every atomic (the compiler cannot tell that the adds leave the descriptor alone).
    AccT *const acc = static_cast<AccT *>(a.acc);
    const float4 *const rec = a.rec;
    const uint32_t *const ids = a.ids + rg.x;

    if (tid == 0) s_walk = 0;
    if (COUNT)
        for (int i = tid; i < CNT_SLOTS; i += TILE * TILE) s_cnt[i] = 0;
    __syncthreads();
    // Entries past every pixel's n_contrib contribute nothing: the block walks to its deepest
    // pixel, each wave only to its own.
    const uint32_t wmax = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_max_u32(nc));
    if (lane == 0) atomicMax(&s_walk, wmax);
    __syncthreads();
    const int walk = (int)s_walk;

    uint64_t c_eval = 0, c_active = 0, c_we = 0, c_red = 0, c_plain = 0, c_instr = 0, c_visit = 0;
    uint32_t issued = 0;
    if (COUNT) {
        // E = sum of n_contrib: every pixel walks its entries 1..n_contrib.
        uint32_t s = nc;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) s += (uint32_t)__shfl_xor((int)s, d, 64);
        c_eval = s;
    }

    for (int end = walk; end > 0; end -= BATCH) {
        const int start = end > BATCH ? end - BATCH : 0;
        const int cnt = end - start;
        __syncthreads();
        if (tid < cnt) stage_record(rec, ids[start + tid], s0[tid], s1[tid], s2[tid]);
        if (BLOCK) {
            for (int i = tid; i < cnt * 9; i += TILE * TILE) s_acc[i] = 0.0f;
            if (tid < cnt) s_touch[tid] = 0u;
        }
        __syncthreads();
        const int jtop = min(cnt, (int)wmax - start) - 1;
        // Entries this wave must visit (at or below its walk bound, not culled), one bit each.
        uint64_t vis[BATCH / 64];
        wave_visit_masks<BATCH>(s0, s1, s2, jtop + 1, qcx, qcy, lane, vis);
        // One visited entry for the whole wave (uniform control flow).
        const auto visit = [&](int j, const float4 &r0, const float4 &r1, const float4 &r2) {
            const uint32_t pos = (uint32_t)(start + j + 1);
            const float rb = r2.x;
            const SplatEval e = eval_splat(fpx, fpy, r0.x, r0.y, r0.z, r0.w, r1.x, r1.y);
            const bool walked = pos <= nc;
            const bool active = walked && e.pass;
            // the ballot as the AND of the three compares' own lane masks
            const uint64_t am = __ballot(walked) & __ballot(!(e.lp > 0.0f)) & __ballot(e.alpha >= kAlphaMin);
            // No lane takes the entry (an eighth of the visits): T, S and the sums stay exactly as
            // they are, so the wave skips the rest.
            if (am == 0) {
                if (COUNT) c_visit += 1;
                return;
            }
            // Lanes that skip this entry run the same arithmetic with alpha and G set to zero:
            // their nine values come out as zeros and T, S stay as they are (the hardware
            // reciprocal of 1 is exactly 1).
            const float al = active ? e.alpha : 0.0f;
            const float gz = active ? e.G : 0.0f;
            // Transmittance in front of this entry; hardware reciprocal (1 ulp) instead of the
            // IEEE division sequence.
            T = T * __builtin_amdgcn_rcpf(1.0f - al);
            float v[9];
            const float w = al * T;
            v[6] = w * G0;
            v[7] = w * G1;
            v[8] = w * G2;
            const float dc = (r1.z * G0 + r1.w * G1 + rb * G2) - S;
            const float dL_dalpha = T * dc;
            S = fmaf(al, dc, S);
            // h = dL/do of this pixel = G dL/d(oG), zero where alpha = min(0.99, o G) saturates
            // (and, through gz, for lanes that skip the entry).
            const float h = gz * (e.raw > kAlphaMax ? 0.0f : dL_dalpha);
            v[5] = h;
            // dL/dpower = o G dL/d(oG) = o h. Moments of h over the pixel offsets: o and the conic,
            // the same for every pixel, turn them into the mean and conic gradients once per
            // Gaussian.
            const float mx = h * e.dx, my = h * e.dy;
            v[0] = mx;
            v[1] = my;
            v[2] = mx * e.dx;
            v[3] = mx * e.dy;
            v[4] = my * e.dy;
            // The record carries its Gaussian's id (the same in every lane): the row address is
            // formed in scalar registers.
            const uint32_t gid = (uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(r2.y));
            AccT *dst = acc + (size_t)gid * GSR_ACC_STRIDE;
            uint64_t red_mask = 0;
            if (BLOCK) {
                if (__popcll(am) >= p.threshold) {
                    red_mask = am;
                    const float mine = wave_sum9_scatter(v, lane);
                    if (sum9_issues(lane)) atomicAdd(&s_acc[j * 9 + sum9_slot(lane)], mine);
                    if (lane == 0) s_touch[j] = 1u;
                } else if (active) {
    #pragma unroll
                    for (int k = 0; k < 9; ++k) atomic_acc(dst + k, v[k]);
                    issued += 9;
                }
            } else {
                issued += emit9<MODE, SPLIT>(active, am, v, dst, p.threshold, lane, red_mask);
            }
            if (COUNT) {
                const int ca = __popcll(am);
                c_visit += 1;
                c_active += ca;
                if (ca) {
                    c_we += 1;
                    if (red_mask) {
                        c_red += 1;
                        c_instr += BLOCK ? 0 : ((SPLIT || MODE == GSR_BWD_SERIAL_REDUCE) ? 1 : 9);
                    } else {
                        c_plain += ca;
                        c_instr += 9;
                    }
                    if (lane == 0) atomicAdd(&s_cnt[CNT_HIST + ca], 1ull);
                }
            }
        };
#pragma unroll
        for (int q = BATCH / 64 - 1; q >= 0; --q) {
            // Visited entries two at a time, last first: both records are read before the first
            // is processed (an odd last one is paired with itself and not processed twice).
            for (uint64_t mq = vis[q]; mq;) {
                const int j1 = q * 64 + 63 - __builtin_clzll(mq);
                mq ^= 1ull << (j1 - q * 64);
                const bool two = mq != 0;
                const int j2 = two ? q * 64 + 63 - __builtin_clzll(mq) : j1;
                mq = two ? mq ^ (1ull << (j2 - q * 64)) : mq;
                const float4 a0 = s0[j1], a1 = s1[j1], a2 = s2[j1];
                const float4 b0 = s0[j2], b1 = s1[j2], b2 = s2[j2];
                visit(j1, a0, a1, a2);
                if (two) visit(j2, b0, b1, b2);
            }
        }
        if (BLOCK) {
            // Flush: consecutive lanes take consecutive values of one entry, so each wave-wide
            // atomic instruction covers about seven entries' 36-byte runs.
            __syncthreads();
            for (int i = tid; i < cnt * 9; i += TILE * TILE) {
                const int e = i / 9;
                const bool f = s_touch[e] != 0u;
                if (f) {
                    atomic_acc(acc + (size_t)__float_as_uint(s2[e].y) * GSR_ACC_STRIDE +
                                   (i - 9 * e), s_acc[i]);
                    ++issued;
                }
                if (COUNT && __ballot(f)) c_instr += 1;
            }
        }
    }
    if (COUNT) {
        atomicAdd(&s_cnt[CNT_LANE_ATOMICS], (unsigned long long)issued);
        if (lane == 0) {
            atomicAdd(&s_cnt[CNT_EVAL], (unsigned long long)c_eval);
            atomicAdd(&s_cnt[CNT_ACTIVE], (unsigned long long)c_active);
            atomicAdd(&s_cnt[CNT_WAVE_ENTRIES], (unsigned long long)c_we);
            atomicAdd(&s_cnt[CNT_REDUCED], (unsigned long long)c_red);
            atomicAdd(&s_cnt[CNT_PLAIN_LANES], (unsigned long long)c_plain);
            atomicAdd(&s_cnt[CNT_INSTRS], (unsigned long long)c_instr);
            atomicAdd(&s_cnt[CNT_VISITED], (unsigned long long)c_visit);
            atomicMax(&s_cnt[CNT_MAX_WAVE_VISITS], (unsigned long long)c_visit);
        }
        if (tid == 0) s_cnt[CNT_WALKED] = (unsigned long long)walk;
        __syncthreads();
        for (int i = tid; i < CNT_SLOTS; i += TILE * TILE)
            if (s_cnt[i]) {
                if (i == CNT_MAX_WAVE_VISITS) atomicMax(&p.counters[i], s_cnt[i]);
                else atomicAdd(&p.counters[i], s_cnt[i]);
            }
    }
}

template <int MODE, bool SPLIT>
__global__ __launch_bounds__(64) void wave_reduce_selftest_kernel(const float *vals, const uint8_t *active,
                                                                   int threshold, float *sums,
                                                                   unsigned long long *lane_atomics) {
    const int lane = threadIdx.x;
    const size_t i = (size_t)blockIdx.x * 64 + lane;
    float v[9];
    const bool act = active[i] != 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = act ? vals[i * 9 + k] : 0.0f;
    uint64_t red;
    const uint32_t issued = emit9<MODE, SPLIT, float>(act, __ballot(act), v, sums, threshold, lane, red);
    if (issued) atomicAdd(lane_atomics, (unsigned long long)issued);
}

// The batch's (view, tile) pairs in index order, or ordered by decreasing
// work (longest first, so the dispatcher's greedy assignment of workgroups to
// free CUs approximates longest-processing-time scheduling; a batch of views
// is one pool of tiles). Work = the tile's deepest n_contrib (tile_walk) or
// its list length. Counting sort on a log-scale bucket of the work (16
// buckets per octave), one block.

__device__ __forceinline__ void order_tiles_block(const ViewBatch &vb, int mode, uint2 *work) {
    __shared__ uint32_t s_count[256];
    // The views' tile bases and work arrays, copied once: indexing the by-value argument with a
    // per-item view number would reload them from memory for every item.
    __shared__ uint32_t s_base[kMaxViews + 1];
    __shared__ const uint32_t *s_walk[kMaxViews];
    __shared__ const uint2 *s_ranges[kMaxViews];
    const uint32_t n = vb.base[vb.n];
    if (threadIdx.x <= (unsigned)vb.n) s_base[threadIdx.x] = vb.base[threadIdx.x];
    if (threadIdx.x < (unsigned)vb.n) {
        s_walk[threadIdx.x] = vb.v[threadIdx.x].tile_walk;
        s_ranges[threadIdx.x] = vb.v[threadIdx.x].ranges;
    }
    if (threadIdx.x < 256) s_count[threadIdx.x] = 0;
    __syncthreads();
    const int nv = vb.n;
    const auto locate_s = [&](uint32_t i) {
        int v = 0;
        while (v + 1 < nv && i >= s_base[v + 1]) ++v;
        return make_uint2((uint32_t)v, i - s_base[v]);
    };
    if (mode == ORDER_IDENTITY) {
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) work[i] = locate_s(i);
        return;
    }
    const auto bucket = [&](uint2 vt) -> uint32_t {
        uint32_t w;
        if (mode == ORDER_BY_WALK) {
            w = s_walk[vt.x][vt.y];
        } else {
            const uint2 r = s_ranges[vt.x][vt.y];
            w = r.y - r.x;
        }
        const int b = w ? min(255, 1 + (int)(16.0f * __log2f((float)w))) : 0;
        return 255u - (uint32_t)b; // ascending key = descending work
    };
    // Four items per thread and round, their work values loaded together (positions clamped to
    // the last item instead of a test around each load, which would serialise the loads).
    // The first round's items stay in registers for the scatter pass (one round covers every
    // tile of a single view up to 4096 tiles), so that pass reloads nothing for them.
    constexpr int U = 4;
    uint2 vt0[U];
    uint32_t b0[U];
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        uint2 vt[U];
        uint32_t b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vt[u] = locate_s(min(i0 + u * blockDim.x, n - 1));
            b[u] = bucket(vt[u]);
        }
        if (i0 == threadIdx.x) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                vt0[u] = vt[u];
                b0[u] = b[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * blockDim.x < n) atomicAdd(&s_count[b[u]], 1u);
    }
    __syncthreads();
    // Exclusive scan of the 256 bucket counts by the first four waves.
    __shared__ uint32_t s_part[4];
    uint32_t c = 0, inc = 0;
    if (threadIdx.x < 256) {
        c = s_count[threadIdx.x];
        inc = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, 64);
            if ((threadIdx.x & 63) >= d) inc += o;
        }
        if ((threadIdx.x & 63) == 63) s_part[threadIdx.x >> 6] = inc;
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        uint32_t off = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) off += s_part[w];
        s_count[threadIdx.x] = off + inc - c;
    }
    __syncthreads();
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        uint2 vt[U];
        uint32_t b[U];
        if (i0 == threadIdx.x) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                vt[u] = vt0[u];
                b[u] = b0[u];
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                vt[u] = locate_s(min(i0 + u * blockDim.x, n - 1));
                b[u] = bucket(vt[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * blockDim.x < n) work[atomicAdd(&s_count[b[u]], 1u)] = vt[u];
    }
}

__global__ __launch_bounds__(1024) void order_tiles_kernel(ViewBatch vb, int mode, uint2 *work) {
    order_tiles_block(vb, mode, work);
}

// One view's backward set-up in one launch: block 0 builds the tile order (as
// order_tiles_kernel), the other blocks clear the listed accumulator rows, one thread per
// 16-byte chunk so that consecutive threads fill whole rows; the order's one-block latency
// overlaps the clearing's writes. m_dev (nullable): the list's length on the device, at most m.
__global__ __launch_bounds__(1024) void clear_rows_and_order_kernel(ViewBatch vb, int mode, uint2 *work,
                                                                     const uint32_t *ids, int64_t m,
                                                                     const uint32_t *m_dev, uint4 *acc,
                                                                     int chunks) {
    if (blockIdx.x == 0) {
        order_tiles_block(vb, mode, work);
        return;
    }
    const int64_t t = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
    const int64_t v = t / chunks;
    if (m_dev && (int64_t)*m_dev < m) m = *m_dev;
    if (v >= m) return;
    acc[(int64_t)ids[v] * chunks + (t - v * chunks)] = make_uint4(0u, 0u, 0u, 0u);
}

template <int TILE, int BATCH>
hipError_t fwd_t(const ViewBatch &vb, int remap, const uint2 *work, hipStream_t st) {
    const int n_tiles = vb.v[0].cam.grid_x * vb.v[0].cam.grid_y;
    const unsigned grid = work ? vb.base[vb.n] : (unsigned)grid_for_tiles(n_tiles, remap);
    if (grid == 0) return hipSuccess;
    composite_fwd_kernel<TILE, BATCH><<<grid, TILE * TILE, 0, st>>>(vb, remap, work);
    return hipGetLastError();
}

template <int TILE, int BATCH, typename AccT>
hipError_t bwd_acc(const dim3 grid, const ViewBatch &vb, int remap, int mode, bool count, bool split,
                   const BwdParams &p, const uint2 *work, hipStream_t st) {
    const dim3 block(TILE * TILE);
#define GSR_BWD(M, C, S) composite_bwd_kernel<TILE, BATCH, M, C, S, AccT><<<grid, block, 0, st>>>(vb, remap, work, p)
    if (mode == GSR_BWD_PLAIN_ATOMIC) {
        if (count) GSR_BWD(GSR_BWD_PLAIN_ATOMIC, true, false);
        else GSR_BWD(GSR_BWD_PLAIN_ATOMIC, false, false);
    } else if (mode == GSR_BWD_SERIAL_REDUCE) {
        if (count) GSR_BWD(GSR_BWD_SERIAL_REDUCE, true, true);
        else GSR_BWD(GSR_BWD_SERIAL_REDUCE, false, true);
    } else if (mode == GSR_BWD_BLOCK_REDUCE) {
        if (count) GSR_BWD(GSR_BWD_BLOCK_REDUCE, true, true);
        else GSR_BWD(GSR_BWD_BLOCK_REDUCE, false, true);
    } else if (split) {
        if (count) GSR_BWD(GSR_BWD_WAVE_REDUCE, true, true);
        else GSR_BWD(GSR_BWD_WAVE_REDUCE, false, true);
    } else {
        if (count) GSR_BWD(GSR_BWD_WAVE_REDUCE, true, false);
        else GSR_BWD(GSR_BWD_WAVE_REDUCE, false, false);
    }
#undef GSR_BWD
    return hipGetLastError();
}

template <int TILE, int BATCH>
hipError_t bwd_t(const ViewBatch &vb, int remap, int mode, bool count, bool split, bool f64, const BwdParams &p,
                 const uint2 *work, hipStream_t st) {
    const int n_tiles = vb.v[0].cam.grid_x * vb.v[0].cam.grid_y;
    const dim3 grid(work ? vb.base[vb.n] : (unsigned)grid_for_tiles(n_tiles, remap));
    if (grid.x == 0) return hipSuccess;
    return f64 ? bwd_acc<TILE, BATCH, double>(grid, vb, remap, mode, count, split, p, work, st)
               : bwd_acc<TILE, BATCH, float>(grid, vb, remap, mode, count, split, p, work, st);
}

} // namespace

#ifndef GSR_COMPOSITE_COMPILER_REDUCE
hipError_t launch_order_tiles(const ViewBatch &vb, int mode, uint2 *work, hipStream_t st) {
    if (vb.n <= 0 || vb.base[vb.n] == 0) return hipSuccess;
    order_tiles_kernel<<<1, 1024, 0, st>>>(vb, mode, work);
    return hipGetLastError();
}

hipError_t launch_clear_rows_and_order(const ViewBatch &vb, int mode, uint2 *work, const uint32_t *ids, int64_t m,
                                       const uint32_t *m_dev, void *acc, bool acc_f64, hipStream_t st) {
    if (vb.n != 1) return hipErrorInvalidValue;
    const int chunks = GSR_ACC_STRIDE * (acc_f64 ? 8 : 4) / 16;
    const int64_t threads = (m > 0 ? m : 0) * chunks;
    const unsigned blocks = (unsigned)(1 + (threads + 1023) / 1024);
    clear_rows_and_order_kernel<<<blocks, 1024, 0, st>>>(vb, mode, work, ids, m > 0 ? m : 0, m_dev,
                                                         static_cast<uint4 *>(acc), chunks);
    return hipGetLastError();
}

hipError_t launch_composite_fwd(const ViewBatch &vb, int t, int lds_batch, int remap, const uint2 *work,
                                hipStream_t st) {
    if (vb.n <= 0 || (vb.n > 1 && !work)) return hipErrorInvalidValue;
#define GSR_F(T, B) return fwd_t<T, B>(vb, remap, work, st)
    if (t == 8) GSR_F(8, 64);
    if (t == 16) {
        if (lds_batch == 64) GSR_F(16, 64);
        if (lds_batch == 128) GSR_F(16, 128);
        GSR_F(16, 256);
    }
    if (lds_batch == 64) GSR_F(32, 64);
    if (lds_batch == 128) GSR_F(32, 128);
    GSR_F(32, 256);
#undef GSR_F
}

hipError_t launch_composite_bwd(const ViewBatch &vb, int t, int lds_batch, int remap, int mode, bool count,
                                bool lane_split, bool acc_f64, const BwdParams &p, const uint2 *work,
                                hipStream_t st) {
    if (vb.n <= 0 || (vb.n > 1 && !work)) return hipErrorInvalidValue;
#define GSR_B(T, B) return bwd_t<T, B>(vb, remap, mode, count, lane_split, acc_f64, p, work, st)
    if (t == 8) GSR_B(8, 64);
    if (t == 16) {
        if (lds_batch == 64) GSR_B(16, 64);
        if (lds_batch == 128) GSR_B(16, 128);
        GSR_B(16, 256);
    }
    if (lds_batch == 64) GSR_B(32, 64);
    if (lds_batch == 128) GSR_B(32, 128);
    GSR_B(32, 256);
#undef GSR_B
}

hipError_t launch_wave_reduce_selftest(const float *vals, const uint8_t *active, int n_waves, int mode,
                                       int threshold, int lane_split, float *sums, unsigned long long *lane_atomics,
                                       hipStream_t st) {
    if (n_waves <= 0) return hipSuccess;
    if (mode == GSR_BWD_PLAIN_ATOMIC)
        wave_reduce_selftest_kernel<GSR_BWD_PLAIN_ATOMIC, false><<<n_waves, 64, 0, st>>>(vals, active, threshold,
                                                                                         sums, lane_atomics);
    else if (mode == GSR_BWD_SERIAL_REDUCE)
        wave_reduce_selftest_kernel<GSR_BWD_SERIAL_REDUCE, true><<<n_waves, 64, 0, st>>>(vals, active, threshold,
                                                                                         sums, lane_atomics);
    else if (lane_split)
        wave_reduce_selftest_kernel<GSR_BWD_WAVE_REDUCE, true><<<n_waves, 64, 0, st>>>(vals, active, threshold, sums,
                                                                                       lane_atomics);
    else
        wave_reduce_selftest_kernel<GSR_BWD_WAVE_REDUCE, false><<<n_waves, 64, 0, st>>>(vals, active, threshold,
                                                                                        sums, lane_atomics);
    return hipGetLastError();
}

#else
// This file compiled a second time with the compiler's atomic optimizer on: only the plain-atomic
// backward is instantiated, so that build differs from the default one in the atomic rewrite alone.
namespace {
template <int TILE, int BATCH>
hipError_t bwd_compiler_reduce_t(const ViewBatch &vb, int remap, bool f64, const BwdParams &p, const uint2 *work,
                                 hipStream_t st) {
    const int n_tiles = vb.v[0].cam.grid_x * vb.v[0].cam.grid_y;
    const dim3 grid(work ? vb.base[vb.n] : (unsigned)grid_for_tiles(n_tiles, remap));
    if (grid.x == 0) return hipSuccess;
    if (f64)
        composite_bwd_kernel<TILE, BATCH, GSR_BWD_PLAIN_ATOMIC, false, false, double>
            <<<grid, TILE * TILE, 0, st>>>(vb, remap, work, p);
    else
        composite_bwd_kernel<TILE, BATCH, GSR_BWD_PLAIN_ATOMIC, false, false, float>
            <<<grid, TILE * TILE, 0, st>>>(vb, remap, work, p);
    return hipGetLastError();
}
} // namespace

hipError_t launch_composite_bwd_compiler_reduce(const ViewBatch &vb, int t, int lds_batch, int remap, bool acc_f64,
                                                const BwdParams &p, const uint2 *work, hipStream_t st) {
    if (vb.n <= 0 || (vb.n > 1 && !work)) return hipErrorInvalidValue;
#define GSR_B(T, B) return bwd_compiler_reduce_t<T, B>(vb, remap, acc_f64, p, work, st)
    if (t == 8) GSR_B(8, 64);
    if (t == 16) {
        if (lds_batch == 64) GSR_B(16, 64);
        if (lds_batch == 128) GSR_B(16, 128);
        GSR_B(16, 256);
    }
    if (lds_batch == 64) GSR_B(32, 64);
    if (lds_batch == 128) GSR_B(32, 128);
    GSR_B(32, 256);
#undef GSR_B
}
#endif

} // namespace gsr
