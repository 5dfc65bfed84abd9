// Tile binning for the 3DGS rasteriser: device exclusive scan, stable LSD
// radix sort, (tile, Gaussian) pair emission and per-tile ranges.
//
// The lists the gradient kernel consumes are ordered by (tile, depth, index)
// (3DGS sorts one composite (tile, depth) key). Here the LSD radix sort of
// that composite key is split in two: the depth digits are sorted over the n
// Gaussians before the pairs are emitted (emission in depth order keeps the
// relative order of equal tiles), then only the tile digits are sorted over
// the P pairs. Same order, but P is touched by 1-2 passes instead of ~6.
#include "device_common.hpp"

namespace gsr {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTileItems = kThreads * kItems; // 4096 items per block
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread across the block; returns the
// thread's exclusive prefix and the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_wave, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint32_t x = s_wave[w];
        off += (w < wave) ? x : 0u;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// A thread's K items at positions pos(k) < n, zero past the end. The loads are
// unconditional (positions clamped to n - 1, n >= 1) and issued together, the
// gathered ones after all their indices: bounds tests around each load would
// make the compiler wait for every load before issuing the next.
template <int K, bool GATHER, typename Pos>
__device__ __forceinline__ void load_items(const uint32_t *in, const uint32_t *gather, int64_t n, Pos pos,
                                           uint32_t (&v)[K]) {
    int64_t idx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) idx[k] = pos(k) < n ? pos(k) : n - 1;
    if (GATHER) {
#pragma unroll
        for (int k = 0; k < K; ++k) idx[k] = gather[idx[k]];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = in[idx[k]];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = pos(k) < n ? v[k] : 0u;
}

// A thread's kItems consecutive items [base, base + kItems): four 16-byte
// loads when the chunk is whole, ungathered and 16-byte aligned (a wave's
// scalar loads of consecutive chunks would fetch every line kItems times
// through the CU's L1), else the clamped scalar loads.
template <bool GATHER>
__device__ __forceinline__ void load_chunk(const uint32_t *in, const uint32_t *gather, int64_t n, int64_t base,
                                           uint32_t (&v)[kItems]) {
    if (!GATHER && base + kItems <= n && ((reinterpret_cast<uintptr_t>(in) & 15) == 0)) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
        uint4 q[kItems / 4];
#pragma unroll
        for (int c = 0; c < kItems / 4; ++c) q[c] = p[c];
#pragma unroll
        for (int c = 0; c < kItems / 4; ++c) {
            v[4 * c] = q[c].x;
            v[4 * c + 1] = q[c].y;
            v[4 * c + 2] = q[c].z;
            v[4 * c + 3] = q[c].w;
        }
        return;
    }
    if (base >= n) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = 0u;
        return;
    }
    // clamped loads at 32-bit offsets from the chunk's start (64-bit positions would take two
    // registers each)
    const int last = n - base < kItems ? (int)(n - base) - 1 : kItems - 1;
    const uint32_t *src = GATHER ? gather + base : in + base;
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = src[k < last ? k : last];
    if (GATHER) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = in[v[k]];
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = k <= last ? v[k] : 0u;
}

// out[base + k] = run + v[0] + ... + v[k-1] for the positions below n (16-byte stores when whole
// and aligned); returns run plus all kItems values.
__device__ __forceinline__ uint32_t store_chunk_scan(uint32_t *out, int64_t n, int64_t base, uint32_t run,
                                                     const uint32_t (&v)[kItems]) {
    uint32_t o[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + kItems <= n && ((reinterpret_cast<uintptr_t>(out) & 15) == 0)) {
        uint4 *p = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int c = 0; c < kItems / 4; ++c) p[c] = make_uint4(o[4 * c], o[4 * c + 1], o[4 * c + 2], o[4 * c + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (base + k < n) out[base + k] = o[k];
    }
    return run;
}

// Per-block sums of 4096 consecutive items.
template <bool GATHER>
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t *in, const uint32_t *gather,
                                                               int64_t n, uint32_t *partials) {
    __shared__ uint32_t s_wave[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTileItems + threadIdx.x;
    uint32_t v[kItems];
    load_items<kItems, GATHER>(in, gather, n, [&](int k) { return base + (int64_t)k * kThreads; }, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += v[k];
    uint32_t total;
    block_exclusive_scan(s, s_wave, total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Exclusive scan of each block's 4096 items plus the block's offset
// (offsets == nullptr: single block, offset 0; fused != 0: offsets holds the
// blocks' unscanned sums and each block adds up those before it itself, for
// grids too small to pay for a launch that scans them). Thread t owns items
// [t*16, t*16+16) of the block so the order is the natural one.
template <bool GATHER>
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const uint32_t *in, const uint32_t *gather, int64_t n,
                                                              const uint32_t *offsets, int fused, uint32_t *out,
                                                              uint32_t *total_out) {
    __shared__ uint32_t s_wave[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    load_chunk<GATHER>(in, gather, n, base, v);
    uint32_t boff = 0;
    if (offsets && fused) {
        uint32_t acc = 0;
        for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += kThreads) acc += offsets[j];
        block_exclusive_scan(acc, s_wave, boff);
    } else if (offsets) {
        boff = offsets[blockIdx.x];
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += v[k];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, s_wave, total) + boff;
    run = store_chunk_scan(out, n, base, run, v);
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) {
        // Last item of the last block: its exclusive prefix plus itself is the grand total.
        *total_out = run;
    }
}

// Exclusive scan of up to kOneBlockMax items by one 1024-thread block, in
// tiles of 16384 (thread t owns items [t*16, t*16+16) of a tile), carrying
// the running total from tile to tile: one launch where the two-level scan
// needs three.
constexpr int kOneThreads = 1024;
constexpr int64_t kOneBlockMax = 4 * kOneThreads * kItems; // 65536

template <bool GATHER, int NT>
__global__ __launch_bounds__(kOneThreads) void scan_one_block_kernel(const uint32_t *in, const uint32_t *gather,
                                                                     int64_t n, uint32_t *out, uint32_t *total_out) {
    // Rounds of NT tiles of kOneThreads * kItems items; a round's loads are all issued before its
    // first scan, so the block waits for memory once per round, not once per tile (more than two
    // tiles in flight would exceed the 128 registers a 1024-thread block allows). In-place use
    // (out == in) is safe: each thread stores only the items it loaded itself.
    constexpr int64_t TILE = (int64_t)kOneThreads * kItems;
    __shared__ uint32_t s_wave[NT][kOneThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t round = 0; round < n; round += NT * TILE) {
        uint32_t v[NT][kItems];
#pragma unroll
        for (int t = 0; t < NT; ++t)
            load_chunk<GATHER>(in, gather, n, round + t * TILE + (int64_t)threadIdx.x * kItems, v[t]);
        uint32_t sum[NT], inc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            sum[t] = 0;
#pragma unroll
            for (int k = 0; k < kItems; ++k) sum[t] += v[t][k];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) inc[t] = wave_inclusive_scan(sum[t], lane);
        if (lane == 63) {
#pragma unroll
            for (int t = 0; t < NT; ++t) s_wave[t][wave] = inc[t];
        }
        __syncthreads();
        uint32_t off[NT], tot[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            off[t] = 0;
            tot[t] = 0;
#pragma unroll
            for (int w = 0; w < kOneThreads / 64; ++w) {
                const uint32_t x = s_wave[t][w];
                off[t] += (w < wave) ? x : 0u;
                tot[t] += x;
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            store_chunk_scan(out, n, round + t * TILE + (int64_t)threadIdx.x * kItems, carry + off[t] + inc[t] - sum[t],
                             v[t]);
            carry += tot[t];
        }
    }
    if (total_out && threadIdx.x == 0) *total_out = carry;
}

template <bool GATHER>
void launch_scan_one_block(const uint32_t *in, const uint32_t *gather, int64_t n, uint32_t *out, uint32_t *total,
                           hipStream_t st) {
    if (n <= (int64_t)kOneThreads * kItems)
        scan_one_block_kernel<GATHER, 1><<<1, kOneThreads, 0, st>>>(in, gather, n, out, total);
    else
        scan_one_block_kernel<GATHER, 2><<<1, kOneThreads, 0, st>>>(in, gather, n, out, total);
}

// out[i] = in[gather[i]]
__global__ __launch_bounds__(256) void gather_u32_kernel(const uint32_t *in, const uint32_t *gather, int64_t n,
                                                         uint32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = in[gather[i]];
}

} // namespace

size_t scan_partial_count(int64_t n) {
    // Level sizes: ceil(n/4096) + ceil(that/4096) + ... (plus slack).
    size_t total = 0;
    int64_t m = n;
    while (m > kTileItems) {
        m = (m + kTileItems - 1) / kTileItems;
        total += (size_t)m + 1;
    }
    return total + 8;
}

hipError_t device_exclusive_scan(const uint32_t *in, const uint32_t *gather, uint32_t *out, int64_t n,
                                 uint32_t *total, uint32_t *partials, hipStream_t st) {
    if (n <= 0) {
        if (total) return launch_fill_u32(total, 0u, 1, st);
        return hipSuccess;
    }
    const int64_t blocks = (n + kTileItems - 1) / kTileItems;
    if (gather && blocks > 1) {
        // More than one tile: gather into out first (index reads coalesced, one random read per
        // item), then scan out in place; the scan kernels would each gather again, through
        // thread-contiguous index chunks. out aliases neither in nor gather.
        gather_u32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(in, gather, n, out);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return device_exclusive_scan(out, nullptr, out, n, total, partials, st);
    }
    if (blocks == 1) {
        if (gather) scan_apply_kernel<true><<<1, kThreads, 0, st>>>(in, gather, n, nullptr, 0, out, total);
        else scan_apply_kernel<false><<<1, kThreads, 0, st>>>(in, gather, n, nullptr, 0, out, total);
        return hipGetLastError();
    }
    if (n <= kOneBlockMax) {
        if (gather) launch_scan_one_block<true>(in, gather, n, out, total, st);
        else launch_scan_one_block<false>(in, gather, n, out, total, st);
        return hipGetLastError();
    }
    if (gather) scan_reduce_kernel<true><<<(unsigned)blocks, kThreads, 0, st>>>(in, gather, n, partials);
    else scan_reduce_kernel<false><<<(unsigned)blocks, kThreads, 0, st>>>(in, gather, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // Up to 128 blocks each applying block adds up the partials before it; else the partials are
    // scanned in place (recursively) first.
    const int fused = blocks <= 128 ? 1 : 0;
    if (!fused) {
        e = device_exclusive_scan(partials, nullptr, partials, blocks, nullptr, partials + blocks + 1, st);
        if (e != hipSuccess) return e;
    }
    if (gather)
        scan_apply_kernel<true><<<(unsigned)blocks, kThreads, 0, st>>>(in, gather, n, partials, fused, out, total);
    else
        scan_apply_kernel<false><<<(unsigned)blocks, kThreads, 0, st>>>(in, gather, n, partials, fused, out, total);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Radix sort: 8-bit digits (fewer in the last pass), reduce-then-scan.
namespace {

constexpr int kBins = 256;
constexpr int64_t kFusedScanBlocks = 128; // radix passes of at most this many blocks derive offsets in the scatter

// Sorts of fewer than kSmallSort items use 1024-item blocks (4 per thread)
// instead of 4096: the visible Gaussians and pairs of a single view would
// otherwise fill only a few dozen to a few hundred workgroups.
constexpr int64_t kSmallSort = int64_t(1) << 21;
__host__ __device__ __forceinline__ int sort_items(int64_t n) { return n < kSmallSort ? 4 : kItems; }
__host__ __device__ __forceinline__ int64_t sort_blocks(int64_t n) {
    const int64_t t = (int64_t)kThreads * sort_items(n);
    return (n + t - 1) / t;
}

// A sort whose item count and key range exist only on the device (enqueued before the host has
// read them back): n_dev (nullable) holds the item count, at most the launch's n, and range_dev
// (nullable) holds (max ~key, max key). A pass whose digit lies wholly above the keys' highest
// varying bit copies its items unchanged: a stable pass over a digit that every key shares is the
// identity, and the copy keeps the host's buffer parity.
__device__ __forceinline__ int64_t dev_items(int64_t n, const uint32_t *n_dev) {
    return n_dev ? (n < (int64_t)*n_dev ? n : (int64_t)*n_dev) : n;
}
__device__ __forceinline__ bool dev_skip(int shift, const uint32_t *range_dev) {
    if (!range_dev) return false;
    const uint32_t lo = ~range_dev[0], hi = range_dev[1];
    const int bits = lo < hi ? 32 - __clz((int)(lo ^ hi)) : 0;
    return shift >= bits;
}

// Digit histogram of each block of ITEMS * 256 items, written digit-major (mask + 1
// rows of `stride` entries, one column per block) so one exclusive scan of the whole
// table yields every block's output offsets. Columns from gridDim.x to stride - 1 (the
// padding of a table the scatter reads with 16-byte loads) are written as zeros.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t *keys, int64_t n, int shift,
                                                              uint32_t mask, uint32_t *hist, int64_t stride,
                                                              const uint32_t *n_dev, const uint32_t *range_dev) {
    n = dev_items(n, n_dev);
    if (n <= 0 || dev_skip(shift, range_dev)) return; // the scatter then ignores the table
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x <= mask)
        for (int64_t c = gridDim.x; c < stride; ++c) hist[(int64_t)threadIdx.x * stride + c] = 0u;
    if ((int64_t)blockIdx.x * (kThreads * ITEMS) >= n) { // past the device-side count: an empty column
        if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * stride + blockIdx.x] = 0u;
        return;
    }
    __shared__ uint32_t s_count[kBins];
    s_count[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kThreads * ITEMS) + threadIdx.x;
    uint32_t k[ITEMS];
    const auto pos = [&](int r) { return base + (int64_t)r * kThreads; };
    load_items<ITEMS, false>(keys, nullptr, n, pos, k);
    // A narrow digit (the top pass of the tile sort: a few dozen values over long sorted runs)
    // puts many lanes of a wave on one LDS counter, where their atomics serialise: lanes find
    // their equal-digit peers with one ballot per bit and one lane adds the group's size. Wide
    // digits vary from lane to lane and keep one atomic per lane (measured faster there: on the
    // 7.5M-pair tile sort at 1080p, peers up to 6 bits took 122.5 us, up to 8 bits 136 us, up
    // to 5 bits 127 us).
    const int nbits = __popc(mask);
    const int lane = threadIdx.x & 63;
    if (nbits <= 6) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const bool valid = pos(r) < n;
            const uint32_t d = (k[r] >> shift) & mask;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                const uint64_t bal = __ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bal : ~bal;
            }
            if (valid && __ffsll((long long)peers) - 1 == lane) atomicAdd(&s_count[d], (uint32_t)__popcll(peers));
        }
    } else {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (pos(r) < n) atomicAdd(&s_count[(k[r] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * stride + blockIdx.x] = s_count[threadIdx.x];
}

// Stable scatter of one block of ITEMS * 256 items. Wave w ranks items
// [w*64*ITEMS, (w+1)*64*ITEMS) of the block in ITEMS rounds of 64; lanes
// with equal digits find each other with one ballot per digit bit. Items are
// staged in LDS in digit order and written out with consecutive threads on
// consecutive addresses. offsets: the scanned digit-major table (rows of
// `stride` = gridDim.x entries), or with fused != 0 the unscanned histogram
// table (rows padded with zeros to `stride`, a multiple of 4), from which each
// block derives its own offsets (thread d sums row d with 16-byte loads: its
// total and the part before this block; a scan over the digit totals adds the
// rows before it) - for tables of few blocks, where a separate scan launch
// costs more than these reads.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(const uint32_t *keys_in, const uint32_t *vals_in,
                                                                 uint32_t *keys_out, uint32_t *vals_out, int64_t n,
                                                                 int shift, int nbits, const uint32_t *offsets,
                                                                 int64_t stride, int fused, const uint32_t *n_dev,
                                                                 const uint32_t *range_dev) {
    constexpr int TILE_ITEMS = kThreads * ITEMS;
    n = dev_items(n, n_dev);
    if ((int64_t)blockIdx.x * TILE_ITEMS >= n) return; // past the device-side count: no items
    if (dev_skip(shift, range_dev)) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int64_t i = (int64_t)blockIdx.x * TILE_ITEMS + (int64_t)r * kThreads + threadIdx.x;
            if (i < n) {
                keys_out[i] = keys_in[i];
                vals_out[i] = vals_in[i];
            }
        }
        return;
    }
    __shared__ uint32_t s_wcount[kWaves][kBins];
    __shared__ uint32_t s_dstart[kBins];
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_key[TILE_ITEMS];
    __shared__ uint32_t s_val[TILE_ITEMS];
    __shared__ uint32_t s_goff[kBins];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t mask = (1u << nbits) - 1u;
    for (int i = threadIdx.x; i < kWaves * kBins; i += kThreads) (&s_wcount[0][0])[i] = 0;
    if (fused) {
        const uint32_t d = threadIdx.x; // kThreads == kBins
        uint32_t before = 0, all = 0;
        if (d <= mask) {
            // Eight 16-byte loads in flight per round (a row of at most 128 columns takes four).
            const uint4 *row = reinterpret_cast<const uint4 *>(offsets + (int64_t)d * stride);
            const int64_t me = blockIdx.x;
#pragma unroll 8
            for (int64_t q = 0; q < (stride >> 2); ++q) {
                const uint4 h = row[q];
                const int64_t c = 4 * q;
                all += h.x + h.y + h.z + h.w;
                before += (c < me ? h.x : 0u) + (c + 1 < me ? h.y : 0u) + (c + 2 < me ? h.z : 0u) +
                          (c + 3 < me ? h.w : 0u);
            }
        }
        uint32_t unused;
        s_goff[d] = block_exclusive_scan(all, s_wave, unused) + before;
    }
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * TILE_ITEMS;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[ITEMS], val[ITEMS], pos[ITEMS];
    const int64_t first = base + (int64_t)wave * (ITEMS * 64) + lane;
    const auto at = [&](int r) { return first + r * 64; };
    load_items<ITEMS, false>(keys_in, nullptr, n, at, key);
    load_items<ITEMS, false>(vals_in, nullptr, n, at, val);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = at(r) < n;
        const uint32_t d = (key[r] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const int leader = __ffsll((long long)peers) - 1;
        uint32_t old = 0;
        if (valid && rank == 0) old = atomicAdd(&s_wcount[wave][d], (uint32_t)__popcll(peers));
        old = __shfl(old, leader < 0 ? 0 : leader, 64);
        pos[r] = valid ? old + rank : 0xffffffffu;
    }
    __syncthreads();
    // Per digit: exclusive prefix over the waves, then over the digits.
    uint32_t tot = 0;
    {
        const int d = threadIdx.x; // kThreads == kBins
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            uint32_t c = s_wcount[w][d];
            s_wcount[w][d] = tot;
            tot += c;
        }
    }
    uint32_t block_total;
    const uint32_t dstart = block_exclusive_scan(tot, s_wave, block_total);
    s_dstart[threadIdx.x] = dstart;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (pos[r] == 0xffffffffu) continue;
        const uint32_t d = (key[r] >> shift) & mask;
        const uint32_t slot = s_dstart[d] + s_wcount[wave][d] + pos[r];
        s_key[slot] = key[r];
        s_val[slot] = val[r];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < block_total; i += kThreads) {
        const uint32_t k = s_key[i];
        const uint32_t d = (k >> shift) & mask;
        const int64_t dst = (int64_t)(fused ? s_goff[d] : offsets[(int64_t)d * stride + blockIdx.x]) + (i - s_dstart[d]);
        keys_out[dst] = k;
        vals_out[dst] = s_val[i];
    }
}

template <int ITEMS>
hipError_t radix_pass(const uint32_t *k_in, const uint32_t *v_in, uint32_t *k_out, uint32_t *v_out, int64_t n,
                      int shift, int nb, int64_t blocks, uint32_t *hist, uint32_t *partials, const uint32_t *n_dev,
                      const uint32_t *range_dev, hipStream_t st) {
    // Few blocks: each scatter block reads the histogram rows itself instead of a scan launch,
    // over rows padded to whole 16-byte groups.
    const int fused = blocks <= kFusedScanBlocks ? 1 : 0;
    const int64_t stride = fused ? (blocks + 3) & ~int64_t(3) : blocks;
    radix_hist_kernel<ITEMS><<<(unsigned)blocks, kThreads, 0, st>>>(k_in, n, shift, (1u << nb) - 1u, hist, stride,
                                                                     n_dev, range_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (!fused) {
        e = device_exclusive_scan(hist, nullptr, hist, blocks << nb, nullptr, partials, st); // (1 << nb) rows
        if (e != hipSuccess) return e;
    }
    radix_scatter_kernel<ITEMS><<<(unsigned)blocks, kThreads, 0, st>>>(k_in, v_in, k_out, v_out, n, shift, nb, hist,
                                                                        stride, fused, n_dev, range_dev);
    return hipGetLastError();
}

} // namespace

size_t radix_hist_count(int64_t n) {
    // Room for every sort of at most n items: below kSmallSort the blocks are smaller, so a
    // shorter sort can need more blocks than a longer one.
    int64_t b = sort_blocks(n);
    if (n >= kSmallSort) b = b > sort_blocks(kSmallSort - 1) ? b : sort_blocks(kSmallSort - 1);
    return (size_t)(b + 4) * kBins + 8; // + 4 columns: a fused table's rows are padded to a multiple of 4
}

bool radix_sort_fused(int64_t n) { return sort_blocks(n) <= kFusedScanBlocks; }

hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, int64_t n, int bits,
                            uint32_t *hist, uint32_t *partials, int *which, hipStream_t st, const uint32_t *n_dev,
                            const uint32_t *range_dev) {
    *which = 0;
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int64_t blocks = sort_blocks(n);
    const bool small = sort_items(n) == 4;
    uint32_t *ks[2] = {k0, k1}, *vs[2] = {v0, v1};
    // As few passes as 8-bit digits allow. Sorts of 1024-item blocks take 8-bit digits and the
    // remainder last, whose table has only 1 << remainder rows (12 bits as 8 + 4 measured faster
    // than as 6 + 6 on 0.8M pairs: the narrow last pass has a one-launch scan). Sorts of 4096-item
    // blocks split the bits evenly: fewer digits make longer runs per block and digit, so the
    // scatter writes fuller lines (13 bits on 7.5M pairs: 7 + 6 took 125 us, 8 + 5 134 us).
    const int passes = (bits + 7) / 8;
    const bool even = !small;
    int cur = 0;
    for (int p = 0, shift = 0; p < passes; ++p) {
        const int rest = bits - shift;
        const int nb = even ? (rest + (passes - p) - 1) / (passes - p) : (rest < 8 ? rest : 8);
        const hipError_t e =
            small ? radix_pass<4>(ks[cur], vs[cur], ks[cur ^ 1], vs[cur ^ 1], n, shift, nb, blocks, hist, partials,
                                  n_dev, range_dev, st)
                  : radix_pass<kItems>(ks[cur], vs[cur], ks[cur ^ 1], vs[cur ^ 1], n, shift, nb, blocks, hist,
                                       partials, n_dev, range_dev, st);
        if (e != hipSuccess) return e;
        cur ^= 1;
        shift += nb;
    }
    *which = cur;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
namespace {

// Inclusive prefix maximum over the 64 lanes (signed), in DPP steps: row shifts by 1, 2, 4 and
// 8 within each 16-lane row, then the row broadcasts of lanes 15 and 31 (lanes a step has no
// source for keep their value).
__device__ __forceinline__ int wave_prefix_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xF, 0xF, false)); // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xF, 0xF, false)); // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xF, 0xF, false)); // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xF, 0xF, false)); // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xA, 0xF, false)); // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xC, 0xF, false)); // row_bcast:31
    return v;
}

// A wave takes 64 consecutive depth-ordered Gaussians and writes their pairs together: the
// wave's pairs are one contiguous run of the list (each Gaussian's rectangle row by row, the
// Gaussians in depth order), so lane l writes entries l, l + 64, ... of that run and each
// store instruction covers consecutive addresses. Entry k belongs to the last of the 64
// Gaussians whose exclusive prefix count is at most k. For each window of 64 entries, every
// Gaussian with pairs that starts inside the window marks its start in LDS with its index,
// and a prefix maximum over the lanes carries each mark to the entries after it (entries
// before the window's first mark belong to the Gaussian that ended the previous window).
__global__ __launch_bounds__(256) void emit_pairs_kernel(int64_t n, const uint32_t *sorted_ids,
                                                          const uint32_t *offsets, const float4 *rec,
                                                          const int32_t *radius, DevCamera cam, uint32_t *pair_tile,
                                                          uint32_t *pair_id, uint32_t cap) {
    __shared__ uint32_t s_pre[4][64], s_off[4][64], s_g[4][64];
    __shared__ int s_x0[4][64], s_y0[4][64], s_w[4][64], s_mark[4][64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
    uint32_t o = 0, g = 0;
    if (i < n) {
        g = sorted_ids[i];
        const int r = radius[g];
        if (r > 0) {
            const float4 r0 = rec[3 * (int64_t)g];
            rect_of(r0.x, r0.y, r, cam, x0, x1, y0, y1);
            o = offsets[i];
        }
    }
    const uint32_t cnt = (uint32_t)((x1 - x0) * (y1 - y0));
    uint32_t inc = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, d, 64);
        if (lane >= d) inc += t;
    }
    const uint32_t pre = inc - cnt;
    s_pre[wave][lane] = pre;
    s_off[wave][lane] = o;
    s_g[wave][lane] = g;
    s_x0[wave][lane] = x0;
    s_y0[wave][lane] = y0;
    s_w[wave][lane] = x1 - x0;
    __syncthreads();
    const uint32_t total = (uint32_t)__shfl((int)inc, 63, 64);
    int carry = -1; // the Gaussian that owns the entry before the window
    for (uint32_t w0 = 0; w0 < total; w0 += 64) {
        s_mark[wave][lane] = -1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (cnt > 0 && pre >= w0 && pre - w0 < 64u) s_mark[wave][pre - w0] = lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int j = max(wave_prefix_max(s_mark[wave][lane]), carry);
        carry = __builtin_amdgcn_readlane(j, 63);
        __builtin_amdgcn_wave_barrier();
        const uint32_t k = w0 + (uint32_t)lane;
        if (k >= total) continue;
        const uint32_t local = k - s_pre[wave][j];
        const uint32_t w = (uint32_t)s_w[wave][j];
        const uint32_t row = local / w;
        const uint32_t oo = s_off[wave][j] + local;
        if (oo < cap) { // pairs past the buffer's capacity are dropped (the overflow word flags it)
            pair_tile[oo] = (uint32_t)((s_y0[wave][j] + (int)row) * cam.grid_x + s_x0[wave][j] + (int)(local - row * w));
            pair_id[oo] = s_g[wave][j];
        }
    }
}

// Capacity mode: overflow[0] = 1 when the pairs did not fit (the lists then hold the first cap).
__global__ __launch_bounds__(64) void pair_overflow_kernel(const uint32_t *total, uint32_t cap, uint32_t *overflow) {
    if (threadIdx.x == 0) overflow[0] = total[0] > cap ? 1u : 0u;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, uint32_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// Every tile's [start, end) in the tile-sorted list, written once per tile with no
// clearing pass: thread i (0 <= i <= P) looks at the boundary before position i,
// between tile a = tile[i - 1] (-1 before the list) and b = tile[i] (n_tiles past it).
// Where a < b it ends a, starts b and gives each tile strictly between them the empty
// range [i, i). P_dev (nullable): a device-side count that bounds P (capacity mode).
__global__ __launch_bounds__(256) void tile_ranges_kernel(int64_t P, const uint32_t *P_dev, const uint32_t *tile,
                                                           uint2 *ranges, uint32_t n_tiles) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P_dev && (int64_t)*P_dev < P) P = *P_dev;
    if (i > P) return;
    const int64_t a = i == 0 ? -1 : (int64_t)min(tile[i - 1], n_tiles);
    const int64_t b = i == P ? (int64_t)n_tiles : (int64_t)min(tile[i], n_tiles);
    if (a >= b) return;
    const uint32_t at = (uint32_t)i;
    if (a >= 0) ranges[a].y = at;
    if (b < (int64_t)n_tiles) ranges[b].x = at;
    for (int64_t t = a + 1; t < b; ++t) ranges[t] = make_uint2(at, at);
}

// The same for four consecutive boundaries per thread: one 16-byte load of the keys and the key
// before them (16-byte aligned key arrays); the last chunk loads key by key below P.
__global__ __launch_bounds__(256) void tile_ranges4_kernel(int64_t P, const uint32_t *P_dev, const uint32_t *tile,
                                                            uint2 *ranges, uint32_t n_tiles) {
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (P_dev && (int64_t)*P_dev < P) P = *P_dev;
    if (i0 > P) return;
    uint32_t k[5];
    k[0] = i0 == 0 ? 0u : tile[i0 - 1];
    if (i0 + 3 < P) {
        const uint4 q = *reinterpret_cast<const uint4 *>(tile + i0);
        k[1] = q.x;
        k[2] = q.y;
        k[3] = q.z;
        k[4] = q.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < P ? tile[i0 + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = i0 + j;
        if (i > P) break;
        const int64_t a = i == 0 ? -1 : (int64_t)min(k[j], n_tiles);
        const int64_t b = i == P ? (int64_t)n_tiles : (int64_t)min(k[j + 1], n_tiles);
        if (a >= b) continue;
        const uint32_t at = (uint32_t)i;
        if (a >= 0) ranges[a].y = at;
        if (b < (int64_t)n_tiles) ranges[b].x = at;
        for (int64_t t = a + 1; t < b; ++t) ranges[t] = make_uint2(at, at);
    }
}

} // namespace

hipError_t launch_emit_pairs(int64_t n, const uint32_t *sorted_ids, const uint32_t *offsets, const float4 *rec,
                             const int32_t *radius, const DevCamera &cam, uint32_t *pair_tile, uint32_t *pair_id,
                             int64_t cap, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    emit_pairs_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, sorted_ids, offsets, rec, radius, cam,
                                                                   pair_tile, pair_id, (uint32_t)cap);
    return hipGetLastError();
}

hipError_t launch_pair_overflow(const uint32_t *total, int64_t cap, uint32_t *overflow, hipStream_t st) {
    pair_overflow_kernel<<<1, 64, 0, st>>>(total, (uint32_t)cap, overflow);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    fill_u32_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(p, value, count);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(int64_t P, const uint32_t *P_dev, const uint32_t *sorted_tile, uint2 *ranges,
                              int64_t n_tiles, hipStream_t st) {
    if (n_tiles <= 0) return hipSuccess;
    if (P < 0) P = 0;
    // Four boundaries per thread from one 16-byte load (a quarter of the threads): the ranges
    // stage of 7.5M pairs at 1080p took 13.6 us against 17.7 us with one boundary per thread.
    if ((reinterpret_cast<uintptr_t>(sorted_tile) & 15) == 0) {
        const int64_t threads = (P + 1 + 3) / 4;
        tile_ranges4_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(P, P_dev, sorted_tile, ranges,
                                                                              (uint32_t)n_tiles);
        return hipGetLastError();
    }
    tile_ranges_kernel<<<(unsigned)((P + 1 + 255) / 256), 256, 0, st>>>(P, P_dev, sorted_tile, ranges,
                                                                      (uint32_t)n_tiles);
    return hipGetLastError();
}

} // namespace gsr

namespace gsr {
namespace {

// out[0] += number of entries with r[i] > 0 (one atomic per block).
__global__ __launch_bounds__(256) void count_positive_kernel(const int32_t *r, int64_t n, uint32_t *out) {
    __shared__ uint32_t s_wave[4];
    uint32_t c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += r[i] > 0 ? 1u : 0u;
    uint32_t total;
    block_exclusive_scan(c, s_wave, total);
    if (threadIdx.x == 0 && total) atomicAdd(out, total);
}

// Compaction of the visible Gaussians (radius > 0) in index order, in three launches over blocks
// of 1024 Gaussians (four per thread, at stride 256): per-block statistics, one block that scans
// the blocks' counts and reduces the rest, and the scatter. Per-block partials rather than
// atomics into one word: same-address atomics from thousands of blocks serialise at one L2
// channel.
constexpr int kVisItems = 4;
constexpr int kVisBlock = 256 * kVisItems;

// part[b] = (visible count, max ~key, max key, sum of tile counts) over block b's visible entries.
__global__ __launch_bounds__(256) void visible_stats_kernel(const int32_t *r, int64_t n, const uint32_t *key,
                                                            const uint32_t *tiles, uint4 *part) {
    __shared__ uint4 s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kVisBlock + threadIdx.x;
    // loads from clamped positions, all issued before any is used (no bounds test around a load)
    int32_t rv[kVisItems];
    uint32_t kv[kVisItems], tv[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
        const int64_t i = base + 256 * j < n ? base + 256 * j : n - 1;
        rv[j] = r[i];
        kv[j] = key[i];
        tv[j] = tiles[i];
    }
    uint32_t c = 0, lo = 0, hi = 0, t = 0;
#pragma unroll
    for (int j = 0; j < kVisItems; ++j)
        if (base + 256 * j < n && rv[j] > 0) {
            c += 1;
            lo = max(lo, ~kv[j]);
            hi = max(hi, kv[j]);
            t += tv[j];
        }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        c += (uint32_t)__shfl_xor((int)c, d, 64);
        t += (uint32_t)__shfl_xor((int)t, d, 64);
        lo = max(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
    }
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = make_uint4(c, lo, hi, t);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 a = s_w[0];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
            const uint4 b = s_w[w];
            a = make_uint4(a.x + b.x, max(a.y, b.y), max(a.z, b.z), a.w + b.w);
        }
        part[blockIdx.x] = a;
    }
}

// One block of 1024 threads: part[b].x becomes the exclusive prefix of the blocks' visible counts;
// totals[0] = sum of tile counts (P), totals[1] = visible count, totals[4] = max ~key,
// totals[5] = max key. Thread t takes four consecutive blocks of each 4096-block chunk.
constexpr int kTotThreads = 1024;
__global__ __launch_bounds__(kTotThreads) void visible_totals_kernel(uint4 *part, int64_t nb, uint32_t *totals) {
    __shared__ uint32_t s_wave[kTotThreads / 64];
    __shared__ uint4 s_red[kTotThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0, lo = 0, hi = 0, t = 0;
    for (int64_t chunk = 0; chunk < nb; chunk += 4 * kTotThreads) {
        const int64_t b0 = chunk + 4 * (int64_t)threadIdx.x;
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = part[b0 + k < nb ? b0 + k : nb - 1];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (b0 + k < nb) {
                sum += v[k].x;
                lo = max(lo, v[k].y);
                hi = max(hi, v[k].z);
                t += v[k].w;
            }
        const uint32_t inc = wave_inclusive_scan(sum, lane);
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kTotThreads / 64; ++w) {
            const uint32_t x = s_wave[w];
            off += (w < wave) ? x : 0u;
            tot += x;
        }
        __syncthreads();
        uint32_t run = carry + off + inc - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (b0 + k < nb) {
                reinterpret_cast<uint32_t *>(part)[4 * (b0 + k)] = run;
                run += v[k].x;
            }
        carry += tot;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        t += (uint32_t)__shfl_xor((int)t, d, 64);
        lo = max(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
    }
    if (lane == 0) s_red[wave] = make_uint4(0u, lo, hi, t);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint4 a = s_red[0];
        for (int w = 1; w < kTotThreads / 64; ++w) {
            const uint4 b = s_red[w];
            a = make_uint4(0u, max(a.y, b.y), max(a.z, b.z), a.w + b.w);
        }
        totals[0] = a.w;
        totals[1] = carry;
        totals[4] = a.y;
        totals[5] = a.z;
    }
}

// Visible entry i of block b goes to the block's offset plus its rank among the block's visible
// entries (index order: item j of every wave before item j + 1, waves in order, lanes in order).
// The offset is part[b].x as scanned by visible_totals_kernel, or with totals != nullptr (few
// blocks, no totals launch) the sum of the earlier blocks' counts, which the block reads itself;
// the last block then also writes the totals.
__global__ __launch_bounds__(256) void compact_visible_kernel(const int32_t *r, int64_t n, const uint32_t *key,
                                                              const uint4 *part, int64_t nb, uint32_t *totals,
                                                              uint32_t *key_out, uint32_t *id_out) {
    __shared__ uint32_t s_cnt[kVisItems][4];
    __shared__ uint4 s_red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kVisBlock + threadIdx.x;
    uint32_t boff;
    if (totals) {
        const bool last_block = (int64_t)blockIdx.x == nb - 1;
        uint32_t before = 0, all = 0, lo = 0, hi = 0, t = 0;
        for (int64_t j = threadIdx.x; j < nb; j += 256) {
            const uint4 q = part[j];
            before += j < (int64_t)blockIdx.x ? q.x : 0u;
            all += q.x;
            lo = max(lo, q.y);
            hi = max(hi, q.z);
            t += q.w;
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            before += (uint32_t)__shfl_xor((int)before, d, 64);
            all += (uint32_t)__shfl_xor((int)all, d, 64);
            lo = max(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
            t += (uint32_t)__shfl_xor((int)t, d, 64);
        }
        if (lane == 0) s_red[wave] = make_uint4(before, lo, hi, t);
        if (lane == 0) s_cnt[0][wave] = all;
        __syncthreads();
        boff = s_red[0].x + s_red[1].x + s_red[2].x + s_red[3].x;
        if (last_block && threadIdx.x == 0) {
            totals[0] = s_red[0].w + s_red[1].w + s_red[2].w + s_red[3].w;
            totals[1] = s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3];
            totals[4] = max(max(s_red[0].y, s_red[1].y), max(s_red[2].y, s_red[3].y));
            totals[5] = max(max(s_red[0].z, s_red[1].z), max(s_red[2].z, s_red[3].z));
        }
        __syncthreads(); // s_cnt is reused below
    } else {
        boff = part[blockIdx.x].x;
    }
    int32_t rv[kVisItems];
    uint32_t kv[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
        const int64_t i = base + 256 * j < n ? base + 256 * j : n - 1;
        rv[j] = r[i];
        kv[j] = key[i];
    }
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    bool vis[kVisItems];
    uint32_t rank[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
        vis[j] = base + 256 * j < n && rv[j] > 0;
        const uint64_t m = __ballot(vis[j]);
        rank[j] = (uint32_t)__popcll(m & below);
        if (lane == 0) s_cnt[j][wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t before = boff;
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (w < wave) before += s_cnt[j][w];
        if (vis[j]) {
            key_out[before + rank[j]] = kv[j];
            id_out[before + rank[j]] = (uint32_t)(base + 256 * j);
        }
#pragma unroll
        for (int w = 0; w < 4; ++w)
            if (w >= wave) before += s_cnt[j][w];
    }
}

} // namespace

size_t visible_partial_count(int64_t n) { return (size_t)((n + kVisBlock - 1) / kVisBlock) + 1; }

hipError_t launch_compact_visible(const int32_t *r, int64_t n, const uint32_t *key, const uint32_t *tiles,
                                  uint4 *part, uint32_t *totals, uint32_t *key_out, uint32_t *id_out,
                                  hipStream_t st) {
    if (n <= 0) {
        hipError_t e = launch_fill_u32(totals, 0u, 2, st);
        return e != hipSuccess ? e : launch_fill_u32(totals + 4, 0u, 2, st);
    }
    const int64_t nb = (n + kVisBlock - 1) / kVisBlock;
    visible_stats_kernel<<<(unsigned)nb, 256, 0, st>>>(r, n, key, tiles, part);
    // Up to 128 blocks every compaction block sums the earlier blocks' counts itself (at most 2 KB
    // of reads) and the totals launch is skipped.
    const bool fused = nb <= 128;
    if (!fused) visible_totals_kernel<<<1, kTotThreads, 0, st>>>(part, nb, totals);
    compact_visible_kernel<<<(unsigned)nb, 256, 0, st>>>(r, n, key, part, nb, fused ? totals : nullptr, key_out,
                                                         id_out);
    return hipGetLastError();
}

hipError_t launch_count_positive(const int32_t *r, int64_t n, uint32_t *out, hipStream_t st) {
    hipError_t e = launch_fill_u32(out, 0u, 1, st);
    if (e != hipSuccess || n <= 0) return e;
    // Few blocks: each adds its count to one address, and same-address atomics serialise.
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    count_positive_kernel<<<(unsigned)blocks, 256, 0, st>>>(r, n, out);
    return hipGetLastError();
}

} // namespace gsr
