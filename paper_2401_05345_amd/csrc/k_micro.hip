// Micro-benchmarks of the memory operations the backward is made of, to
// measure the roofs it is held against on this GPU: streaming copies, a
// write-only and a read-only stream (HBM bandwidth), a gather of 48-byte
// records (the composite kernels' record reads, also a reference of known
// bytes for the hardware traffic counters) and no-return atomic adds in the
// access patterns of the plain and the reduced kernels (the atomic rate of
// the L2/fabric). Every
// kernel runs a fixed number of iterations per thread over a power-of-two
// working set; nothing here is on the rendering path.
#include <algorithm>

#include "gsr_internal.hpp"

namespace gsr {
namespace {

constexpr int kBlock = 256;

// Four independent 16-byte loads in flight per thread before their stores.
__global__ __launch_bounds__(kBlock) void copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                      int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const float4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Write-only stream: eight 16-byte non-temporal stores per thread and round, consecutive lanes
// on consecutive chunks (the store pattern of the per-Gaussian gradient writes).
__global__ __launch_bounds__(kBlock) void write_kernel(v4f *__restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const v4f z = {0.f, 0.f, 0.f, 0.f};
    for (; i + 7 * stride < n4; i += 8 * stride) {
#pragma unroll
        for (int k = 0; k < 8; ++k) __builtin_nontemporal_store(z, dst + i + k * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(z, dst + i);
}

// Read-only stream: eight 16-byte loads in flight per thread; the sum is stored only when it
// takes a value the data cannot produce, so the loads stay.
__global__ __launch_bounds__(kBlock) void read_kernel(const v4f *__restrict__ src, int64_t n4, float *sink) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + 7 * stride < n4; i += 8 * stride) {
        v4f x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += x[k];
    }
    for (; i < n4; i += stride) acc += src[i];
    if (acc.x + acc.y + acc.z + acc.w == -1.0f) sink[0] = acc.x;
}

// Copy with eight non-temporal 16-byte loads in flight per thread, then eight non-temporal stores.
__global__ __launch_bounds__(kBlock) void copy_nt_kernel(const v4f *__restrict__ src, v4f *__restrict__ dst,
                                                         int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 7 * stride < n4; i += 8 * stride) {
        v4f x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < 8; ++k) __builtin_nontemporal_store(x[k], dst + i + k * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(src[i], dst + i);
}

// Gather of 48-byte records (the composite kernels' splat records): thread t reads record
// (t * 40503) mod R, a permutation of the R = 2^k records, so every record is read exactly once
// per launch in scattered order; three 16-byte loads per record.
__global__ __launch_bounds__(kBlock) void gather48_kernel(const float4 *__restrict__ rec, uint64_t mask,
                                                          float *sink) {
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t > mask) return;
    const uint64_t r = (t * 40503ull) & mask;
    const float4 a = rec[3 * r], b = rec[3 * r + 1], c = rec[3 * r + 2];
    const float s = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w + c.x + c.y + c.z + c.w;
    if (s == -1.0f) sink[0] = s;
}

// Every lane its own address: lanes of a wave on consecutive elements, the
// grid sweeping the working set (mask + 1 elements) iters times.
template <typename T>
__global__ __launch_bounds__(kBlock) void atomic_distinct_kernel(T *buf, uint64_t mask, int iters) {
    const uint64_t threads = (uint64_t)gridDim.x * kBlock;
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int it = 0; it < iters; ++it) unsafeAtomicAdd(&buf[(t + (uint64_t)it * threads) & mask], (T)1);
}

// One 128-byte slot per wave and iteration (slots = (mask + 1) / 32 floats):
// all 64 lanes add to the slot's first float (the plain kernel's pattern),
// lane 0 alone (one reduced sum per instruction), or lanes 0..8 to the
// slot's first nine doubles (the reduced kernel's nine-lane issue).
enum { SLOT_ALL_LANES = 0, SLOT_ONE_LANE = 1, SLOT_NINE_F64 = 2 };
template <int PATTERN>
__global__ __launch_bounds__(kBlock) void atomic_slot_kernel(float *buf, uint64_t slot_mask, int iters) {
    const int lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / 64);
    const uint64_t w = (uint64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    for (int it = 0; it < iters; ++it) {
        float *slot = buf + 32 * ((w + (uint64_t)it * waves) & slot_mask);
        if (PATTERN == SLOT_ALL_LANES) unsafeAtomicAdd(slot, 1.0f);
        if (PATTERN == SLOT_ONE_LANE && lane == 0) unsafeAtomicAdd(slot, 1.0f);
        if (PATTERN == SLOT_NINE_F64 && lane < 9) unsafeAtomicAdd(reinterpret_cast<double *>(slot) + lane, 1.0);
    }
}

} // namespace

hipError_t launch_microbench(int kind, void *buf, int64_t bytes, int64_t *ops, hipStream_t st) {
    // bytes: power of two >= 1 MiB (checked by the caller)
    const int grid = 256 * 32; // 8192 workgroups, 32 per CU (atomic patterns)
    const int iters = 64;
    // Streams: one round of U chunks per thread, so the workgroups in flight at any time cover one
    // contiguous stretch of memory (a grid-stride loop over a fixed smaller grid spreads the
    // concurrent stores over the whole buffer and measured ~25 % less write bandwidth).
    const auto stream_grid = [&](int64_t n4, int u) {
        return (unsigned)std::max<int64_t>(1, (n4 + (int64_t)kBlock * u - 1) / ((int64_t)kBlock * u));
    };
    const uint64_t threads = (uint64_t)grid * kBlock, waves = threads / 64;
    switch (kind) {
    case GSR_MB_COPY: {
        const int64_t n4 = bytes / 2 / 16;
        copy_kernel<<<stream_grid(n4, 4), kBlock, 0, st>>>(static_cast<const float4 *>(buf),
                                             static_cast<float4 *>(buf) + n4, n4);
        *ops = 2 * n4 * 16; // bytes read + written
        break;
    }
    case GSR_MB_ATOMIC_F32_DISTINCT:
        atomic_distinct_kernel<float><<<grid, kBlock, 0, st>>>(static_cast<float *>(buf), (uint64_t)bytes / 4 - 1,
                                                               iters);
        *ops = (int64_t)(threads * iters);
        break;
    case GSR_MB_ATOMIC_F64_DISTINCT:
        atomic_distinct_kernel<double><<<grid, kBlock, 0, st>>>(static_cast<double *>(buf), (uint64_t)bytes / 8 - 1,
                                                                iters);
        *ops = (int64_t)(threads * iters);
        break;
    case GSR_MB_ATOMIC_F32_SAME_ADDRESS:
        atomic_slot_kernel<SLOT_ALL_LANES><<<grid, kBlock, 0, st>>>(static_cast<float *>(buf),
                                                                    (uint64_t)bytes / 128 - 1, iters);
        *ops = (int64_t)(threads * iters);
        break;
    case GSR_MB_ATOMIC_F32_ONE_LANE:
        atomic_slot_kernel<SLOT_ONE_LANE><<<grid, kBlock, 0, st>>>(static_cast<float *>(buf),
                                                                   (uint64_t)bytes / 128 - 1, iters);
        *ops = (int64_t)(waves * iters);
        break;
    case GSR_MB_ATOMIC_F64_NINE_LANES:
        atomic_slot_kernel<SLOT_NINE_F64><<<grid, kBlock, 0, st>>>(static_cast<float *>(buf),
                                                                   (uint64_t)bytes / 128 - 1, iters);
        *ops = (int64_t)(waves * iters * 9);
        break;
    case GSR_MB_WRITE: {
        const int64_t n4 = bytes / 16;
        write_kernel<<<stream_grid(n4, 8), kBlock, 0, st>>>(static_cast<v4f *>(buf), n4);
        *ops = n4 * 16;
        break;
    }
    case GSR_MB_READ: {
        // the last 16 bytes hold the sink
        const int64_t n4 = bytes / 16 - 1;
        read_kernel<<<stream_grid(n4, 8), kBlock, 0, st>>>(static_cast<const v4f *>(buf), n4,
                                             reinterpret_cast<float *>(static_cast<v4f *>(buf) + n4));
        *ops = n4 * 16;
        break;
    }
    case GSR_MB_COPY_NT: {
        const int64_t n4 = bytes / 2 / 16;
        copy_nt_kernel<<<stream_grid(n4, 8), kBlock, 0, st>>>(static_cast<const v4f *>(buf),
                                                               static_cast<v4f *>(buf) + n4, n4);
        *ops = 2 * n4 * 16;
        break;
    }
    case GSR_MB_GATHER48: {
        // R = the largest power of two with 48 R + 16 <= bytes; the sink follows the records
        uint64_t R = 1;
        while ((R * 2) * 48 + 16 <= (uint64_t)bytes) R *= 2;
        gather48_kernel<<<(unsigned)((R + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            static_cast<const float4 *>(buf), R - 1, reinterpret_cast<float *>(static_cast<uint8_t *>(buf) + 48 * R));
        *ops = (int64_t)(R * 48);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace gsr
