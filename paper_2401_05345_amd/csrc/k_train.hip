// Training-step kernels around the render/backward path: the optimiser step
// that follows the gradient computation (step 7 of the paper's training
// pipeline figure), a device-side uniform target image for synthetic
// requests, and the L1 loss value.
#include "gsr_internal.hpp"

namespace gsr {
namespace {

// Adam (Kingma and Ba, 2015) with bias correction; one thread per float4 of
// the flat parameter block, plain tail handled by the first threads. With
// `skip` given, nothing is updated when *skip is non-zero (a step whose
// gradient came from an overflowed capacity-mode render).
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, int64_t count,
                                                   float lr, float b1, float b2, float eps, float c1, float c2,
                                                   const uint32_t *skip) {
    if (skip && *skip) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const auto one = [&](int64_t k) {
        const float gk = g[k];
        const float mk = fmaf(b1, m[k], (1.0f - b1) * gk);
        const float vk = fmaf(b2, v[k], (1.0f - b2) * gk * gk);
        m[k] = mk;
        v[k] = vk;
        p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    };
    const int64_t n4 = count / 4;
    if (i < n4) {
        float4 pk = reinterpret_cast<float4 *>(p)[i];
        const float4 gk = reinterpret_cast<const float4 *>(g)[i];
        float4 mk = reinterpret_cast<float4 *>(m)[i];
        float4 vk = reinterpret_cast<float4 *>(v)[i];
        float *pp = &pk.x, *mm = &mk.x, *vv = &vk.x;
        const float *gg = &gk.x;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            mm[j] = fmaf(b1, mm[j], (1.0f - b1) * gg[j]);
            vv[j] = fmaf(b2, vv[j], (1.0f - b2) * gg[j] * gg[j]);
            pp[j] -= lr * (mm[j] / c1) / (sqrtf(vv[j] / c2) + eps);
        }
        reinterpret_cast<float4 *>(p)[i] = pk;
        reinterpret_cast<float4 *>(m)[i] = mk;
        reinterpret_cast<float4 *>(v)[i] = vk;
    }
    if (i < count - 4 * n4) one(4 * n4 + i);
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output of the
// generator whose state is seed + (index + 1) * golden gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t index) {
    uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void uniform_kernel(float *out, int64_t count, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    // Top 24 bits as a float in [0, 1), exactly representable.
    out[i] = (float)(splitmix64(seed, (uint64_t)i) >> 40) * (1.0f / 16777216.0f);
}

// sum |a - b| over count floats into *out (pre-zeroed), one atomic per block.
__global__ __launch_bounds__(256) void l1_sum_kernel(const float *a, const float *b, int64_t count, float *out) {
    __shared__ float part[4];
    float s = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        s += fabsf(a[i] - b[i]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

} // namespace

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr, float b1, float b2,
                       float eps, int step, hipStream_t st, const uint32_t *skip) {
    if (count <= 0) return hipSuccess;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    const int64_t threads = count / 4 > 3 ? count / 4 : 3;
    adam_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(p, g, m, v, count, lr, b1, b2, eps, c1, c2, skip);
    return hipGetLastError();
}

hipError_t launch_uniform(float *out, int64_t count, uint64_t seed, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    uniform_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(out, count, seed);
    return hipGetLastError();
}

hipError_t launch_l1_sum(const float *a, const float *b, int64_t count, float *out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    // Few blocks: each adds its partial sum to one address (same-address atomics serialise).
    int64_t blocks = (count + 255) / 256;
    if (blocks > 256) blocks = 256;
    l1_sum_kernel<<<(unsigned)blocks, 256, 0, st>>>(a, b, count, out);
    return hipGetLastError();
}

} // namespace gsr
