// Image loss L = (1 - lambda) L1 + lambda (1 - SSIM) and dL/dimage on the
// device (the loss of the 3D Gaussian Splatting training the paper profiles).
// SSIM uses an 11x11 normalised Gaussian window (sigma 1.5) applied as two
// separable zero-padded same-size passes per channel, C1 = 0.01^2,
// C2 = 0.03^2, and is averaged over all 3HW values.
//
// With mu_x = G*x, mu_y = G*y, E_xx = G*x^2, E_yy = G*y^2, E_xy = G*xy and
// S = (A B) / (C D), A = 2 mu_x mu_y + C1, B = 2 (E_xy - mu_x mu_y) + C2,
// C = mu_x^2 + mu_y^2 + C1, D = E_xx + E_yy - mu_x^2 - mu_y^2 + C2:
//   dS/dmu_x = (2 mu_y B - 2 mu_y A) / (C D) - S (2 mu_x / C - 2 mu_x / D)
//   dS/dE_xx = -S / D,   dS/dE_xy = 2 A / (C D)
// and, the zero-padded convolution with a symmetric window being its own
// adjoint, dSum(S)/dx = G*(dS/dmu_x) + 2 x G*(dS/dE_xx) + y G*(dS/dE_xy).
// Stage 1 forms the five blurred maps in LDS (horizontal then vertical pass
// over a tile with a 5-pixel halo), S and the three partial maps; stage 2
// blurs the partial maps the same way and combines them into dL/dimage.
#include "gsr_internal.hpp"

namespace gsr {
namespace {

constexpr int TX = 32, TY = 8, R = 5, WX = TX + 2 * R, WY = TY + 2 * R;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct Window {
    float w[2 * R + 1];
};

__device__ __forceinline__ float load_or_zero(const float *p, int x, int y, int W, int H) {
    return (x >= 0 && x < W && y >= 0 && y < H) ? p[(size_t)y * W + x] : 0.0f;
}

// One block: a TX x TY output tile of one channel (blockIdx.z).
__global__ __launch_bounds__(TX *TY) void ssim_stage1_kernel(const float *__restrict__ img,
                                                             const float *__restrict__ ref, int W, int H, Window g,
                                                             float *__restrict__ dmu, float *__restrict__ dexx,
                                                             float *__restrict__ dexy, float *__restrict__ sums) {
    __shared__ float sx[WY][WX], sy[WY][WX];
    __shared__ float hb[5][WY][TX];
    __shared__ float part[2][TX * TY / 64];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX - R, y0 = blockIdx.y * TY - R;
    const size_t plane = (size_t)W * H;
    const float *X = img + blockIdx.z * plane, *Y = ref + blockIdx.z * plane;
    for (int i = tid; i < WX * WY; i += TX * TY) {
        const int lx = i % WX, ly = i / WX;
        sx[ly][lx] = load_or_zero(X, x0 + lx, y0 + ly, W, H);
        sy[ly][lx] = load_or_zero(Y, x0 + lx, y0 + ly, W, H);
    }
    __syncthreads();
    // horizontal pass: every halo row, TX output columns, five products
    for (int i = tid; i < WY * TX; i += TX * TY) {
        const int lx = i % TX, ly = i / TX;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) {
            const float xv = sx[ly][lx + k], yv = sy[ly][lx + k], w = g.w[k];
            a0 = fmaf(w, xv, a0);
            a1 = fmaf(w, yv, a1);
            a2 = fmaf(w, xv * xv, a2);
            a3 = fmaf(w, yv * yv, a3);
            a4 = fmaf(w, xv * yv, a4);
        }
        hb[0][ly][lx] = a0;
        hb[1][ly][lx] = a1;
        hb[2][ly][lx] = a2;
        hb[3][ly][lx] = a3;
        hb[4][ly][lx] = a4;
    }
    __syncthreads();
    const int lx = tid % TX, ly = tid / TX;
    const int px = blockIdx.x * TX + lx, py = blockIdx.y * TY + ly;
    float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        const float w = g.w[k];
        mx = fmaf(w, hb[0][ly + k][lx], mx);
        my = fmaf(w, hb[1][ly + k][lx], my);
        exx = fmaf(w, hb[2][ly + k][lx], exx);
        eyy = fmaf(w, hb[3][ly + k][lx], eyy);
        exy = fmaf(w, hb[4][ly + k][lx], exy);
    }
    float s = 0.0f, l1 = 0.0f;
    if (px < W && py < H) {
        const float A = 2.0f * mx * my + kC1;
        const float B = 2.0f * (exy - mx * my) + kC2;
        const float C = mx * mx + my * my + kC1;
        const float D = (exx - mx * mx) + (eyy - my * my) + kC2;
        const float CD = C * D;
        s = (A * B) / CD;
        const size_t o = blockIdx.z * plane + (size_t)py * W + px;
        dmu[o] = (2.0f * my * (B - A)) / CD - s * (2.0f * mx / C - 2.0f * mx / D);
        dexx[o] = -s / D;
        dexy[o] = 2.0f * A / CD;
        l1 = fabsf(sx[ly + R][lx + R] - sy[ly + R][lx + R]);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s += __shfl_xor(s, d, 64);
        l1 += __shfl_xor(l1, d, 64);
    }
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = s;
        part[1][tid >> 6] = l1;
    }
    __syncthreads();
    if (tid == 0 && sums) {
        // One partial pair per block (a same-address atomic per block would serialise
        // thousands of adds at one L2 line); ssim_finalize_kernel sums them.
        float a = 0.f, b = 0.f;
        for (int i = 0; i < TX * TY / 64; ++i) {
            a += part[0][i];
            b += part[1][i];
        }
        const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        sums[2 * blk] = a;
        sums[2 * blk + 1] = b;
    }
}

__global__ __launch_bounds__(TX *TY) void ssim_stage2_kernel(const float *__restrict__ img,
                                                             const float *__restrict__ ref, int W, int H, Window g,
                                                             const float *__restrict__ dmu,
                                                             const float *__restrict__ dexx,
                                                             const float *__restrict__ dexy, float l1_scale,
                                                             float ssim_scale, float *__restrict__ out) {
    __shared__ float sm[3][WY][WX];
    __shared__ float hb[3][WY][TX];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX - R, y0 = blockIdx.y * TY - R;
    const size_t plane = (size_t)W * H;
    const size_t base = blockIdx.z * plane;
    for (int i = tid; i < WX * WY; i += TX * TY) {
        const int lx = i % WX, ly = i / WX;
        sm[0][ly][lx] = load_or_zero(dmu + base, x0 + lx, y0 + ly, W, H);
        sm[1][ly][lx] = load_or_zero(dexx + base, x0 + lx, y0 + ly, W, H);
        sm[2][ly][lx] = load_or_zero(dexy + base, x0 + lx, y0 + ly, W, H);
    }
    __syncthreads();
    for (int i = tid; i < WY * TX; i += TX * TY) {
        const int lx = i % TX, ly = i / TX;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) {
            const float w = g.w[k];
            a0 = fmaf(w, sm[0][ly][lx + k], a0);
            a1 = fmaf(w, sm[1][ly][lx + k], a1);
            a2 = fmaf(w, sm[2][ly][lx + k], a2);
        }
        hb[0][ly][lx] = a0;
        hb[1][ly][lx] = a1;
        hb[2][ly][lx] = a2;
    }
    __syncthreads();
    const int lx = tid % TX, ly = tid / TX;
    const int px = blockIdx.x * TX + lx, py = blockIdx.y * TY + ly;
    if (px >= W || py >= H) return;
    float gm = 0.f, gxx = 0.f, gxy = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
        const float w = g.w[k];
        gm = fmaf(w, hb[0][ly + k][lx], gm);
        gxx = fmaf(w, hb[1][ly + k][lx], gxx);
        gxy = fmaf(w, hb[2][ly + k][lx], gxy);
    }
    const size_t o = base + (size_t)py * W + px;
    const float x = img[o], y = ref[o];
    const float d = x - y;
    const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    const float dS = gm + 2.0f * x * gxx + y * gxy;
    out[o] = l1_scale * sgn - ssim_scale * dS;
}

// One block: the loss from the per-block partial sums (SSIM, |x - y|), in fp64.
__global__ __launch_bounds__(256) void ssim_finalize_kernel(const float *sums, int64_t n_blocks, double inv_n,
                                                             float lambda, float *loss) {
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n_blocks; i += 256) {
        a += (double)sums[2 * i];
        b += (double)sums[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss[0] = (float)((1.0 - (double)lambda) * red[1][0] * inv_n + (double)lambda * (1.0 - red[0][0] * inv_n));
}

// dL/dimage of the mean absolute error: sign(image - target) / count (0 where they are equal).
__device__ __forceinline__ float l1_sign(float a, float b, float inv) {
    const float d = a - b;
    return d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
}

__global__ __launch_bounds__(256) void l1_grad_kernel(const float *image, const float *target, int64_t count,
                                                       float inv, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[i] = l1_sign(image[i], target[i], inv);
}

// The same four values per thread as 16-byte loads and stores (16-byte aligned arrays; the
// count's remainder below 4 goes through l1_grad_kernel).
__global__ __launch_bounds__(256) void l1_grad4_kernel(const float4 *image, const float4 *target, int64_t count4,
                                                        float inv, float4 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count4) return;
    const float4 a = image[i], b = target[i];
    out[i] = make_float4(l1_sign(a.x, b.x, inv), l1_sign(a.y, b.y, inv), l1_sign(a.z, b.z, inv),
                         l1_sign(a.w, b.w, inv));
}

} // namespace

hipError_t launch_l1_dssim_grad(const float *img, const float *ref, int C, int W, int H, float lambda, float *dmu,
                                float *dexx, float *dexy, float *sums, float *out, float *loss, hipStream_t st) {
    if (C <= 0 || W <= 0 || H <= 0) return hipSuccess;
    Window g;
    double w[2 * R + 1], tot = 0.0;
    for (int k = 0; k <= 2 * R; ++k) {
        const double x = (double)(k - R);
        w[k] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
        tot += w[k];
    }
    for (int k = 0; k <= 2 * R; ++k) g.w[k] = (float)(w[k] / tot);
    const dim3 grid((W + TX - 1) / TX, (H + TY - 1) / TY, C), block(TX * TY);
    // Per-block partial sums only when the loss value is wanted.
    ssim_stage1_kernel<<<grid, block, 0, st>>>(img, ref, W, H, g, dmu, dexx, dexy, loss ? sums : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double n = (double)C * W * H;
    ssim_stage2_kernel<<<grid, block, 0, st>>>(img, ref, W, H, g, dmu, dexx, dexy, (float)((1.0 - lambda) / n),
                                               (float)(lambda / n), out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (loss) {
        ssim_finalize_kernel<<<1, 256, 0, st>>>(sums, (int64_t)grid.x * grid.y * grid.z, 1.0 / n, lambda, loss);
        e = hipGetLastError();
    }
    return e;
}

size_t dssim_partial_count(int C, int W, int H) {
    return 2 * (size_t)((W + TX - 1) / TX) * ((H + TY - 1) / TY) * (C > 0 ? C : 1);
}

hipError_t launch_l1_grad(const float *image, const float *target, int64_t count, float *out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const float inv = 1.0f / (float)count;
    const auto a16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    int64_t done = 0;
    if (a16(image) && a16(target) && a16(out)) {
        const int64_t count4 = count / 4;
        if (count4 > 0) {
            l1_grad4_kernel<<<(unsigned)((count4 + 255) / 256), 256, 0, st>>>(
                reinterpret_cast<const float4 *>(image), reinterpret_cast<const float4 *>(target), count4, inv,
                reinterpret_cast<float4 *>(out));
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        done = 4 * count4;
    }
    if (done < count)
        l1_grad_kernel<<<(unsigned)((count - done + 255) / 256), 256, 0, st>>>(image + done, target + done,
                                                                           count - done, inv, out + done);
    return hipGetLastError();
}

} // namespace gsr
