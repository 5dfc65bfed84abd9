// Per-Gaussian stages of the 3DGS pipeline (one thread per Gaussian, fp32):
//   a1 preprocess_fwd: projection, EWA 2D covariance and conic, 3-sigma radius,
//      tile count, view-dependent SH colour, depth sort key
//   a7 preprocess_bwd: gradients of the raw parameters (means, log-scales,
//      quaternions, opacity logits, SH) from the nine per-Gaussian
//      accumulators of the backward composite
// These are the first and last steps of the paper's rasterisation pipeline
// figure (projection of the primitives; "gradients for all the parameters");
// the math is the published 3D Gaussian Splatting method.
#include "device_common.hpp"

namespace gsr {
namespace {

struct Proj {
    float tx, ty, tz;
    float R[9];      // rotation of the normalised quaternion, row-major
    float s[3];      // exp(log-scales)
    float M[9];      // R diag(s)
    float Sig[6];    // Sigma: 00 01 02 11 12 22
    float T2[6];     // J * Rc, rows 0 and 1
    float V0[3], V1[3];
    float a, b, c, det;
    float xc, yc;    // guard-band-clamped x, y used by J
    bool clx, cly;
    float qn[4];     // normalised quaternion
    float qinv;      // 1 / |q|
};

__device__ __forceinline__ void project_splat(const DevCamera &cam, float mx, float my, float mz, float tz,
                                              const float *ls, const float *q, Proj &p) {
    p.tz = tz;
    p.tx = fmaf(cam.R[0], mx, fmaf(cam.R[1], my, fmaf(cam.R[2], mz, cam.t[0])));
    p.ty = fmaf(cam.R[3], mx, fmaf(cam.R[4], my, fmaf(cam.R[5], mz, cam.t[1])));

    p.s[0] = expf(ls[0]);
    p.s[1] = expf(ls[1]);
    p.s[2] = expf(ls[2]);
    const float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    p.qinv = 1.0f / sqrtf(qq);
    const float w = q[0] * p.qinv, x = q[1] * p.qinv, y = q[2] * p.qinv, z = q[3] * p.qinv;
    p.qn[0] = w; p.qn[1] = x; p.qn[2] = y; p.qn[3] = z;
    p.R[0] = 1.f - 2.f * (y * y + z * z); p.R[1] = 2.f * (x * y - w * z);       p.R[2] = 2.f * (x * z + w * y);
    p.R[3] = 2.f * (x * y + w * z);       p.R[4] = 1.f - 2.f * (x * x + z * z); p.R[5] = 2.f * (y * z - w * x);
    p.R[6] = 2.f * (x * z - w * y);       p.R[7] = 2.f * (y * z + w * x);       p.R[8] = 1.f - 2.f * (x * x + y * y);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) p.M[3 * r + k] = p.R[3 * r + k] * p.s[k];
    // Sigma = M M^T
    const float *M = p.M;
    p.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    p.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    p.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    p.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    p.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    p.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];

    // Jacobian of the pinhole map, x/z and y/z held inside the guard band.
    const float txtz = p.tx / tz, tytz = p.ty / tz;
    p.clx = txtz < cam.lox || txtz > cam.hix;
    p.cly = tytz < cam.loy || tytz > cam.hiy;
    p.xc = fminf(cam.hix, fmaxf(cam.lox, txtz)) * tz;
    p.yc = fminf(cam.hiy, fmaxf(cam.loy, tytz)) * tz;
    const float itz = 1.0f / tz;
    const float J00 = cam.fx * itz, J02 = -cam.fx * p.xc * itz * itz;
    const float J11 = cam.fy * itz, J12 = -cam.fy * p.yc * itz * itz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        p.T2[k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
        p.T2[3 + k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
    }
    // V = Sigma T2^T (Sigma symmetric), a = T2_0 . V0, b = T2_0 . V1, c = T2_1 . V1
    const float *S = p.Sig;
    const float *T = p.T2;
    p.V0[0] = S[0] * T[0] + S[1] * T[1] + S[2] * T[2];
    p.V0[1] = S[1] * T[0] + S[3] * T[1] + S[4] * T[2];
    p.V0[2] = S[2] * T[0] + S[4] * T[1] + S[5] * T[2];
    p.V1[0] = S[0] * T[3] + S[1] * T[4] + S[2] * T[5];
    p.V1[1] = S[1] * T[3] + S[3] * T[4] + S[4] * T[5];
    p.V1[2] = S[2] * T[3] + S[4] * T[4] + S[5] * T[5];
    p.a = T[0] * p.V0[0] + T[1] * p.V0[1] + T[2] * p.V0[2] + 0.3f;
    p.b = T[0] * p.V1[0] + T[1] * p.V1[1] + T[2] * p.V1[2];
    p.c = T[3] * p.V1[0] + T[4] * p.V1[1] + T[5] * p.V1[2] + 0.3f;
    p.det = fmaf(p.a, p.c, -p.b * p.b);
}

// Depth key: ((R20*mx + R21*my) + R22*mz) + t2, one correctly rounded fp32
// operation at a time, so the sort order is reproducible bit for bit. The
// operations are written in this scope with contraction off: helper
// intrinsics would be inlined as plain products and sums, which the default
// contraction mode may fuse into FMAs.
// A Gaussian's NS colour coefficients: 16-byte loads when the row is a whole number of them and
// the array is 16-byte aligned (a wave's scalar loads of 192-byte rows would each touch 64
// separate lines), else scalar loads.
template <int NS>
__device__ __forceinline__ void load_coeffs(const float *__restrict__ sh, int64_t i, float (&f)[NS]) {
    const float *p = sh + i * NS;
    if (NS % 4 == 0 && (reinterpret_cast<uintptr_t>(sh) & 15) == 0) {
        const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int c = 0; c < NS / 4; ++c) {
            const float4 x = q[c];
            f[4 * c] = x.x;
            f[4 * c + 1] = x.y;
            f[4 * c + 2] = x.z;
            f[4 * c + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) f[k] = p[k];
    }
}

__device__ __forceinline__ float depth_of(const DevCamera &cam, float mx, float my, float mz) {
#pragma clang fp contract(off)
    const float a = cam.R[6] * mx;
    const float b = cam.R[7] * my;
    const float c = cam.R[8] * mz;
    return ((a + b) + c) + cam.t[2];
}

template <int DEG>
__global__ __launch_bounds__(256) void preprocess_fwd_kernel(int n, const float *__restrict__ means,
                                                             const float *__restrict__ log_scales,
                                                             const float *__restrict__ quats,
                                                             const float *__restrict__ opacity_logits,
                                                             const float *__restrict__ sh, DevCamera cam,
                                                             float4 *__restrict__ rec, int32_t *__restrict__ radius,
                                                             uint32_t *__restrict__ tiles_touched,
                                                             uint32_t *__restrict__ depth_key,
                                                             uint32_t *__restrict__ ids,
                                                             uint8_t *__restrict__ clamp_mask) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    ids[i] = (uint32_t)i;
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const float tz = depth_of(cam, mx, my, mz);
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);

    bool vis = tz > cam.znear;
    Proj p;
    float A = 0.f, B = 0.f, C = 0.f, u = 0.f, v = 0.f;
    int r = 0, ntiles = 0;
    if (vis) {
        project_splat(cam, mx, my, mz, tz, log_scales + 3 * i, quats + 4 * i, p);
        vis = p.det > 0.0f;
    }
    if (vis) {
        const float idet = 1.0f / p.det;
        A = p.c * idet;
        B = -p.b * idet;
        C = p.a * idet;
        u = cam.fx * (p.tx / tz) + cam.cx;
        v = cam.fy * (p.ty / tz) + cam.cy;
        const float mid = 0.5f * (p.a + p.c);
        const float lam1 = mid + sqrtf(fmaxf(0.1f, mid * mid - p.det));
        r = (int)ceilf(3.0f * sqrtf(lam1));
        int x0, x1, y0, y1;
        rect_of(u, v, r, cam, x0, x1, y0, y1);
        ntiles = (x1 - x0) * (y1 - y0);
        vis = ntiles > 0;
    }
    if (!vis) {
        rec[3 * (int64_t)i] = zero;
        rec[3 * (int64_t)i + 1] = zero;
        rec[3 * (int64_t)i + 2] = zero;
        radius[i] = 0;
        tiles_touched[i] = 0;
        depth_key[i] = 0xffffffffu;
        clamp_mask[i] = 0;
        return;
    }
    // View-dependent colour along the direction from the camera centre.
    float dx = mx - cam.centre[0], dy = my - cam.centre[1], dz = mz - cam.centre[2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= il; dy *= il; dz *= il;
    float Y[K];
    sh_basis<DEG>(dx, dy, dz, Y);
    float f[3 * K];
    load_coeffs<3 * K>(sh, i, f);
    float rgb[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        rgb[0] = fmaf(Y[k], f[3 * k + 0], rgb[0]);
        rgb[1] = fmaf(Y[k], f[3 * k + 1], rgb[1]);
        rgb[2] = fmaf(Y[k], f[3 * k + 2], rgb[2]);
    }
    uint8_t cm = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        if (rgb[ch] < 0.0f) {
            cm |= (uint8_t)(1u << ch);
            rgb[ch] = 0.0f;
        }
    }
    const float o = 1.0f / (1.0f + expf(-opacity_logits[i]));
    // Reach of the splat: alpha >= 1/255 needs power >= -ln(255 o), i.e. the
    // ellipse d^T K d <= 2 ln(255 o) (K the conic). Composite kernels use it
    // only to skip entries that no pixel of a wavefront can pass; a splat that
    // can never reach 1/255 gets -1.
    const float tau = logf(255.0f * o);
    const float two_tau = tau > 0.0f ? 2.0f * tau : -1.0f;
    rec[3 * (int64_t)i] = make_float4(u, v, A, B);
    rec[3 * (int64_t)i + 1] = make_float4(C, o, rgb[0], rgb[1]);
    // second slot: the Gaussian's own index (bits), so a list entry's record names its accumulator
    // row (next to the blue channel: the backward composite reads both with one 8-byte load)
    rec[3 * (int64_t)i + 2] = make_float4(rgb[2], __uint_as_float((uint32_t)i), two_tau, tz);
    radius[i] = r;
    tiles_touched[i] = (uint32_t)ntiles;
    depth_key[i] = __float_as_uint(tz);
    clamp_mask[i] = cm;
}

// The backward composite adds, per Gaussian, the five moments of h = dL/do
// (each pixel's G dL/d(oG)) over the pixel offsets (dx, dy) = (px - u, py - v):
//   m = (sum h dx, sum h dy, sum h dx^2, sum h dx dy, sum h dy^2).
// A pixel's dL/dpower is o h. With power = -0.5 (A dx^2 + C dy^2) - B dx dy
// and o, (A, B, C) the same for every pixel, the mean and conic gradients
// follow as
//   dL/du = o (A m0 + B m1), dL/dv = o (B m0 + C m1),
//   dL/dA = -o m2 / 2, dL/dB = -o m3, dL/dC = -o m4 / 2,
// in the accumulators' precision.
template <typename AccT>
__device__ __forceinline__ void moments_to_grads(const AccT *m, float o, float A, float B, float C,
                                                 float (&g)[5]) {
    const AccT w = (AccT)o;
    g[0] = (float)(w * ((AccT)A * m[0] + (AccT)B * m[1]));
    g[1] = (float)(w * ((AccT)B * m[0] + (AccT)C * m[1]));
    g[2] = (float)((AccT)-0.5 * w * m[2]);
    g[3] = (float)(-w * m[3]);
    g[4] = (float)((AccT)-0.5 * w * m[4]);
}

// Gradients of one visible Gaussian (radius > 0): o[0..2] means, o[3..5] log-scales,
// o[6..9] quaternion, o[10] opacity logit; the SH gradient is Y[k] * g[ch] (the basis values
// along the view direction times dL/drgb passed through the colour clamp), which the caller
// expands when it writes the rows.
template <int DEG, typename AccT>
__device__ __forceinline__ void gaussian_grads(int64_t i, const float *__restrict__ means,
                                               const float *__restrict__ log_scales,
                                               const float *__restrict__ quats,
                                               const float *__restrict__ opacity_logits,
                                               const float *__restrict__ sh, const DevCamera &cam,
                                               const AccT *__restrict__ acc, float (&o)[11],
                                               float (&Ysh)[(DEG + 1) * (DEG + 1)], float (&gsh)[3]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const AccT *g = acc + (int64_t)i * GSR_ACC_STRIDE;
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const float tz = depth_of(cam, mx, my, mz);
    Proj p;
    project_splat(cam, mx, my, mz, tz, log_scales + 3 * i, quats + 4 * i, p);
    float g5[5];
    {
        // the opacity and the conic as the forward computed them
        const float o = 1.0f / (1.0f + expf(-opacity_logits[i]));
        const float idet = 1.0f / p.det;
        moments_to_grads(g, o, p.c * idet, -p.b * idet, p.a * idet, g5);
    }
    const float gu = g5[0], gv = g5[1], gA = g5[2], gB = g5[3], gC = g5[4], go = (float)g[5];
    const float grgb[3] = {(float)g[6], (float)g[7], (float)g[8]};

    // ---- colour: rgb = max(sum_k Y_k f_k + 0.5, 0) along d = (m - centre)/|m - centre| ----
    float ex = mx - cam.centre[0], ey = my - cam.centre[1], ez = mz - cam.centre[2];
    const float il = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
    const float dxn = ex * il, dyn = ey * il, dzn = ez * il;
    float Y[K];
    sh_basis<DEG>(dxn, dyn, dzn, Y);
    float f[3 * K];
    load_coeffs<3 * K>(sh, i, f);
    float raw[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        raw[0] = fmaf(Y[k], f[3 * k + 0], raw[0]);
        raw[1] = fmaf(Y[k], f[3 * k + 1], raw[1]);
        raw[2] = fmaf(Y[k], f[3 * k + 2], raw[2]);
    }
    float graw[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) graw[ch] = raw[ch] < 0.0f ? 0.0f : grgb[ch];
    float ddir[3] = {0.f, 0.f, 0.f};
    if (DEG > 0) {
        float gx[K], gy[K], gz[K];
        sh_basis_grad<DEG>(dxn, dyn, dzn, gx, gy, gz);
#pragma unroll
        for (int k = 1; k < K; ++k) {
            const float wk = graw[0] * f[3 * k] + graw[1] * f[3 * k + 1] + graw[2] * f[3 * k + 2];
            ddir[0] = fmaf(wk, gx[k], ddir[0]);
            ddir[1] = fmaf(wk, gy[k], ddir[1]);
            ddir[2] = fmaf(wk, gz[k], ddir[2]);
        }
    }
    // d(dir)/d(m) = (I - dir dir^T) / |m - centre|
    const float proj = ddir[0] * dxn + ddir[1] * dyn + ddir[2] * dzn;
    float dm[3] = {(ddir[0] - proj * dxn) * il, (ddir[1] - proj * dyn) * il, (ddir[2] - proj * dzn) * il};
#pragma unroll
    for (int k = 0; k < K; ++k) Ysh[k] = Y[k];
    gsh[0] = graw[0];
    gsh[1] = graw[1];
    gsh[2] = graw[2];

    // ---- conic (A,B,C) = (c, -b, a) / det  ->  2D covariance (a, b, c) ----
    const float a = p.a, b = p.b, c = p.c;
    const float id2 = 1.0f / (p.det * p.det);
    const float ga = (-gA * c * c + gB * b * c - gC * b * b) * id2;
    const float gb = (2.0f * gA * b * c - gB * (a * c + b * b) + 2.0f * gC * a * b) * id2;
    const float gc = (-gA * b * b + gB * a * b - gC * a * a) * id2;

    // ---- Sigma2 = T2 Sigma T2^T: dSigma = T2^T G2 T2, dT2 = 2 G2 T2 Sigma, G2 = [[ga, gb/2],[gb/2, gc]] ----
    const float *T = p.T2;
    float dS[6];
    {
        const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int r = rr[e], q = cc[e];
            dS[e] = ga * T[r] * T[q] + 0.5f * gb * (T[r] * T[3 + q] + T[3 + r] * T[q]) + gc * T[3 + r] * T[3 + q];
        }
    }
    float dT0[3], dT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dT0[k] = 2.0f * ga * p.V0[k] + gb * p.V1[k];
        dT1[k] = gb * p.V0[k] + 2.0f * gc * p.V1[k];
    }
    // ---- T2 = J Rc ----
    const float dJ00 = dT0[0] * cam.R[0] + dT0[1] * cam.R[1] + dT0[2] * cam.R[2];
    const float dJ02 = dT0[0] * cam.R[6] + dT0[1] * cam.R[7] + dT0[2] * cam.R[8];
    const float dJ11 = dT1[0] * cam.R[3] + dT1[1] * cam.R[4] + dT1[2] * cam.R[5];
    const float dJ12 = dT1[0] * cam.R[6] + dT1[1] * cam.R[7] + dT1[2] * cam.R[8];
    // ---- J(t) and (u,v)(t); a clamped coordinate passes no gradient through x/z ----
    const float itz = 1.0f / tz, itz2 = itz * itz, itz3 = itz2 * itz;
    const float fx = cam.fx, fy = cam.fy;
    const float dtx = gu * fx * itz + (p.clx ? 0.0f : -fx * itz2 * dJ02);
    const float dty = gv * fy * itz + (p.cly ? 0.0f : -fy * itz2 * dJ12);
    const float dtz = -(gu * fx * p.tx + gv * fy * p.ty) * itz2 - fx * itz2 * dJ00 - fy * itz2 * dJ11 +
                      dJ02 * fx * p.xc * itz3 * (p.clx ? 1.0f : 2.0f) +
                      dJ12 * fy * p.yc * itz3 * (p.cly ? 1.0f : 2.0f);
    // t = Rc m + tc
#pragma unroll
    for (int k = 0; k < 3; ++k) dm[k] += cam.R[k] * dtx + cam.R[3 + k] * dty + cam.R[6 + k] * dtz;

    // ---- Sigma = M M^T: dM = 2 dSigma M;  M = R diag(s) ----
    const float dSf[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    float dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            dM[3 * r + q] = 2.0f * (dSf[3 * r] * p.M[q] + dSf[3 * r + 1] * p.M[3 + q] + dSf[3 * r + 2] * p.M[6 + q]);
    float dR[9], dls[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float ds = dM[q] * p.R[q] + dM[3 + q] * p.R[3 + q] + dM[6 + q] * p.R[6 + q];
        dls[q] = ds * p.s[q];
#pragma unroll
        for (int r = 0; r < 3; ++r) dR[3 * r + q] = dM[3 * r + q] * p.s[q];
    }
    // ---- R(qn) -> qn -> q (through the normalisation) ----
    const float w = p.qn[0], x = p.qn[1], y = p.qn[2], z = p.qn[3];
    float dq[4];
    dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.f * x * dR[8]);
    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.f * y * dR[8]);
    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const float qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    const float op = 1.0f / (1.0f + expf(-opacity_logits[i]));
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = dm[k], o[3 + k] = dls[k];
    o[6] = (dq[0] - qd * w) * p.qinv;
    o[7] = (dq[1] - qd * x) * p.qinv;
    o[8] = (dq[2] - qd * y) * p.qinv;
    o[9] = (dq[3] - qd * z) * p.qinv;
    o[10] = go * op * (1.0f - op);
}

// a7 over blocks of 256 consecutive Gaussians. The block first lists its visible Gaussians
// (radius > 0) in LDS, so that their chain rule runs on dense lanes (a view from inside the
// cloud keeps about a quarter of them); each computed Gaussian leaves 11 gradients, its K basis
// values and its 3 clamped colour gradients in an LDS row. Then the block writes its whole
// segment of every output array, zeros for culled Gaussians included, as consecutive 16-byte
// non-temporal stores (when the arrays are 16-byte aligned and the block is full; else one float
// per lane and store). accumulate = 1 adds to the outputs instead.
constexpr int kA7Block = 256;

template <int DEG>
struct A7Layout {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    static constexpr int ROW = 11 + K + 3;     // gradients, basis values, colour gradients
    static constexpr int PITCH = ROW | 1;       // odd: rows written by consecutive lanes hit distinct banks
};

template <int W, typename F>
__device__ __forceinline__ void a7_write(float *__restrict__ dst, int count, bool vec, int accumulate, F &&val) {
    // dst: this block's segment of one [n, W] array; count: Gaussians in the block
    if (vec) {
        typedef float v4f __attribute__((ext_vector_type(4)));
        v4f *d4 = reinterpret_cast<v4f *>(dst);
        constexpr int N4 = kA7Block * W / 4;
        for (int c = threadIdx.x; c < N4; c += kA7Block) {
            v4f v = {val(4 * c), val(4 * c + 1), val(4 * c + 2), val(4 * c + 3)};
            if (accumulate) v += d4[c];
            __builtin_nontemporal_store(v, d4 + c);
        }
    } else {
        for (int e = threadIdx.x; e < count * W; e += kA7Block) {
            const float v = val(e);
            dst[e] = accumulate ? dst[e] + v : v;
        }
    }
}

template <int DEG, typename AccT>
__global__ __launch_bounds__(kA7Block) void preprocess_bwd_kernel(int n, const float *__restrict__ means,
                                                                  const float *__restrict__ log_scales,
                                                                  const float *__restrict__ quats,
                                                                  const float *__restrict__ opacity_logits,
                                                                  const float *__restrict__ sh, DevCamera cam,
                                                                  const int32_t *__restrict__ radius,
                                                                  const AccT *__restrict__ acc, gsr_grads out,
                                                                  int accumulate, int aligned) {
    using L = A7Layout<DEG>;
    constexpr int K = L::K, NS = 3 * K, PITCH = L::PITCH;
    __shared__ float s_row[kA7Block * PITCH];
    __shared__ int16_t s_slot[kA7Block];   // LDS row of each Gaussian of the block, -1 = culled
    __shared__ int16_t s_list[kA7Block];   // block-local indices of the visible Gaussians
    __shared__ int s_wave_count[kA7Block / 64];
    const int64_t g0 = (int64_t)blockIdx.x * kA7Block;
    const int count = (int)min<int64_t>(kA7Block, (int64_t)n - g0);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

    // ---- list the visible Gaussians in index order (ballot ranks within each wave) ----
    const bool vis = t < count && radius[g0 + t] > 0;
    const uint64_t mask = __ballot(vis);
    if (lane == 0) s_wave_count[wave] = __popcll(mask);
    __syncthreads();
    int before = 0, nv = 0;
#pragma unroll
    for (int w = 0; w < kA7Block / 64; ++w) {
        before += w < wave ? s_wave_count[w] : 0;
        nv += s_wave_count[w];
    }
    const int rank = before + __popcll(mask & ((1ull << lane) - 1ull));
    s_slot[t] = vis ? (int16_t)rank : (int16_t)-1;
    if (vis) s_list[rank] = (int16_t)t;
    __syncthreads();

    // ---- chain rule of the visible ones on the first nv lanes ----
    if (t < nv) {
        const int64_t i = g0 + s_list[t];
        float o[11], Y[K], g[3];
        gaussian_grads<DEG, AccT>(i, means, log_scales, quats, opacity_logits, sh, cam, acc, o, Y, g);
        float *row = s_row + t * PITCH;
#pragma unroll
        for (int k = 0; k < 11; ++k) row[k] = o[k];
#pragma unroll
        for (int k = 0; k < K; ++k) row[11 + k] = Y[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) row[11 + K + c] = g[c];
    }
    __syncthreads();

    // ---- the block's segment of each output array, culled rows as zeros ----
    const bool vec = aligned && count == kA7Block;
    const auto field = [&](int W, int off) {
        return [=](int e) {
            const int s = s_slot[e / W];
            return s >= 0 ? s_row[s * PITCH + off + e % W] : 0.0f;
        };
    };
    a7_write<3>(out.means3d + 3 * g0, count, vec, accumulate, field(3, 0));
    a7_write<3>(out.log_scales + 3 * g0, count, vec, accumulate, field(3, 3));
    a7_write<4>(out.quats + 4 * g0, count, vec, accumulate, field(4, 6));
    a7_write<1>(out.opacity_logits + g0, count, vec, accumulate, field(1, 10));
    a7_write<NS>(out.sh + NS * g0, count, vec, accumulate, [=](int e) {
        const int s = s_slot[e / NS];
        const int r = e % NS;
        return s >= 0 ? s_row[s * PITCH + 11 + r / 3] * s_row[s * PITCH + 11 + K + r % 3] : 0.0f;
    });
}

} // namespace

hipError_t launch_preprocess_fwd(const gsr_scene &s, const DevCamera &cam, float4 *rec, int32_t *radius,
                                 uint32_t *tiles_touched, uint32_t *depth_key, uint32_t *ids, uint8_t *clamp_mask,
                                 hipStream_t st) {
    if (s.n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((s.n + 255) / 256);
#define GSR_PF(D)                                                                                                  \
    preprocess_fwd_kernel<D><<<blocks, 256, 0, st>>>(s.n, s.means3d, s.log_scales, s.quats, s.opacity_logits, s.sh, \
                                                      cam, rec, radius, tiles_touched, depth_key, ids, clamp_mask)
    switch (s.sh_degree) {
    case 0: GSR_PF(0); break;
    case 1: GSR_PF(1); break;
    case 2: GSR_PF(2); break;
    default: GSR_PF(3); break;
    }
#undef GSR_PF
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const gsr_scene &s, const DevCamera &cam, const int32_t *radius, const void *acc,
                                 bool acc_f64, const gsr_grads &out, int accumulate, hipStream_t st) {
    if (s.n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((s.n + kA7Block - 1) / kA7Block);
    const auto a16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const int aligned = a16(out.means3d) && a16(out.log_scales) && a16(out.quats) && a16(out.opacity_logits) &&
                        a16(out.sh);
#define GSR_PB(D, A)                                                                                               \
    preprocess_bwd_kernel<D, A><<<blocks, kA7Block, 0, st>>>(s.n, s.means3d, s.log_scales, s.quats,                \
                                                              s.opacity_logits, s.sh, cam, radius,                 \
                                                              static_cast<const A *>(acc), out, accumulate, aligned)
    if (acc_f64) {
        switch (s.sh_degree) {
        case 0: GSR_PB(0, double); break;
        case 1: GSR_PB(1, double); break;
        case 2: GSR_PB(2, double); break;
        default: GSR_PB(3, double); break;
        }
    } else {
        switch (s.sh_degree) {
        case 0: GSR_PB(0, float); break;
        case 1: GSR_PB(1, float); break;
        case 2: GSR_PB(2, float); break;
        default: GSR_PB(3, float); break;
        }
    }
#undef GSR_PB
    return hipGetLastError();
}

namespace {
// Rows of the Gaussians that can appear in a tile list (radius > 0) are the only ones the
// backward composite adds into and a7 reads: only they are cleared.
__global__ __launch_bounds__(256) void zero_visible_rows_kernel(const int32_t *radius, int64_t n, uint4 *acc,
                                                                 int chunks_per_row) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || radius[i] <= 0) return;
    uint4 *row = acc + i * chunks_per_row;
    for (int c = 0; c < chunks_per_row; ++c) row[c] = make_uint4(0u, 0u, 0u, 0u);
}

// The same for a list of the visible Gaussians (the depth-sorted ids of a render): one thread per
// 16-byte chunk of a listed row, so consecutive threads fill whole 128-byte lines, and no thread
// is spent on culled Gaussians.
__global__ __launch_bounds__(256) void zero_listed_rows_kernel(const uint32_t *ids, int64_t m, uint4 *acc,
                                                                int chunks_per_row) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = t / chunks_per_row;
    if (v >= m) return;
    acc[(int64_t)ids[v] * chunks_per_row + (t - v * chunks_per_row)] = make_uint4(0u, 0u, 0u, 0u);
}

// Row i of dst: (dL/du, dL/dv, dL/dA, dL/dB, dL/dC, dL/do, dL/drgb) from the
// accumulated moments and the opacity and conic in the record, as fp32; zeros
// for rows never written (radius <= 0).
template <typename AccT>
__global__ __launch_bounds__(256) void export_acc_kernel(const int32_t *radius, const float4 *rec, int64_t n,
                                                          const AccT *acc, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *o = dst + i * GSR_ACC_STRIDE;
    float row[GSR_ACC_STRIDE];
#pragma unroll
    for (int k = 0; k < GSR_ACC_STRIDE; ++k) row[k] = 0.0f;
    if (radius[i] > 0) {
        const AccT *m = acc + i * GSR_ACC_STRIDE;
        const float4 r0 = rec[3 * i], r1 = rec[3 * i + 1];
        float g5[5];
        moments_to_grads(m, r1.y, r0.z, r0.w, r1.x, g5);
#pragma unroll
        for (int k = 0; k < 5; ++k) row[k] = g5[k];
#pragma unroll
        for (int k = 5; k < 9; ++k) row[k] = (float)m[k];
    }
#pragma unroll
    for (int k = 0; k < GSR_ACC_STRIDE; ++k) o[k] = row[k];
}
} // namespace

hipError_t launch_zero_visible_rows(const int32_t *radius, int64_t n, const uint32_t *visible_ids, int64_t n_visible,
                                    void *acc, bool acc_f64, hipStream_t st) {
    const int chunks = GSR_ACC_STRIDE * (acc_f64 ? 8 : 4) / 16;
    if (visible_ids) {
        if (n_visible <= 0) return hipSuccess;
        const int64_t threads = n_visible * chunks;
        zero_listed_rows_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(
            visible_ids, n_visible, static_cast<uint4 *>(acc), chunks);
        return hipGetLastError();
    }
    if (n <= 0) return hipSuccess;
    zero_visible_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(radius, n, static_cast<uint4 *>(acc), chunks);
    return hipGetLastError();
}

hipError_t launch_export_acc(const int32_t *radius, const float4 *rec, int64_t n, const void *acc, bool acc_f64,
                             float *dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (acc_f64)
        export_acc_kernel<double><<<blocks, 256, 0, st>>>(radius, rec, n, static_cast<const double *>(acc), dst);
    else
        export_acc_kernel<float><<<blocks, 256, 0, st>>>(radius, rec, n, static_cast<const float *>(acc), dst);
    return hipGetLastError();
}

} // namespace gsr
