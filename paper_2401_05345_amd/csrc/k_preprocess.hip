// Per-Gaussian stages of the 3DGS pipeline (one thread per Gaussian, fp32):
//   a1 preprocess_fwd: projection, EWA 2D covariance and conic, 3-sigma radius,
//      tile count, view-dependent SH colour, depth sort key
//   a7 preprocess_bwd: gradients of the raw parameters (means, log-scales,
//      quaternions, opacity logits, SH) from the nine per-Gaussian
//      accumulators of the backward composite
// These are the first and last steps of the paper's rasterisation pipeline
// figure (projection of the primitives; "gradients for all the parameters");
// the math is the published 3D Gaussian Splatting method.
#include <algorithm>

#include "device_common.hpp"

namespace gsr {
namespace {

// Projection quantities of one Gaussian. The forward (a1) takes them in fp32; the chain rule
// (a7) recomputes them in fp64 from the same fp32 parameters: for near-isotropic splats the
// rotation and scale gradients are small differences of large conic terms, and fp32 rounding of
// those terms would move them by ~1e-3.
template <typename T>
struct ProjT {
    T tx, ty, tz;
    T R[9];      // rotation of the normalised quaternion, row-major
    T s[3];      // exp(log-scales)
    T M[9];      // R diag(s)
    T Sig[6];    // Sigma: 00 01 02 11 12 22
    T T2[6];     // J * Rc, rows 0 and 1
    T V0[3], V1[3];
    T a, b, c, det;
    T xc, yc;    // guard-band-clamped x, y used by J
    bool clx, cly;
    T qn[4];     // normalised quaternion
    T qinv;      // 1 / |q|
};
using Proj = ProjT<float>;

// fp64 reciprocal: the hardware estimate refined by one Newton step (relative error ~1e-16).
__device__ __forceinline__ double recip64(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return r * fma(-x, r, 2.0);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float div_t(float a, float b) { return a / b; }
__device__ __forceinline__ double div_t(double a, double b) { return a * recip64(b); }
// exp of a parameter: in fp64 the fp32 value upcast (a relative change of ~1e-7 of a free
// parameter, which moves the derivatives by as little; only the chain's sums need fp64).
__device__ __forceinline__ float exp_t(float x) { return expf(x); }
__device__ __forceinline__ double exp_t(double x) { return (double)expf((float)x); }
// 1/sqrt: in fp64 refined by a Newton step, so the normalised quaternion has unit length to
// ~1e-16 and its rotation matrix is orthogonal to that level.
__device__ __forceinline__ float rsqrt_t(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double rsqrt_t(double x) {
    const double r = (double)(1.0f / sqrtf((float)x));
    return r * fma(-0.5 * x * r, r, 1.5);
}
__device__ __forceinline__ float fmin_t(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double fmin_t(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float fmax_t(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double fmax_t(double a, double b) { return fmax(a, b); }

// Guard band of x/z and y/z: the camera's fp32 bounds, or in fp64 the same formula (the image
// extended by 15 % of its size on each side) evaluated in fp64.
__device__ __forceinline__ void guard_band(const DevCamera &cam, float &lox, float &hix, float &loy, float &hiy) {
    lox = cam.lox, hix = cam.hix, loy = cam.loy, hiy = cam.hiy;
}
__device__ __forceinline__ void guard_band(const DevCamera &cam, double &lox, double &hix, double &loy,
                                           double &hiy) {
    const double w = cam.width, h = cam.height, cx = cam.cx, cy = cam.cy;
    const double ifx = recip64((double)cam.fx), ify = recip64((double)cam.fy);
    lox = (-cx - 0.15 * w) * ifx;
    hix = (w - cx + 0.15 * w) * ifx;
    loy = (-cy - 0.15 * h) * ify;
    hiy = (h - cy + 0.15 * h) * ify;
}

template <typename T>
__device__ __forceinline__ void project_splat(const DevCamera &cam, T mx, T my, T mz, T tz, const float *ls,
                                              const float *q, ProjT<T> &p) {
    p.tz = tz;
    p.tx = fma_t((T)cam.R[0], mx, fma_t((T)cam.R[1], my, fma_t((T)cam.R[2], mz, (T)cam.t[0])));
    p.ty = fma_t((T)cam.R[3], mx, fma_t((T)cam.R[4], my, fma_t((T)cam.R[5], mz, (T)cam.t[1])));

    p.s[0] = exp_t((T)ls[0]);
    p.s[1] = exp_t((T)ls[1]);
    p.s[2] = exp_t((T)ls[2]);
    const T q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
    const T qq = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    p.qinv = rsqrt_t(qq);
    const T w = q0 * p.qinv, x = q1 * p.qinv, y = q2 * p.qinv, z = q3 * p.qinv;
    p.qn[0] = w; p.qn[1] = x; p.qn[2] = y; p.qn[3] = z;
    p.R[0] = T(1) - T(2) * (y * y + z * z); p.R[1] = T(2) * (x * y - w * z);       p.R[2] = T(2) * (x * z + w * y);
    p.R[3] = T(2) * (x * y + w * z);       p.R[4] = T(1) - T(2) * (x * x + z * z); p.R[5] = T(2) * (y * z - w * x);
    p.R[6] = T(2) * (x * z - w * y);       p.R[7] = T(2) * (y * z + w * x);       p.R[8] = T(1) - T(2) * (x * x + y * y);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) p.M[3 * r + k] = p.R[3 * r + k] * p.s[k];
    // Sigma = M M^T
    const T *M = p.M;
    p.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    p.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    p.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    p.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    p.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    p.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];

    // Jacobian of the pinhole map, x/z and y/z held inside the guard band.
    T lox, hix, loy, hiy;
    guard_band(cam, lox, hix, loy, hiy);
    const T txtz = div_t(p.tx, tz), tytz = div_t(p.ty, tz);
    p.clx = txtz < lox || txtz > hix;
    p.cly = tytz < loy || tytz > hiy;
    p.xc = fmin_t(hix, fmax_t(lox, txtz)) * tz;
    p.yc = fmin_t(hiy, fmax_t(loy, tytz)) * tz;
    const T itz = div_t(T(1), tz);
    const T fx = cam.fx, fy = cam.fy;
    const T J00 = fx * itz, J02 = -fx * p.xc * itz * itz;
    const T J11 = fy * itz, J12 = -fy * p.yc * itz * itz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        p.T2[k] = J00 * (T)cam.R[k] + J02 * (T)cam.R[6 + k];
        p.T2[3 + k] = J11 * (T)cam.R[3 + k] + J12 * (T)cam.R[6 + k];
    }
    // V = Sigma T2^T (Sigma symmetric), a = T2_0 . V0, b = T2_0 . V1, c = T2_1 . V1
    const T *S = p.Sig;
    const T *Tm = p.T2;
    p.V0[0] = S[0] * Tm[0] + S[1] * Tm[1] + S[2] * Tm[2];
    p.V0[1] = S[1] * Tm[0] + S[3] * Tm[1] + S[4] * Tm[2];
    p.V0[2] = S[2] * Tm[0] + S[4] * Tm[1] + S[5] * Tm[2];
    p.V1[0] = S[0] * Tm[3] + S[1] * Tm[4] + S[2] * Tm[5];
    p.V1[1] = S[1] * Tm[3] + S[3] * Tm[4] + S[4] * Tm[5];
    p.V1[2] = S[2] * Tm[3] + S[4] * Tm[4] + S[5] * Tm[5];
    p.a = Tm[0] * p.V0[0] + Tm[1] * p.V0[1] + Tm[2] * p.V0[2] + T(0.3);
    p.b = Tm[0] * p.V1[0] + Tm[1] * p.V1[1] + Tm[2] * p.V1[2];
    p.c = Tm[3] * p.V1[0] + Tm[4] * p.V1[1] + Tm[5] * p.V1[2] + T(0.3);
    p.det = fma_t(p.a, p.c, -p.b * p.b);
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
        // A culled Gaussian's record is never read (lists and rows hold visible ones only; the
        // export writes zeros for it), so only its counters are written.
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
    const float go = (float)g[5];
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

    // fp64 geometry (see ProjT): camera-space position, covariance, Jacobian and conic
    using D = double;
    const D tz = fma((D)cam.R[6], (D)mx, fma((D)cam.R[7], (D)my, fma((D)cam.R[8], (D)mz, (D)cam.t[2])));
    ProjT<D> p;
    project_splat<D>(cam, (D)mx, (D)my, (D)mz, tz, log_scales + 3 * i, quats + 4 * i, p);
    D g5[5];
    {
        // dL/d(mean2d, conic) from the moments, with the opacity and the conic in fp64
        const D o = (D)(1.0f / (1.0f + expf(-opacity_logits[i])));
        const D idet = recip64(p.det);
        const D A = p.c * idet, B = -p.b * idet, C = p.a * idet;
        const D m0 = (D)g[0], m1 = (D)g[1];
        g5[0] = o * (A * m0 + B * m1);
        g5[1] = o * (B * m0 + C * m1);
        g5[2] = -0.5 * o * (D)g[2];
        g5[3] = -o * (D)g[3];
        g5[4] = -0.5 * o * (D)g[4];
    }
    const D gu = g5[0], gv = g5[1], gA = g5[2], gB = g5[3], gC = g5[4];

    // ---- conic (A,B,C) = (c, -b, a) / det  ->  2D covariance (a, b, c) ----
    const D a = p.a, b = p.b, c = p.c;
    const D idt = recip64(p.det), id2 = idt * idt;
    const D ga = (-gA * c * c + gB * b * c - gC * b * b) * id2;
    const D gb = (2.0 * gA * b * c - gB * (a * c + b * b) + 2.0 * gC * a * b) * id2;
    const D gc = (-gA * b * b + gB * a * b - gC * a * a) * id2;

    // ---- Sigma2 = T2 Sigma T2^T: dSigma = T2^T G2 T2, dT2 = 2 G2 T2 Sigma, G2 = [[ga, gb/2],[gb/2, gc]] ----
    const D *T = p.T2;
    D dS[6];
    {
        const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int r = rr[e], q = cc[e];
            dS[e] = ga * T[r] * T[q] + 0.5 * gb * (T[r] * T[3 + q] + T[3 + r] * T[q]) + gc * T[3 + r] * T[3 + q];
        }
    }
    D dT0[3], dT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dT0[k] = 2.0 * ga * p.V0[k] + gb * p.V1[k];
        dT1[k] = gb * p.V0[k] + 2.0 * gc * p.V1[k];
    }
    // ---- T2 = J Rc ----
    const D R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2], R3 = cam.R[3], R4 = cam.R[4], R5 = cam.R[5];
    const D R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
    const D dJ00 = dT0[0] * R0 + dT0[1] * R1 + dT0[2] * R2;
    const D dJ02 = dT0[0] * R6 + dT0[1] * R7 + dT0[2] * R8;
    const D dJ11 = dT1[0] * R3 + dT1[1] * R4 + dT1[2] * R5;
    const D dJ12 = dT1[0] * R6 + dT1[1] * R7 + dT1[2] * R8;
    // ---- J(t) and (u,v)(t); a clamped coordinate passes no gradient through x/z ----
    const D itz = recip64(tz), itz2 = itz * itz, itz3 = itz2 * itz;
    const D fx = cam.fx, fy = cam.fy;
    const D dtx = gu * fx * itz + (p.clx ? 0.0 : -fx * itz2 * dJ02);
    const D dty = gv * fy * itz + (p.cly ? 0.0 : -fy * itz2 * dJ12);
    const D dtz = -(gu * fx * p.tx + gv * fy * p.ty) * itz2 - fx * itz2 * dJ00 - fy * itz2 * dJ11 +
                  dJ02 * fx * p.xc * itz3 * (p.clx ? 1.0 : 2.0) +
                  dJ12 * fy * p.yc * itz3 * (p.cly ? 1.0 : 2.0);
    // t = Rc m + tc
    const D Rk[9] = {R0, R1, R2, R3, R4, R5, R6, R7, R8};
#pragma unroll
    for (int k = 0; k < 3; ++k) dm[k] = (float)((D)dm[k] + Rk[k] * dtx + Rk[3 + k] * dty + Rk[6 + k] * dtz);

    // ---- Sigma = M M^T: dM = 2 dSigma M;  M = R diag(s) ----
    const D dSf[9] = {dS[0], dS[1], dS[2], dS[1], dS[3], dS[4], dS[2], dS[4], dS[5]};
    D dM[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            dM[3 * r + q] = 2.0 * (dSf[3 * r] * p.M[q] + dSf[3 * r + 1] * p.M[3 + q] + dSf[3 * r + 2] * p.M[6 + q]);
    D dR[9], dls[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const D ds = dM[q] * p.R[q] + dM[3 + q] * p.R[3 + q] + dM[6 + q] * p.R[6 + q];
        dls[q] = ds * p.s[q];
#pragma unroll
        for (int r = 0; r < 3; ++r) dR[3 * r + q] = dM[3 * r + q] * p.s[q];
    }
    // ---- R(qn) -> qn -> q (through the normalisation) ----
    const D w = p.qn[0], x = p.qn[1], y = p.qn[2], z = p.qn[3];
    D dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const D qd = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    const float op = 1.0f / (1.0f + expf(-opacity_logits[i]));
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = dm[k], o[3 + k] = (float)dls[k];
    o[6] = (float)((dq[0] - qd * w) * p.qinv);
    o[7] = (float)((dq[1] - qd * x) * p.qinv);
    o[8] = (float)((dq[2] - qd * y) * p.qinv);
    o[9] = (float)((dq[3] - qd * z) * p.qinv);
    o[10] = go * op * (1.0f - op);
}

// a7 over blocks of kA7Rows consecutive Gaussians. The block first lists its visible Gaussians
// (radius > 0) in LDS, so that their chain rule runs on dense lanes (a view from inside the
// cloud keeps about a quarter of them); each computed Gaussian leaves 11 gradients, its K basis
// values and its 3 clamped colour gradients in an LDS row. Then the block writes its whole
// segment of every output array, zeros for culled Gaussians included, as consecutive 16-byte
// non-temporal stores (one float per lane and store when unaligned); with accumulate = 1 it adds
// to the visible rows only. Culled Gaussians point at an all-zero LDS row, so every output value
// is read the same way, without a branch per value.
// One wave of 64 rows per block. At 3M Gaussians / 1080p, with one wave per 64 rows, blocks of
// 128 and 256 rows measured 0.214 and 0.220 ms against 0.212 ms; with one wave for 128 or 256
// rows (denser chain-rule lanes, each wave writing more) 0.234 and 0.232 ms against 0.204 ms.
// More, smaller blocks overlap one block's chain rule with other blocks' writes.
constexpr int kA7Threads = 64;
constexpr int kA7Rows = 64;              // Gaussians per block, a multiple of kA7Threads
constexpr int kA7ZeroRow = kA7Rows;      // the all-zero row culled Gaussians read

template <int DEG>
struct A7Layout {
    static constexpr int K = (DEG + 1) * (DEG + 1);
    static constexpr int Y = 11;                // basis values
    static constexpr int G = 11 + K;            // colour gradients g0 g1 g2, then g0 g1 again
    static constexpr int ROW = 11 + K + 5;
    static constexpr int PITCH = ROW | 1;       // odd: rows written by consecutive lanes hit distinct banks
};

enum { A7_ALL = 0, A7_ADD = 1 };

// The block's segment of one [n, W] output (count rows; val(e) is float e of the segment, 0 for
// culled rows). A7_ALL: every float, as consecutive 16-byte non-temporal stores when the output
// is 16-byte aligned (one float per lane and store otherwise). A7_ADD: the visible rows only,
// added to (the culled rows keep their values).
template <int W, typename F>
__device__ __forceinline__ void a7_write(float *__restrict__ dst, int count, bool vec, int mode, const int16_t *slot,
                                         F &&val) {
    // No contraction: a value added to an output is rounded as written before the add, so the
    // accumulating and the overwriting calls agree bit for bit (out + value).
#pragma clang fp contract(off)
    typedef float v4f __attribute__((ext_vector_type(4)));
    const int m = count * W;
    if (mode == A7_ADD) {
        for (int e = threadIdx.x; e < m; e += kA7Threads)
            if (slot[e / W] != kA7ZeroRow) dst[e] += val(e);
        return;
    }
    int e0 = 0;
    if (vec) {
        v4f *d4 = reinterpret_cast<v4f *>(dst);
        const int m4 = m / 4;
        for (int c = threadIdx.x; c < m4; c += kA7Threads) {
            const v4f v = {val(4 * c), val(4 * c + 1), val(4 * c + 2), val(4 * c + 3)};
            __builtin_nontemporal_store(v, d4 + c);
        }
        e0 = m4 * 4;
    }
    for (int e = e0 + threadIdx.x; e < m; e += kA7Threads) dst[e] = val(e);
}

// The SH segment (rows of 3K floats, value 3k + ch = Y[k] g[ch]) as 16-byte non-temporal stores,
// for 3K a multiple of 4, so that each store lies in one row. A store starting at value 4m of
// its row covers k0 = floor(4m / 3) and k0 + 1 and the channels c0, c0 + 1, c0 + 2, c0 (mod 3)
// with c0 = m mod 3; the row's colour gradients stored as g0 g1 g2 g0 g1 give the three
// channels in that order at consecutive addresses.
// m mod 3 and floor(m / 3) for m < 12, as 2-bit fields (field m at bit 2m)
constexpr uint32_t a7_pack_thirds(bool quotient) {
    uint32_t t = 0;
    for (int m = 0; m < 12; ++m) t |= (uint32_t)(quotient ? m / 3 : m % 3) << (2 * m);
    return t;
}
constexpr uint32_t kA7Mod3 = a7_pack_thirds(false), kA7Div3 = a7_pack_thirds(true);

template <int DEG>
__device__ __forceinline__ void a7_write_sh4(float *__restrict__ dst, int count, const int16_t *slot,
                                             const float *s_row) {
    using L = A7Layout<DEG>;
    constexpr int F4 = 3 * L::K / 4; // stores per row
    static_assert(F4 * 4 == 3 * L::K && F4 <= 12, "rows of whole 16-byte stores, m < 12");
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f *d4 = reinterpret_cast<v4f *>(dst);
    const int m4 = count * F4;
    // row q and store m within it, stepped as c advances by kA7Threads
    int q = (int)threadIdx.x / F4, m = (int)threadIdx.x - q * F4;
    for (int c = threadIdx.x; c < m4; c += kA7Threads) {
        const int c0 = (int)((kA7Mod3 >> (2 * m)) & 3u);
        const int k0 = m + (int)((kA7Div3 >> (2 * m)) & 3u); // floor(4m / 3)
        const float *row = s_row + slot[q] * L::PITCH;
        const float ya = row[L::Y + k0], yb = row[L::Y + k0 + 1];
        const float ga = row[L::G + c0], gb = row[L::G + c0 + 1], gc = row[L::G + c0 + 2];
        const v4f v = {ya * ga, (c0 == 2 ? yb : ya) * gb, (c0 >= 1 ? yb : ya) * gc, yb * ga};
        __builtin_nontemporal_store(v, d4 + c);
        q += kA7Threads / F4;
        m += kA7Threads % F4;
        if (m >= F4) {
            m -= F4;
            ++q;
        }
    }
}

template <int DEG, typename AccT>
__global__ __launch_bounds__(kA7Threads) void preprocess_bwd_kernel(int n, const float *__restrict__ means,
                                                                  const float *__restrict__ log_scales,
                                                                  const float *__restrict__ quats,
                                                                  const float *__restrict__ opacity_logits,
                                                                  const float *__restrict__ sh, DevCamera cam,
                                                                  const int32_t *__restrict__ radius,
                                                                  const AccT *__restrict__ acc, gsr_grads out,
                                                                  int mode, int aligned) {
    using L = A7Layout<DEG>;
    constexpr int K = L::K, NS = 3 * K, PITCH = L::PITCH;
    __shared__ float s_row[(kA7Rows + 1) * PITCH];
    __shared__ int16_t s_slot[kA7Rows];   // LDS row of each Gaussian of the block, kA7ZeroRow = culled
    __shared__ int16_t s_list[kA7Rows];   // block-local indices of the visible Gaussians
    const int64_t g0 = (int64_t)blockIdx.x * kA7Rows;
    const int count = (int)min<int64_t>(kA7Rows, (int64_t)n - g0);
    const int lane = threadIdx.x;

    // ---- list the visible Gaussians in index order (ballot ranks, 64 rows at a time) ----
    int nv = 0;
#pragma unroll
    for (int r = 0; r < kA7Rows / kA7Threads; ++r) {
        const int row = r * kA7Threads + lane;
        const bool vis = row < count && radius[g0 + row] > 0;
        const uint64_t mask = __ballot(vis);
        const int rank = nv + __popcll(mask & ((1ull << lane) - 1ull));
        s_slot[row] = vis ? (int16_t)rank : (int16_t)kA7ZeroRow;
        if (vis) s_list[rank] = (int16_t)row;
        nv += __popcll(mask);
    }
    for (int k = lane; k < PITCH; k += kA7Threads) s_row[kA7ZeroRow * PITCH + k] = 0.0f;
    __syncthreads();
    if (mode == A7_ADD && nv == 0) return;

    for (int t = lane; t < nv; t += kA7Threads) {
        // ---- chain rule of the visible ones, on dense lanes ----
        const int64_t i = g0 + s_list[t];
        float o[11], Y[K], g[3];
        gaussian_grads<DEG, AccT>(i, means, log_scales, quats, opacity_logits, sh, cam, acc, o, Y, g);
        float *row = s_row + t * PITCH;
#pragma unroll
        for (int k = 0; k < 11; ++k) row[k] = o[k];
#pragma unroll
        for (int k = 0; k < K; ++k) row[L::Y + k] = Y[k];
#pragma unroll
        for (int c = 0; c < 5; ++c) row[L::G + c] = g[c % 3];
    }
    __syncthreads();

    // ---- the block's segment of each output array, culled rows as zeros ----
    const bool vec = aligned != 0;
    const auto field = [&](int W, int off) {
        return [=](int e) { return s_row[s_slot[e / W] * PITCH + off + e % W]; };
    };
    a7_write<3>(out.means3d + 3 * g0, count, vec, mode, s_slot, field(3, 0));
    a7_write<3>(out.log_scales + 3 * g0, count, vec, mode, s_slot, field(3, 3));
    a7_write<4>(out.quats + 4 * g0, count, vec, mode, s_slot, field(4, 6));
    a7_write<1>(out.opacity_logits + g0, count, vec, mode, s_slot, field(1, 10));
    if constexpr (NS % 4 == 0) {
        if (vec && mode == A7_ALL) {
            a7_write_sh4<DEG>(out.sh + NS * g0, count, s_slot, s_row);
            return;
        }
    }
    a7_write<NS>(out.sh + NS * g0, count, vec, mode, s_slot, [=](int e) {
        const float *row = s_row + s_slot[e / NS] * PITCH;
        const int r = e % NS;
        return row[L::Y + r / 3] * row[L::G + r % 3];
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
    const unsigned blocks = (unsigned)((s.n + kA7Rows - 1) / kA7Rows);
    const auto a16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const int aligned = a16(out.means3d) && a16(out.log_scales) && a16(out.quats) && a16(out.opacity_logits) &&
                        a16(out.sh);
    const int mode = accumulate ? A7_ADD : A7_ALL;
#define GSR_PB(D, A)                                                                                               \
    preprocess_bwd_kernel<D, A><<<blocks, kA7Threads, 0, st>>>(s.n, s.means3d, s.log_scales, s.quats,                \
                                                              s.opacity_logits, s.sh, cam, radius,                 \
                                                              static_cast<const A *>(acc), out, mode, aligned)
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
__global__ __launch_bounds__(256) void zero_listed_rows_kernel(const uint32_t *ids, int64_t m, const uint32_t *m_dev,
                                                                uint4 *acc, int chunks_per_row) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = t / chunks_per_row;
    if (m_dev && (int64_t)*m_dev < m) m = *m_dev; // a count that lives on the device (capacity mode)
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
                                    const uint32_t *n_visible_dev, void *acc, bool acc_f64, hipStream_t st) {
    const int chunks = GSR_ACC_STRIDE * (acc_f64 ? 8 : 4) / 16;
    if (visible_ids) {
        if (n_visible <= 0) return hipSuccess;
        const int64_t threads = n_visible * chunks;
        zero_listed_rows_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(
            visible_ids, n_visible, n_visible_dev, static_cast<uint4 *>(acc), chunks);
        return hipGetLastError();
    }
    if (n <= 0) return hipSuccess;
    zero_visible_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(radius, n, static_cast<uint4 *>(acc), chunks);
    return hipGetLastError();
}

// The projected quantities of every Gaussian out of the 48-byte records (u, v, A, B)
// (C, o, r, g) (b, id, reach, depth), zeros for culled ones (whose records are never
// written). Each output is optional.
__global__ __launch_bounds__(256) void export_rec_kernel(const int32_t *radius, const float4 *rec, int64_t n,
                                                         float *mean2d, float *conic_opacity, float *rgb,
                                                         float *depth) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a;
    if (radius[i] > 0) {
        a = rec[3 * i];
        b = rec[3 * i + 1];
        c = rec[3 * i + 2];
    }
    if (mean2d) {
        mean2d[2 * i] = a.x;
        mean2d[2 * i + 1] = a.y;
    }
    if (conic_opacity) {
        conic_opacity[4 * i] = a.z;
        conic_opacity[4 * i + 1] = a.w;
        conic_opacity[4 * i + 2] = b.x;
        conic_opacity[4 * i + 3] = b.y;
    }
    if (rgb) {
        rgb[3 * i] = b.z;
        rgb[3 * i + 1] = b.w;
        rgb[3 * i + 2] = c.x;
    }
    if (depth) depth[i] = c.w;
}

hipError_t launch_export_rec(const int32_t *radius, const float4 *rec, int64_t n, float *mean2d,
                             float *conic_opacity, float *rgb, float *depth, hipStream_t st) {
    if (n <= 0 || !(mean2d || conic_opacity || rgb || depth)) return hipSuccess;
    export_rec_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(radius, rec, n, mean2d, conic_opacity, rgb, depth);
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
