// Device helpers shared by the gfx950 kernels of libgsr.
#pragma once

#include "gsr_internal.hpp"

namespace gsr {

constexpr float kAlphaMin = 1.0f / 255.0f; // entries fainter than this are skipped
constexpr float kAlphaMax = 0.99f;         // opacity saturation
constexpr float kTStop = 1e-4f;            // a pixel stops before transmittance drops below this

// Tile rectangle [x0,x1) x [y0,y1) of a splat with mean (u,v) and integer
// radius r: tiles whose pixel span meets [u-r, u+r-1] (resp. v), clamped to
// the grid. Used by the projection (to count tiles) and by the pair emission
// (to enumerate them) on the same stored fp32 inputs, so both agree exactly.
__device__ __forceinline__ void rect_of(float u, float v, int r, const DevCamera &cam, int &x0, int &x1, int &y0,
                                        int &y1) {
    const float ts = (float)cam.tile;
    const float rf = (float)r;
    x0 = min(max((int)floorf((u - rf) / ts), 0), cam.grid_x);
    x1 = min(max((int)floorf((u + rf + ts - 1.0f) / ts), 0), cam.grid_x);
    y0 = min(max((int)floorf((v - rf) / ts), 0), cam.grid_y);
    y1 = min(max((int)floorf((v + rf + ts - 1.0f) / ts), 0), cam.grid_y);
}

// One (pixel, splat) evaluation. The forward composite and the backward
// recompute it with this same function (no FMA contraction inside), so the
// backward takes exactly the forward's skip decisions.
struct SplatEval {
    float dx, dy, power, G, raw, alpha;
    bool pass; // power <= 0 and alpha >= 1/255
};

__device__ __forceinline__ SplatEval eval_splat(float px, float py, float u, float v, float A, float B, float C,
                                                float o) {
#pragma clang fp contract(off)
    SplatEval e;
    e.dx = px - u;
    e.dy = py - v;
    const float q = fmaf(A * e.dx, e.dx, (C * e.dy) * e.dy);
    e.power = fmaf(-B * e.dx, e.dy, -0.5f * q);
    // Hardware exp2 of power*log2(e): relative error ~|power|*2^-24 (3e-7 where alpha meets
    // 1/255), against ~12 instructions for the correctly rounded expf.
    e.G = __expf(e.power);
    e.raw = o * e.G;
    e.alpha = fminf(kAlphaMax, e.raw);
    e.pass = !(e.power > 0.0f) && e.alpha >= kAlphaMin;
    return e;
}

// ---- wavefront (64-lane) helpers ----

// Sum over all 64 lanes, valid in lane 63; every lane must be active.
// In-row (16-lane) butterfly with DPP quad permutes and mirrors, then the
// GFX9 row broadcasts carry row sums upward: 6 DPP-fused adds per value.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, false)); // quad_perm [1,0,3,2]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E, 0xF, 0xF, false)); // quad_perm [2,3,0,1]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x141, 0xF, 0xF, false)); // row_half_mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x140, 0xF, 0xF, false)); // row_mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xA, 0xF, false)); // row_bcast:15
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xC, 0xF, false)); // row_bcast:31
    return v;
}

// Nine values summed over the 64 lanes, the total of value k delivered to the
// lanes whose index within their 16-lane row is k (k < 9), every lane active.
//  1. in-row butterfly, the four DPP steps interleaved across the nine values
//     (independent chains, so no hazard padding between dependent DPP ops);
//  2. transpose: lane k of each row keeps its row's partial of value k;
//  3. the four rows added by two lane permutes (xor 16, xor 32). (The gfx950
//     row-swap builtins were not used: this toolchain returned the first
//     operand for both results of the swap.)
__device__ __forceinline__ float wave_sum9_to_row_lanes(float (&v)[9], int lane) {
#define GSR_DPP_STEP(ctrl)                                                                                           \
    _Pragma("unroll") for (int k = 0; k < 9; ++k) v[k] += __builtin_bit_cast(                                       \
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[k]), ctrl, 0xF, 0xF, false));
    GSR_DPP_STEP(0xB1)  // quad_perm [1,0,3,2]
    GSR_DPP_STEP(0x4E)  // quad_perm [2,3,0,1]
    GSR_DPP_STEP(0x141) // row_half_mirror
    GSR_DPP_STEP(0x140) // row_mirror
#undef GSR_DPP_STEP
    const int r = lane & 15;
    float w = v[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) w = (r == k) ? v[k] : w;
    w += __shfl_xor(w, 16, 64);
    w += __shfl_xor(w, 32, 64);
    return w;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
    return v;
}

// Real spherical harmonics constants, l <= 3 (closed forms: sqrt(1/4pi),
// sqrt(3/4pi), sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4, sqrt(35/2pi)/4,
// sqrt(105/pi)/2, sqrt(21/2pi)/4, sqrt(7/pi)/4, sqrt(105/pi)/4).
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.48860251190291992f;
constexpr float kSH2a = 1.0925484305920792f;
constexpr float kSH2b = 0.31539156525252005f;
constexpr float kSH2c = 0.54627421529603959f;
constexpr float kSH3a = 0.59004358992664352f;
constexpr float kSH3b = 2.8906114426405538f;
constexpr float kSH3c = 0.45704579946446572f;
constexpr float kSH3d = 0.3731763325901154f;
constexpr float kSH3e = 1.4453057213202769f;

// Basis values Y_k(x,y,z) for k < (DEG+1)^2, coefficient order k = l*l + l + m.
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    Y[0] = kSH0;
    if (DEG >= 1) {
        Y[1] = -kSH1 * y;
        Y[2] = kSH1 * z;
        Y[3] = -kSH1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * x * y;
        Y[5] = -kSH2a * y * z;
        Y[6] = kSH2b * (2.0f * zz - xx - yy);
        Y[7] = -kSH2a * x * z;
        Y[8] = kSH2c * (xx - yy);
        if (DEG >= 3) {
            Y[9] = -kSH3a * y * (3.0f * xx - yy);
            Y[10] = kSH3b * x * y * z;
            Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
            Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
            Y[14] = kSH3e * z * (xx - yy);
            Y[15] = -kSH3a * x * (xx - 3.0f * yy);
        }
    }
}

// Gradient of each basis polynomial with respect to (x,y,z), treating the
// components as independent (the caller projects onto the unit sphere).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float *gx, float *gy, float *gz) {
    gx[0] = gy[0] = gz[0] = 0.0f;
    if (DEG >= 1) {
        gx[1] = 0.0f;   gy[1] = -kSH1; gz[1] = 0.0f;
        gx[2] = 0.0f;   gy[2] = 0.0f;  gz[2] = kSH1;
        gx[3] = -kSH1;  gy[3] = 0.0f;  gz[3] = 0.0f;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx[4] = kSH2a * y;          gy[4] = kSH2a * x;          gz[4] = 0.0f;
        gx[5] = 0.0f;               gy[5] = -kSH2a * z;         gz[5] = -kSH2a * y;
        gx[6] = -2.0f * kSH2b * x;  gy[6] = -2.0f * kSH2b * y;  gz[6] = 4.0f * kSH2b * z;
        gx[7] = -kSH2a * z;         gy[7] = 0.0f;               gz[7] = -kSH2a * x;
        gx[8] = 2.0f * kSH2c * x;   gy[8] = -2.0f * kSH2c * y;  gz[8] = 0.0f;
        if (DEG >= 3) {
            gx[9] = -6.0f * kSH3a * x * y;
            gy[9] = -kSH3a * (3.0f * xx - 3.0f * yy);
            gz[9] = 0.0f;
            gx[10] = kSH3b * y * z;
            gy[10] = kSH3b * x * z;
            gz[10] = kSH3b * x * y;
            gx[11] = 2.0f * kSH3c * x * y;
            gy[11] = -kSH3c * (4.0f * zz - xx - 3.0f * yy);
            gz[11] = -8.0f * kSH3c * y * z;
            gx[12] = -6.0f * kSH3d * x * z;
            gy[12] = -6.0f * kSH3d * y * z;
            gz[12] = kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
            gx[13] = -kSH3c * (4.0f * zz - 3.0f * xx - yy);
            gy[13] = 2.0f * kSH3c * x * y;
            gz[13] = -8.0f * kSH3c * x * z;
            gx[14] = 2.0f * kSH3e * x * z;
            gy[14] = -2.0f * kSH3e * y * z;
            gz[14] = kSH3e * (xx - yy);
            gx[15] = -kSH3a * (3.0f * xx - 3.0f * yy);
            gy[15] = 6.0f * kSH3a * x * y;
            gz[15] = 0.0f;
        }
    }
}

} // namespace gsr
