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

// Records as the composite kernels stage them in LDS: the conic (A, B, C) of
// power = -0.5 (A dx^2 + C dy^2) - B dx dy is prescaled to
// (a, b, c) = -log2(e) (A/2, B, C/2), so that power log2(e) = a dx^2 + b dx dy
// + c dy^2 costs five operations and the Gaussian is one hardware exp2; the
// reach 2 ln(255 o) of the splat is rescaled to the same units
// (log2(255 o)). Everything else is the record as stored.
constexpr float kLog2e = 1.4426950408889634f;
__device__ __forceinline__ void prescale_record(float4 &r0, float4 &r1, float4 &r2) {
    r0.z *= -0.5f * kLog2e;
    r0.w *= -kLog2e;
    r1.x *= -0.5f * kLog2e;
    r2.z *= 0.5f * kLog2e;
}
__device__ __forceinline__ void stage_record(const float4 *__restrict__ rec, uint32_t g, float4 &r0, float4 &r1,
                                             float4 &r2) {
    r0 = rec[3 * (size_t)g];
    r1 = rec[3 * (size_t)g + 1];
    r2 = rec[3 * (size_t)g + 2];
    prescale_record(r0, r1, r2);
}

// One (pixel, splat) evaluation on a staged record. The forward composite and
// the backward recompute it with this same function (no FMA contraction
// inside), so the backward takes exactly the forward's skip decisions.
struct SplatEval {
    float dx, dy, lp, G, raw, alpha; // lp = power log2(e)
    bool pass;                       // power <= 0 and alpha >= 1/255
};

__device__ __forceinline__ SplatEval eval_splat(float px, float py, float u, float v, float a, float b, float c,
                                                float o) {
#pragma clang fp contract(off)
    SplatEval e;
    e.dx = px - u;
    e.dy = py - v;
    const float t = fmaf(a, e.dx, b * e.dy);
    e.lp = fmaf(t, e.dx, (c * e.dy) * e.dy);
    // Hardware exp2: relative error about 1 ulp.
    e.G = __builtin_amdgcn_exp2f(e.lp);
    e.raw = o * e.G;
    e.alpha = fminf(kAlphaMax, e.raw);
    e.pass = !(e.lp > 0.0f) && e.alpha >= kAlphaMin;
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

// Nine values summed over the 64 lanes as a reduce-scatter: each step pairs two
// registers and halves the lanes that carry each of them, so the work shrinks
// with every step instead of repeating a nine-value butterfly at every level.
//  1. lanes l and l^32: the gfx950 lane swap v_permlane32_swap on a register
//     pair (a, b) returns the lower halves of both in one result and the upper
//     halves in the other; their sum holds a's partial in lanes 0..31 and b's
//     in lanes 32..63 (one swap and one add for two values);
//  2. lanes l and l^16 likewise with v_permlane16_swap (rows 0 and 2 keep the
//     first register, rows 1 and 3 the second);
//  3. within each 16-lane row, DPP partners l^8 (row rotate by 8), l^7 (row
//     half mirror), l^2 and l^1; where two registers are paired, each lane
//     keeps the sum of the register its half of the pair carries.
// Value k's total ends in the lanes whose sum9_slot is k; sum9_issues marks one
// lane per value (lanes 0, 8, ..., 56 and lane 4). Every lane must be active.
__device__ __forceinline__ int sum9_slot(int lane) {
    return (lane & 4) ? 8 : ((lane >> 1) & 4) + ((lane >> 3) & 2) + ((lane >> 5) & 1);
}
__device__ __forceinline__ bool sum9_issues(int lane) { return (lane & 3) == 0 && ((lane & 4) == 0 || lane == 4); }

__device__ __forceinline__ float swap32_sum(float a, float b) {
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float swap16_sum(float a, float b) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp_sum(float v) {
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF,
                                                                     false));
}

__device__ __forceinline__ float wave_sum9_scatter(const float (&v)[9], int lane) {
    const float a0 = swap32_sum(v[0], v[1]), a1 = swap32_sum(v[2], v[3]);
    const float a2 = swap32_sum(v[4], v[5]), a3 = swap32_sum(v[6], v[7]);
    const float a4 = swap32_sum(v[8], v[8]);
    const float b0 = swap16_sum(a0, a1), b1 = swap16_sum(a2, a3), b2 = swap16_sum(a4, a4);
    // row rotate by 8 (ctrl 0x128): partner l^8
    const float c0x = dpp_sum<0x128>(b0), c0y = dpp_sum<0x128>(b1);
    const float c0 = (lane & 8) ? c0y : c0x;
    const float c1 = dpp_sum<0x128>(b2);
    // row half mirror (0x141): partner l^7
    const float dx = dpp_sum<0x141>(c0), dy = dpp_sum<0x141>(c1);
    float d = (lane & 4) ? dy : dx;
    d = dpp_sum<0x4E>(d); // quad_perm [2,3,0,1]: l^2
    d = dpp_sum<0xB1>(d); // quad_perm [1,0,3,2]: l^1
    return d;
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
