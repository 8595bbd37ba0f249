// Device-side helpers of the gfx950 renderer: number formats, the per-pixel
// alpha evaluation shared by the forward and backward blend kernels, wave-level
// reductions and the XCD-aware block mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kTile = 16;
constexpr int kTilePix = kTile * kTile;   // 256 pixels = one 256-thread block
constexpr int kWave = 64;

// Constants of the blend (readings of Sec. 3.1, as in the 3DGS rasterizer).
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;

// ------------------------------------------------------------------ formats

// bfloat16 bits from FP32, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// OCP E4M3FN code -> value.  Exponent field e (bias 7), mantissa m: normal codes
// are (1 + m/8) 2^(e-7), built directly as FP32 bits; e = 0 codes are m 2^-9.
__device__ __forceinline__ float e4m3_to_f32(uint32_t c) {
    uint32_t e = (c >> 3) & 15u, m = c & 7u;
    float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;
    return (c & 0x80u) ? -v : v;
}

// FP32 -> E4M3FN code, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint32_t f32_to_e4m3(float y) {
    uint32_t u = __float_as_uint(y);
    uint32_t sign = (u >> 31) << 7;
    float a = fabsf(y);
    if (a != a) return sign | 0x7Fu;
    if (a >= 448.0f) return sign | 0x7Eu;
    if (a < 0.015625f) {                           // below 2^-6: multiples of 2^-9
        return sign | (uint32_t)rintf(a * 512.0f);  // 8 -> code 0x08 = 2^-6
    }
    int E = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;   // a in [2^E, 2^(E+1))
    float t = a * __uint_as_float((uint32_t)(127 + 3 - E) << 23); // a 2^(3-E) in [8, 16)
    uint32_t r = (uint32_t)rintf(t);
    if (r == 16u) { E += 1; r = 8u; }
    uint32_t code = ((uint32_t)(E + 7) << 3) | (r - 8u);
    return sign | (code > 0x7Eu ? 0x7Eu : code);
}

// ------------------------------------------------------------------ blend

// Opacity of a projected Gaussian at a pixel centre: alpha = min(0.99, o e^-sigma).
// The forward and backward blend kernels call this same function, compiled without
// FP contraction, so both take identical skip / stop decisions.  raw_out receives
// o e^-sigma (to tell the clamped case), e_out receives e^-sigma.
__device__ __forceinline__ float blend_alpha(float px, float py, float mx, float my, float ca,
                                             float cb, float cc, float o, float &dx_out,
                                             float &dy_out, float &raw_out, float &e_out) {
    float dx = px - mx;
    float dy = py - my;
    float sigma = fmaf(0.5f * ca, dx * dx, fmaf(0.5f * cc, dy * dy, cb * (dx * dy)));
    sigma = fmaxf(sigma, 0.0f);
    float e = __expf(-sigma);
    float raw = o * e;
    dx_out = dx;
    dy_out = dy;
    raw_out = raw;
    e_out = e;
    return fminf(kAlphaMax, raw);
}

// ------------------------------------------------------------------ waves

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum over all 64 lanes, returned to every lane.  Rows of 16 lanes are reduced
// with DPP moves, the four row sums are read back with readlane.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);    // quad_perm(1,0,3,2): lane ^ 1
    v += dpp_mov<0x4E>(v);    // quad_perm(2,3,0,1): lane ^ 2
    v += dpp_mov<0x141>(v);   // row_half_mirror: 8-lane halves
    v += dpp_mov<0x140>(v);   // row_mirror: 16-lane rows
    float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Sums of N values over all 64 lanes at once (independent DPP chains interleave).
// Rows of 16 are reduced with DPP moves, then row_bcast:15 / row_bcast:31 fold the
// four row sums into lane 63, which is read back.  Every lane must be active.
template <int N>
__device__ __forceinline__ void wave_sum_many(float (&v)[N], float (&out)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0xB1>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x4E>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x141>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x140>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x142, 0xA, 0xF, false));
#pragma unroll
    for (int q = 0; q < N; ++q)
        v[q] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[q]), 0x143, 0xC, 0xF, false));
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[q]), 63));
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// ------------------------------------------------------------------ mapping

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Remap so each XCD walks one contiguous range of work items: neighbouring tiles,
// which share Gaussians and feature rows, then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    int per = (nblocks + 7) >> 3;
    return (b & 7) * per + (b >> 3);
}

}  // namespace lgs
