// Entry points of the Top-K feature render (Eq. 3-4, Sec. 3.2) and its adjoint, which
// dispatch to the per-K launches (feature_k*.hip), plus the storage quantizers of the
// feature table, the L1 loss gradient and the Top-K union count.
#include <algorithm>

#include "feature_launch.hpp"
#include "lgs_device.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

// ---------------------------------------------------------------- quantize, L1, union

__global__ __launch_bounds__(256) void quant_bf16_kernel(long n8, const float *__restrict__ src,
                                                         uint16_t *__restrict__ dst) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const f32x4 *s = (const f32x4 *)src + 2 * i;
    f32x4 a = s[0], b = s[1];
    u32x4 o;
    o.x = (uint32_t)f32_to_bf16(a.x) | ((uint32_t)f32_to_bf16(a.y) << 16);
    o.y = (uint32_t)f32_to_bf16(a.z) | ((uint32_t)f32_to_bf16(a.w) << 16);
    o.z = (uint32_t)f32_to_bf16(b.x) | ((uint32_t)f32_to_bf16(b.y) << 16);
    o.w = (uint32_t)f32_to_bf16(b.z) | ((uint32_t)f32_to_bf16(b.w) << 16);
    ((u32x4 *)dst)[i] = o;
}

__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_mov<0xB1>(v));
    v = fmaxf(v, dpp_mov<0x4E>(v));
    v = fmaxf(v, dpp_mov<0x141>(v));
    v = fmaxf(v, dpp_mov<0x140>(v));
    float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// One wave per row: power-of-two scale from the row's largest magnitude, then codes.
// Eight channels per lane and step (two 16-byte loads, one 8-byte store of codes); up
// to kQSteps steps (2048 channels) the row stays in registers between the two passes,
// longer rows are read again.
constexpr int kQSteps = 4;

__device__ __forceinline__ uint32_t e4m3x4(f32x4 v, float inv) {
    return f32_to_e4m3(v.x * inv) | (f32_to_e4m3(v.y * inv) << 8) | (f32_to_e4m3(v.z * inv) << 16) |
           (f32_to_e4m3(v.w * inv) << 24);
}
__device__ __forceinline__ float amax4(f32x4 v, float m) {
    return fmaxf(fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y))), fmaxf(fabsf(v.z), fabsf(v.w)));
}

// Codes and scales of NR rows of D values, by one wave (lane = its lane index): the
// loads of all NR rows are issued before the first row's maximum is taken.  rows[u] < 0
// skips row u (the same for every lane).
template <int NR>
__device__ __forceinline__ void fp8_rows(const float *__restrict__ src, uint8_t *__restrict__ dst,
                                         float *__restrict__ scale, const long (&rows)[NR], int D, int lane) {
    const int steps = (D + 511) >> 9;
    f32x4 v[NR][kQSteps][2];
    float amax[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        amax[u] = 0.f;
        const float *x = src + (rows[u] < 0 ? 0 : rows[u]) * D;
#pragma unroll
        for (int s = 0; s < kQSteps; ++s) {
            const int c = s * 512 + lane * 8;
            v[u][s][0] = v[u][s][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
            if (rows[u] >= 0 && c < D) {
                v[u][s][0] = *(const f32x4 *)(x + c);
                v[u][s][1] = *(const f32x4 *)(x + c + 4);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        if (rows[u] < 0) continue;
        const float *x = src + rows[u] * D;
        uint8_t *y = dst + rows[u] * D;
        float am = 0.f;
#pragma unroll
        for (int s = 0; s < kQSteps; ++s) am = amax4(v[u][s][1], amax4(v[u][s][0], am));
        for (int s = kQSteps; s < steps; ++s) {
            const int c = s * 512 + lane * 8;
            if (c < D) am = amax4(*(const f32x4 *)(x + c + 4), amax4(*(const f32x4 *)(x + c), am));
        }
        am = wave_max(am);
        // s = 2^floor(log2(amax / 224)): with amax = m 2^E (m in [1, 2)) the exponent is
        // E - 7, less one when m < 1.75
        int e = 0;
        if (am > 0.f) {
            uint32_t uu = __float_as_uint(am);
            int E = (int)(uu >> 23) - 127;
            uint32_t mant = uu & 0x7FFFFFu;
            e = E - 7 - (mant < 0x600000u ? 1 : 0);
            if ((uu >> 23) == 0) e = -126;      // subnormal amax
            e = max(e, -126);
        }
        const float sc = __uint_as_float((uint32_t)(127 + e) << 23);
        const float inv = __uint_as_float((uint32_t)(127 - e) << 23);
#pragma unroll
        for (int s = 0; s < kQSteps; ++s) {
            const int c = s * 512 + lane * 8;
            if (c < D) *(u32x2 *)(y + c) = (u32x2){e4m3x4(v[u][s][0], inv), e4m3x4(v[u][s][1], inv)};
        }
        for (int s = kQSteps; s < steps; ++s) {
            const int c = s * 512 + lane * 8;
            if (c < D)
                *(u32x2 *)(y + c) =
                    (u32x2){e4m3x4(*(const f32x4 *)(x + c), inv), e4m3x4(*(const f32x4 *)(x + c + 4), inv)};
        }
        if (lane == 0) scale[rows[u]] = sc;
    }
}

__global__ __launch_bounds__(256) void quant_fp8_kernel(int n, int D, const float *__restrict__ src,
                                                        uint8_t *__restrict__ dst,
                                                        float *__restrict__ scale) {
    const long row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;   // whole wave leaves together
    const long rows[1] = {row};
    fp8_rows<1>(src, dst, scale, rows, D, threadIdx.x & 63);
}

__device__ __forceinline__ uint32_t bf16x2(float a, float b) {
    return (uint32_t)f32_to_bf16(a) | ((uint32_t)f32_to_bf16(b) << 16);
}

// BF16 codes of NR rows of D values by one wave, 8 channels per lane and step; the
// loads of all NR rows of a step are issued before the first conversion.  rows[u] < 0
// skips row u (the same for every lane).
template <int NR>
__device__ __forceinline__ void bf16_rows(const float *__restrict__ src, uint16_t *__restrict__ dst,
                                          const long (&rows)[NR], int D, int lane) {
    for (int c = lane * 8; c < D; c += 512) {
        f32x4 a[NR], b[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            if (rows[u] < 0) continue;
            a[u] = *(const f32x4 *)(src + rows[u] * D + c);
            b[u] = *(const f32x4 *)(src + rows[u] * D + c + 4);
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            if (rows[u] < 0) continue;
            *(u32x4 *)(dst + rows[u] * D + c) =
                (u32x4){bf16x2(a[u].x, a[u].y), bf16x2(a[u].z, a[u].w), bf16x2(b[u].x, b[u].y), bf16x2(b[u].z, b[u].w)};
        }
    }
}

// Quantizes the rows whose row_gen equals gen: each wave takes kMarkRows rows, finds the
// marked ones with a ballot and converts them with the whole wave, NR rows at a time.
// Top-K ids cluster, so a range of rows may be marked throughout: short ranges per wave
// and NR rows per pass (their loads issued together) keep such a wave from waiting one
// load latency per row.
constexpr int kMarkRows = 16;
template <int DT>
__global__ __launch_bounds__(256) void quant_marked_rows_kernel(int n, int D, int gen,
                                                                const int *__restrict__ row_gen,
                                                                const float *__restrict__ src, void *__restrict__ dst,
                                                                float *__restrict__ scale) {
    constexpr int NR = DT == LGS_BF16 ? 8 : 2;
    const int lane = threadIdx.x & 63;
    const long r0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * kMarkRows;
    if (r0 >= n) return;   // whole wave
    const long r = r0 + lane;
    unsigned long long m = __ballot(lane < kMarkRows && r < n && row_gen[r] == gen);
    while (m) {
        long rows[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            rows[u] = -1;
            if (m) {
                rows[u] = r0 + __builtin_ctzll(m);
                m &= m - 1;
            }
        }
        if constexpr (DT == LGS_BF16)
            bf16_rows<NR>(src, (uint16_t *)dst, rows, D, lane);
        else
            fp8_rows<NR>(src, (uint8_t *)dst, scale, rows, D, lane);
    }
}

__device__ __forceinline__ float l1_sign(float d, float g) { return d > 0.f ? g : (d < 0.f ? -g : 0.f); }

// grad = scale * sign(x - target), eight elements per thread with 16-byte accesses;
// the last thread also finishes the n % 8 tail element by element.
template <int DT>
__global__ __launch_bounds__(256) void l1_grad_kernel(long n, const void *__restrict__ x,
                                                      const void *__restrict__ tgt, float scale,
                                                      void *__restrict__ grad) {
    const long n8 = n >> 3;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (DT == MT_F32) {
        if (i < n8) {
            const f32x4 *a = (const f32x4 *)x + 2 * i, *b = (const f32x4 *)tgt + 2 * i;
            f32x4 a0 = a[0], a1 = a[1], b0 = b[0], b1 = b[1];
            f32x4 o0 = {l1_sign(a0.x - b0.x, scale), l1_sign(a0.y - b0.y, scale),
                        l1_sign(a0.z - b0.z, scale), l1_sign(a0.w - b0.w, scale)};
            f32x4 o1 = {l1_sign(a1.x - b1.x, scale), l1_sign(a1.y - b1.y, scale),
                        l1_sign(a1.z - b1.z, scale), l1_sign(a1.w - b1.w, scale)};
            f32x4 *g = (f32x4 *)grad + 2 * i;
            g[0] = o0;
            g[1] = o1;
        }
        if (i == n8)
            for (long j = n8 * 8; j < n; ++j)
                ((float *)grad)[j] = l1_sign(((const float *)x)[j] - ((const float *)tgt)[j], scale);
    } else {
        const float gs = bf16_to_f32(f32_to_bf16(scale));
        const uint32_t pos = f32_to_bf16(gs), neg = f32_to_bf16(-gs);
        auto pick = [&](uint32_t xa, uint32_t xb) -> uint32_t {
            float d = bf16_to_f32(xa) - bf16_to_f32(xb);
            return d > 0.f ? pos : (d < 0.f ? neg : 0u);
        };
        if (i < n8) {
            u32x4 a = ((const u32x4 *)x)[i], b = ((const u32x4 *)tgt)[i];
            u32x4 o;
            o.x = pick(a.x & 0xFFFFu, b.x & 0xFFFFu) | (pick(a.x >> 16, b.x >> 16) << 16);
            o.y = pick(a.y & 0xFFFFu, b.y & 0xFFFFu) | (pick(a.y >> 16, b.y >> 16) << 16);
            o.z = pick(a.z & 0xFFFFu, b.z & 0xFFFFu) | (pick(a.z >> 16, b.z >> 16) << 16);
            o.w = pick(a.w & 0xFFFFu, b.w & 0xFFFFu) | (pick(a.w >> 16, b.w >> 16) << 16);
            ((u32x4 *)grad)[i] = o;
        }
        if (i == n8)
            for (long j = n8 * 8; j < n; ++j)
                ((uint16_t *)grad)[j] = (uint16_t)pick(((const uint16_t *)x)[j], ((const uint16_t *)tgt)[j]);
    }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(long n, int *__restrict__ a) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(256) void union_mark_kernel(long m, const int *__restrict__ ids, int n,
                                                         int *__restrict__ flags) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int g = ids[i];
    if (g >= 0 && g < n) flags[g] = 1;
}

__global__ __launch_bounds__(256) void union_sum_kernel(int n, int *__restrict__ flags) {
    __shared__ int s[256];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    s[threadIdx.x] = i < n ? flags[i] : 0;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && s[0]) atomicAdd(&flags[n], s[0]);
}

// Rows of the feature-gradient table the adjoint can write: row_gen[g] = gen for each
// Gaussian g named in a Top-K slot.
__global__ __launch_bounds__(256) void mark_rows_kernel(long m, const int *__restrict__ ids, int n, int gen,
                                                        int *__restrict__ row_gen) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int g = ids[i];
    if (g >= 0 && g < n) row_gen[g] = gen;
}

// Zeroes the rows whose row_gen equals gen: each wave takes 64 rows, finds the marked
// ones with a ballot and clears each with the whole wave (16-byte stores).
__global__ __launch_bounds__(256) void zero_marked_rows_kernel(int n, int d, int gen, const int *__restrict__ row_gen,
                                                               float *__restrict__ table) {
    const int lane = threadIdx.x & 63;
    const long r0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    if (r0 >= n) return;   // whole wave
    const long r = r0 + lane;
    unsigned long long m = __ballot(r < n && row_gen[r] == gen);
    while (m) {
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        f32x4 *row = (f32x4 *)(table + (r0 + j) * (long)d);
        for (int c = lane; c < d / 4; c += 64) row[c] = (f32x4){0.f, 0.f, 0.f, 0.f};
    }
}

// ---------------------------------------------------------------- dispatch

template <int FT, int MT>
lgs_status fwd_dispatch(int k, int W, int H, int views, int D, const void *feat, const float *scale,
                        const int *ids, const float *tw, void *F, hipStream_t st) {
#define CALL(KK) \
    case KK: return feature_fwd_launch<KK, FT, MT>(W, H, views, D, feat, scale, ids, tw, F, st);
    switch (k) { CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(8) CALL(10) CALL(16) }
#undef CALL
    set_error("K = %d is not compiled", k);
    return LGS_ERR_UNSUPPORTED;
}

template <int FT, int MT, int MODE>
lgs_status bwd_dispatch(int k, int W, int H, int views, int D, const void *feat, const float *scale,
                        const int *ids, const float *tw, const void *dF, float l1_scale, float *dfeat,
                        float *dtw, void *Fo, hipStream_t st) {
#define CALL(KK)                                                                                        \
    case KK:                                                                                            \
        return feature_bwd_launch<KK, FT, MT, MODE>(W, H, views, D, feat, scale, ids, tw, dF, l1_scale, \
                                                    dfeat, dtw, Fo, st);
    switch (k) { CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(8) CALL(10) CALL(16) }
#undef CALL
    set_error("K = %d is not compiled", k);
    return LGS_ERR_UNSUPPORTED;
}

template <int MODE>
lgs_status bwd_entry(int32_t width, int32_t height, int32_t views, int32_t k, int32_t d, lgs_dtype feat_dt,
                     const void *feat, const float *feat_scale, const int32_t *topk_ids, const float *topk_w,
                     lgs_dtype map_dt, const void *dF, float l1_scale, float *dL_dfeat, float *dL_dtopkw,
                     void *Fo, hipStream_t stream) {
#define ARGS k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dF, l1_scale, dL_dfeat, dL_dtopkw, Fo, stream
    if (feat_dt == LGS_F32) return bwd_dispatch<FT_F32, MT_F32, MODE>(ARGS);
    if (feat_dt == LGS_BF16 && map_dt == LGS_BF16) return bwd_dispatch<FT_BF16, MT_BF16, MODE>(ARGS);
    if (feat_dt == LGS_BF16) return bwd_dispatch<FT_BF16, MT_F32, MODE>(ARGS);
    if (map_dt == LGS_BF16) return bwd_dispatch<FT_FP8, MT_BF16, MODE>(ARGS);
    return bwd_dispatch<FT_FP8, MT_F32, MODE>(ARGS);
#undef ARGS
}

lgs_status check_feature_args(int W, int H, int views, int k, int d, lgs_dtype fdt, const void *feat,
                              const float *scale, lgs_dtype mdt) {
    LGS_REQUIRE(W > 0 && H > 0 && views > 0, LGS_ERR_INVALID_ARG, "bad image size %dx%dx%d", W, H, views);
    LGS_REQUIRE(k_supported(k), LGS_ERR_UNSUPPORTED, "K = %d is not compiled", k);
    LGS_REQUIRE(d > 0 && d % 8 == 0, LGS_ERR_UNSUPPORTED, "d = %d must be a positive multiple of 8", d);
    bool ok = (fdt == LGS_F32 && mdt == LGS_F32) || (fdt == LGS_BF16 && (mdt == LGS_BF16 || mdt == LGS_F32)) ||
              (fdt == LGS_FP8_E4M3 && (mdt == LGS_BF16 || mdt == LGS_F32));
    LGS_REQUIRE(ok, LGS_ERR_UNSUPPORTED, "feature/map dtype pair (%d, %d) unsupported", (int)fdt, (int)mdt);
    LGS_REQUIRE(feat, LGS_ERR_INVALID_ARG, "feat is NULL");
    LGS_REQUIRE(aligned16(feat), LGS_ERR_INVALID_ARG, "feat must be 16-byte aligned");
    LGS_REQUIRE(fdt != LGS_FP8_E4M3 || scale, LGS_ERR_INVALID_ARG, "FP8 features need feat_scale");
    return LGS_OK;
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_feature_render_fwd(int32_t width, int32_t height, int32_t views, int32_t k,
                                             int32_t d, lgs_dtype feat_dt, const void *feat,
                                             const float *feat_scale, const int32_t *topk_ids,
                                             const float *topk_w, lgs_dtype map_dt, void *F,
                                             hipStream_t stream) {
    lgs_status st = check_feature_args(width, height, views, k, d, feat_dt, feat, feat_scale, map_dt);
    if (st) return st;
    LGS_REQUIRE(topk_ids && topk_w && F, LGS_ERR_INVALID_ARG, "lgs_feature_render_fwd: NULL pointer");
    LGS_REQUIRE(aligned16(F), LGS_ERR_INVALID_ARG, "F must be 16-byte aligned");
#define ARGS k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, F, stream
    if (feat_dt == LGS_F32) return fwd_dispatch<FT_F32, MT_F32>(ARGS);
    if (feat_dt == LGS_BF16 && map_dt == LGS_BF16) return fwd_dispatch<FT_BF16, MT_BF16>(ARGS);
    if (feat_dt == LGS_BF16) return fwd_dispatch<FT_BF16, MT_F32>(ARGS);
    if (map_dt == LGS_BF16) return fwd_dispatch<FT_FP8, MT_BF16>(ARGS);
    return fwd_dispatch<FT_FP8, MT_F32>(ARGS);
#undef ARGS
}

extern "C" lgs_status lgs_feature_render_bwd(int32_t width, int32_t height, int32_t views, int32_t k,
                                             int32_t d, lgs_dtype feat_dt, const void *feat,
                                             const float *feat_scale, const int32_t *topk_ids,
                                             const float *topk_w, lgs_dtype map_dt, const void *dL_dF,
                                             float *dL_dfeat, float *dL_dtopkw, hipStream_t stream) {
    lgs_status st = check_feature_args(width, height, views, k, d, feat_dt, feat, feat_scale, map_dt);
    if (st) return st;
    LGS_REQUIRE(topk_ids && topk_w && dL_dF && dL_dfeat && dL_dtopkw, LGS_ERR_INVALID_ARG,
                "lgs_feature_render_bwd: NULL pointer");
    LGS_REQUIRE(aligned16(dL_dF), LGS_ERR_INVALID_ARG, "dL_dF must be 16-byte aligned");
    return bwd_entry<0>(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w, map_dt,
                        dL_dF, 0.0f, dL_dfeat, dL_dtopkw, nullptr, stream);
}

extern "C" lgs_status lgs_feature_render_bwd_l1(int32_t width, int32_t height, int32_t views, int32_t k,
                                                int32_t d, lgs_dtype feat_dt, const void *feat,
                                                const float *feat_scale, const int32_t *topk_ids,
                                                const float *topk_w, lgs_dtype map_dt, const void *F_target,
                                                float scale, float *dL_dfeat, float *dL_dtopkw,
                                                hipStream_t stream) {
    lgs_status st = check_feature_args(width, height, views, k, d, feat_dt, feat, feat_scale, map_dt);
    if (st) return st;
    LGS_REQUIRE(topk_ids && topk_w && F_target && dL_dfeat && dL_dtopkw, LGS_ERR_INVALID_ARG,
                "lgs_feature_render_bwd_l1: NULL pointer");
    LGS_REQUIRE(aligned16(F_target), LGS_ERR_INVALID_ARG, "F_target must be 16-byte aligned");
    return bwd_entry<1>(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w, map_dt,
                        F_target, scale, dL_dfeat, dL_dtopkw, nullptr, stream);
}

extern "C" lgs_status lgs_feature_render_fwd_bwd_l1(int32_t width, int32_t height, int32_t views, int32_t k,
                                                    int32_t d, lgs_dtype feat_dt, const void *feat,
                                                    const float *feat_scale, const int32_t *topk_ids,
                                                    const float *topk_w, lgs_dtype map_dt, void *F,
                                                    const void *F_target, float scale, float *dL_dfeat,
                                                    float *dL_dtopkw, hipStream_t stream) {
    lgs_status st = check_feature_args(width, height, views, k, d, feat_dt, feat, feat_scale, map_dt);
    if (st) return st;
    LGS_REQUIRE(topk_ids && topk_w && F && F_target && dL_dfeat && dL_dtopkw, LGS_ERR_INVALID_ARG,
                "lgs_feature_render_fwd_bwd_l1: NULL pointer");
    LGS_REQUIRE(aligned16(F) && aligned16(F_target), LGS_ERR_INVALID_ARG,
                "F and F_target must be 16-byte aligned");
    const size_t map_bytes = (size_t)width * height * views * d * (map_dt == LGS_F32 ? 4 : 2);
    const char *a = (const char *)F, *b = (const char *)F_target;
    LGS_REQUIRE(a + map_bytes <= b || b + map_bytes <= a, LGS_ERR_INVALID_ARG, "F and F_target overlap");
    return bwd_entry<2>(width, height, views, k, d, feat_dt, feat, feat_scale, topk_ids, topk_w, map_dt,
                        F_target, scale, dL_dfeat, dL_dtopkw, F, stream);
}

extern "C" lgs_status lgs_quantize_features(int32_t n, int32_t d, const float *src, lgs_dtype dst_dt,
                                            void *dst, float *dst_scale, hipStream_t stream) {
    LGS_REQUIRE(n >= 0 && d > 0 && d % 8 == 0, LGS_ERR_INVALID_ARG, "bad sizes n=%d d=%d", n, d);
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(src && dst, LGS_ERR_INVALID_ARG, "lgs_quantize_features: NULL pointer");
    LGS_REQUIRE(aligned16(src) && aligned16(dst), LGS_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
    if (dst_dt == LGS_BF16) {
        long n8 = (long)n * d / 8;
        hipLaunchKernelGGL(quant_bf16_kernel, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, stream, n8,
                           src, (uint16_t *)dst);
        return check_launch("quantize bf16");
    }
    LGS_REQUIRE(dst_dt == LGS_FP8_E4M3, LGS_ERR_UNSUPPORTED, "quantize target must be BF16 or FP8");
    LGS_REQUIRE(dst_scale, LGS_ERR_INVALID_ARG, "FP8 quantization needs dst_scale");
    hipLaunchKernelGGL(quant_fp8_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, n, d, src,
                       (uint8_t *)dst, dst_scale);
    return check_launch("quantize fp8");
}

extern "C" lgs_status lgs_l1_grad(int64_t n, lgs_dtype dt, const void *x, const void *target, float scale,
                                  void *grad, hipStream_t stream) {
    LGS_REQUIRE(n >= 0, LGS_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(x && target && grad, LGS_ERR_INVALID_ARG, "lgs_l1_grad: NULL pointer");
    LGS_REQUIRE(aligned16(x) && aligned16(target) && aligned16(grad), LGS_ERR_INVALID_ARG,
                "lgs_l1_grad: arrays must be 16-byte aligned");
    unsigned grid = (unsigned)(((n >> 3) + 1 + 255) / 256);
    if (dt == LGS_F32)
        hipLaunchKernelGGL(l1_grad_kernel<MT_F32>, dim3(grid), dim3(256), 0, stream, (long)n, x, target, scale, grad);
    else if (dt == LGS_BF16)
        hipLaunchKernelGGL(l1_grad_kernel<MT_BF16>, dim3(grid), dim3(256), 0, stream, (long)n, x, target, scale, grad);
    else {
        set_error("lgs_l1_grad: dtype must be F32 or BF16");
        return LGS_ERR_UNSUPPORTED;
    }
    return check_launch("l1_grad");
}

extern "C" lgs_status lgs_union_count(int64_t n_pix, int32_t k, int32_t n, const int32_t *topk_ids,
                                      int32_t *flags, int64_t *count, hipStream_t stream) {
    LGS_REQUIRE(n_pix >= 0 && k > 0 && n >= 0 && count, LGS_ERR_INVALID_ARG, "lgs_union_count: bad args");
    LGS_REQUIRE(flags && (topk_ids || n_pix == 0), LGS_ERR_INVALID_ARG, "lgs_union_count: NULL pointer");
    long m = (long)n_pix * k;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, stream, (long)n + 1, flags);
    if (m > 0)
        hipLaunchKernelGGL(union_mark_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, m, topk_ids, n, flags);
    if (n > 0)
        hipLaunchKernelGGL(union_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, flags);
    lgs_status st = check_launch("union_count");
    if (st) return st;
    int32_t c = 0;
    st = check_hip(hipMemcpyAsync(&c, flags + n, sizeof(c), hipMemcpyDeviceToHost, stream), "union copy");
    if (st) return st;
    st = check_hip(hipStreamSynchronize(stream), "union sync");
    if (st) return st;
    *count = c;
    return LGS_OK;
}

extern "C" lgs_status lgs_mark_topk_rows(int64_t n_slots, const int32_t *topk_ids, int32_t n, int32_t gen,
                                         int32_t *row_gen, hipStream_t stream) {
    LGS_REQUIRE(n_slots >= 0 && n >= 0, LGS_ERR_INVALID_ARG, "lgs_mark_topk_rows: bad sizes");
    if (n_slots == 0 || n == 0) return LGS_OK;
    LGS_REQUIRE(topk_ids && row_gen, LGS_ERR_INVALID_ARG, "lgs_mark_topk_rows: NULL pointer");
    hipLaunchKernelGGL(mark_rows_kernel, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, stream, (long)n_slots,
                       topk_ids, n, gen, row_gen);
    return check_launch("mark_topk_rows");
}

extern "C" lgs_status lgs_zero_marked_rows(int32_t n, int32_t d, int32_t gen, const int32_t *row_gen, float *table,
                                           hipStream_t stream) {
    LGS_REQUIRE(n >= 0 && d > 0 && d % 4 == 0, LGS_ERR_INVALID_ARG, "lgs_zero_marked_rows: bad sizes n=%d d=%d", n,
                d);
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(row_gen && table, LGS_ERR_INVALID_ARG, "lgs_zero_marked_rows: NULL pointer");
    LGS_REQUIRE(aligned16(table), LGS_ERR_INVALID_ARG, "table must be 16-byte aligned");
    const long waves = ((long)n + 63) / 64;
    hipLaunchKernelGGL(zero_marked_rows_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, stream, n, d, gen,
                       row_gen, table);
    return check_launch("zero_marked_rows");
}

extern "C" lgs_status lgs_quantize_marked_rows(int32_t n, int32_t d, int32_t gen, const int32_t *row_gen,
                                               const float *src, lgs_dtype dst_dt, void *dst, float *dst_scale,
                                               hipStream_t stream) {
    LGS_REQUIRE(n >= 0 && d > 0 && d % 8 == 0, LGS_ERR_INVALID_ARG, "lgs_quantize_marked_rows: bad sizes n=%d d=%d",
                n, d);
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(row_gen && src && dst, LGS_ERR_INVALID_ARG, "lgs_quantize_marked_rows: NULL pointer");
    LGS_REQUIRE(aligned16(src) && aligned16(dst), LGS_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
    const unsigned grid = (unsigned)((((long)n + kMarkRows - 1) / kMarkRows + 3) / 4);
    if (dst_dt == LGS_BF16) {
        hipLaunchKernelGGL(quant_marked_rows_kernel<LGS_BF16>, dim3(grid), dim3(256), 0, stream, n, d, gen, row_gen,
                           src, dst, (float *)nullptr);
        return check_launch("quantize marked rows bf16");
    }
    LGS_REQUIRE(dst_dt == LGS_FP8_E4M3, LGS_ERR_UNSUPPORTED, "quantize target must be BF16 or FP8");
    LGS_REQUIRE(dst_scale, LGS_ERR_INVALID_ARG, "FP8 quantization needs dst_scale");
    hipLaunchKernelGGL(quant_marked_rows_kernel<LGS_FP8_E4M3>, dim3(grid), dim3(256), 0, stream, n, d, gen, row_gen,
                       src, dst, dst_scale);
    return check_launch("quantize marked rows fp8");
}
