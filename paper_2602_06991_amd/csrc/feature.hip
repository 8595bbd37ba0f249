// Top-K feature rendering (Eq. 3-4, Sec. 3.2) and its adjoint, the storage
// quantizers of the feature table, the L1 loss gradient and the Top-K union count.
//
// Forward: one wave per pixel; each lane owns 8 consecutive channels and reads the
// K gathered feature rows with 128-bit loads (FP32: two), accumulating in FP32 and
// writing the map row once with non-temporal 128-bit stores.  Since K is fixed,
// every pixel costs the same: the paper's fixed thread allocation (Sec. 3.2).
//
// Backward: one block per 16x16 tile.  The block first builds the union of the
// tile's Top-K ids in an LDS hash table and, for every distinct Gaussian, the list
// of (pixel, slot) entries that selected it.  It then walks the channels in chunks
// of 32: the tile's dL/dF chunk is staged in LDS once, each pixel accumulates its K
// dot products from it, and each distinct Gaussian's gradient row chunk is summed
// in registers over its list and added to global memory with one coalesced atomic
// per channel - U_t atomics per channel per tile instead of 256 K.
#include "lgs_device.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

enum { FT_F32 = 0, FT_BF16 = 1, FT_FP8 = 2 };
enum { MT_F32 = 0, MT_BF16 = 1 };

// Load 8 consecutive feature values of row `row` starting at channel c.
template <int FT>
__device__ __forceinline__ void load8(const void *feat, long row, int D, int c, float (&v)[8]) {
    if constexpr (FT == FT_F32) {
        const f32x4 *p = (const f32x4 *)((const float *)feat + row * D + c);
        f32x4 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else if constexpr (FT == FT_BF16) {
        u32x4 a = *(const u32x4 *)((const uint16_t *)feat + row * D + c);
        v[0] = bf16_to_f32(a.x & 0xFFFFu); v[1] = bf16_to_f32(a.x >> 16);
        v[2] = bf16_to_f32(a.y & 0xFFFFu); v[3] = bf16_to_f32(a.y >> 16);
        v[4] = bf16_to_f32(a.z & 0xFFFFu); v[5] = bf16_to_f32(a.z >> 16);
        v[6] = bf16_to_f32(a.w & 0xFFFFu); v[7] = bf16_to_f32(a.w >> 16);
    } else {
        u32x2 a = *(const u32x2 *)((const uint8_t *)feat + row * D + c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] = e4m3_to_f32((a.x >> (8 * i)) & 0xFFu);
            v[4 + i] = e4m3_to_f32((a.y >> (8 * i)) & 0xFFu);
        }
    }
}

template <int MT>
__device__ __forceinline__ void store8(void *F, long row, int D, int c, const float (&v)[8]) {
    if constexpr (MT == MT_F32) {
        f32x4 *p = (f32x4 *)((float *)F + row * D + c);
        f32x4 a = {v[0], v[1], v[2], v[3]}, b = {v[4], v[5], v[6], v[7]};
        __builtin_nontemporal_store(a, p);
        __builtin_nontemporal_store(b, p + 1);
    } else {
        u32x4 a;
        a.x = (uint32_t)f32_to_bf16(v[0]) | ((uint32_t)f32_to_bf16(v[1]) << 16);
        a.y = (uint32_t)f32_to_bf16(v[2]) | ((uint32_t)f32_to_bf16(v[3]) << 16);
        a.z = (uint32_t)f32_to_bf16(v[4]) | ((uint32_t)f32_to_bf16(v[5]) << 16);
        a.w = (uint32_t)f32_to_bf16(v[6]) | ((uint32_t)f32_to_bf16(v[7]) << 16);
        __builtin_nontemporal_store(a, (u32x4 *)((uint16_t *)F + row * D + c));
    }
}

constexpr int kFwdPixPerBlock = 64;   // 16 pixels per wave, consecutive in memory

template <int K, int FT, int MT>
__global__ __launch_bounds__(256) void feature_fwd_kernel(long n_pix, int D, const void *__restrict__ feat,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ ids,
                                                          const float *__restrict__ tw,
                                                          void *__restrict__ F) {
    const int nblk = (int)((n_pix + kFwdPixPerBlock - 1) / kFwdPixPerBlock);
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (b >= nblk) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int groups = D >> 3;
    const long p0 = (long)b * kFwdPixPerBlock;
    for (int i = wave; i < kFwdPixPerBlock; i += 4) {
        const long p = p0 + i;
        if (p >= n_pix) break;
        int id[K];
        float wk[K];
        float W = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            id[k] = ids[p * K + k];
            wk[k] = tw[p * K + k];
            W += wk[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float wp = (W > 0.f && id[k] >= 0) ? wk[k] / W : 0.f;
            if constexpr (FT == FT_FP8) wp = (id[k] >= 0) ? wp * scale[id[k]] : 0.f;
            wk[k] = wp;
        }
        for (int gi = lane; gi < groups; gi += 64) {
            float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (id[k] < 0) continue;
                float v[8];
                load8<FT>(feat, id[k], D, gi * 8, v);
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = fmaf(wk[k], v[c], acc[c]);
            }
            store8<MT>(F, p, D, gi * 8, acc);
        }
    }
}

// ---------------------------------------------------------------- backward

constexpr int kCh = 32;          // channels per chunk
constexpr int kGStride = kCh + 1;

struct BwdLds {
    // byte offsets into the dynamic LDS buffer
    int region;      // hash keys [HS] (phase 1), then G[256][33] floats
    int region_bytes;
    int uid;         // [256K] distinct Gaussian ids
    int wp;          // [256K] renormalised weights, index t*K + k
    int elist;       // [256K] list entries t*K + k grouped by distinct Gaussian
    int lstart;      // [256K + 1] list starts (counts first)
    int total;
};

__host__ __device__ inline int hash_size(int K) {
    int need = 2 * 256 * K, hs = 1;
    while (hs < need) hs <<= 1;
    return hs;
}

__host__ __device__ inline BwdLds bwd_lds(int K) {
    BwdLds L;
    int hs = hash_size(K);
    int a = hs * 4, b = 256 * kGStride * 4;
    L.region = 0;
    L.region_bytes = a > b ? a : b;
    L.uid = L.region_bytes;
    L.wp = L.uid + 256 * K * 4;
    L.elist = L.wp + 256 * K * 4;
    L.lstart = L.elist + 256 * K * 4;
    L.total = L.lstart + (256 * K + 1) * 4;
    return L;
}

template <int K, int FT, int MT>
__global__ __launch_bounds__(256) void feature_bwd_kernel(int W, int H, int views, int D,
                                                          const void *__restrict__ feat,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ ids,
                                                          const float *__restrict__ tw,
                                                          const void *__restrict__ dF,
                                                          float *__restrict__ dfeat,
                                                          float *__restrict__ dtw) {
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int HS = (2 * 256 * K <= 512) ? 512 : (2 * 256 * K <= 1024) ? 1024 :
                       (2 * 256 * K <= 2048) ? 2048 : (2 * 256 * K <= 4096) ? 4096 : 8192;
    const BwdLds L = bwd_lds(K);
    int *hkey = (int *)(lds + L.region);
    float *G = (float *)(lds + L.region);
    int *uid = (int *)(lds + L.uid);
    float *wps = (float *)(lds + L.wp);
    int *elist = (int *)(lds + L.elist);
    int *lstart = (int *)(lds + L.lstart);
    __shared__ int s_scan[256];

    const int ntx = (W + kTile - 1) / kTile, nty = (H + kTile - 1) / kTile;
    const int ntiles = ntx * nty * views;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int view = tile / (ntx * nty);
    const int tv = tile - view * ntx * nty;
    const int t = threadIdx.x;
    const int px = (tv % ntx) * kTile + (t & 15);
    const int py = (tv / ntx) * kTile + (t >> 4);
    const bool inside = px < W && py < H;
    const long p = (long)view * W * H + (long)py * W + px;

    // phase 0: this pixel's slots
    int id[K];
    float wv[K];
    float Wsum = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        id[k] = inside ? ids[p * K + k] : -1;
        wv[k] = inside ? tw[p * K + k] : 0.f;
        Wsum += wv[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float wp = (Wsum > 0.f && id[k] >= 0) ? wv[k] / Wsum : 0.f;
        if (!(Wsum > 0.f)) id[k] = -1;
        wps[t * K + k] = wp;
    }

    // phase 1: union of ids through an LDS hash table (linear probing)
    for (int h = t; h < HS; h += 256) hkey[h] = -1;
    __syncthreads();
    int slot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        slot[k] = -1;
        if (id[k] < 0) continue;
        uint32_t h = ((uint32_t)id[k] * 2654435761u) & (HS - 1);
        while (true) {
            int prev = atomicCAS(&hkey[h], -1, id[k]);
            if (prev == -1 || prev == id[k]) break;
            h = (h + 1) & (HS - 1);
        }
        slot[k] = (int)h;
    }
    __syncthreads();
    // dense index of every occupied slot, in slot order
    constexpr int per = HS / 256;
    int occ = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) occ += hkey[t * per + j] >= 0;
    s_scan[t] = occ;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int x = t >= off ? s_scan[t - off] : 0;
        __syncthreads();
        s_scan[t] += x;
        __syncthreads();
    }
    const int U = s_scan[255];
    int u = s_scan[t] - occ;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        int h = t * per + j;
        int key = hkey[h];
        if (key >= 0) {
            uid[u] = key;
            hkey[h] = u;    // the slot now maps to its dense index
            ++u;
        }
    }
    for (int i = t; i <= U; i += 256) lstart[i] = 0;
    __syncthreads();
    int uk[K];
    int pos[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uk[k] = slot[k] >= 0 ? hkey[slot[k]] : -1;
        pos[k] = uk[k] >= 0 ? atomicAdd(&lstart[uk[k]], 1) : 0;
    }
    __syncthreads();
    // exclusive scan of the list lengths (U <= 256 K entries)
    {
        const int chunk = (U + 255) / 256;
        int s = 0;
        for (int j = 0; j < chunk; ++j) {
            int i = t * chunk + j;
            if (i < U) s += lstart[i];
        }
        s_scan[t] = s;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int x = t >= off ? s_scan[t - off] : 0;
            __syncthreads();
            s_scan[t] += x;
            __syncthreads();
        }
        int run = s_scan[t] - s;
        for (int j = 0; j < chunk; ++j) {
            int i = t * chunk + j;
            if (i < U) {
                int c = lstart[i];
                lstart[i] = run;
                run += c;
            }
        }
        if (t == 255) lstart[U] = s_scan[255];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (uk[k] >= 0) elist[lstart[uk[k]] + pos[k]] = t * K + k;
    __syncthreads();

    // phase 2: channel chunks
    float dot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dot[k] = 0.f;
    const int wave = t >> 6, lane = t & 63;
    const int worker = wave * 2 + (lane >> 5);   // 8 half-wave row workers
    const int cl = lane & 31;
    const int tile_x0 = (tv % ntx) * kTile, tile_y0 = (tv / ntx) * kTile;
    for (int c0 = 0; c0 < D; c0 += kCh) {
        const int cw = min(kCh, D - c0);      // a multiple of 8
        // stage dL/dF[256 pixels][cw] as FP32
        for (int q = t; q < 256 * (kCh / 8); q += 256) {
            int pix = q >> 2, part = q & 3;   // 4 groups of 8 channels per pixel
            int c = part * 8;
            int lx = tile_x0 + (pix & 15), ly = tile_y0 + (pix >> 4);
            float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (c < cw && lx < W && ly < H) {
                long pp = (long)view * W * H + (long)ly * W + lx;
                if constexpr (MT == MT_F32) load8<FT_F32>(dF, pp, D, c0 + c, v);
                else load8<FT_BF16>(dF, pp, D, c0 + c, v);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) G[pix * kGStride + c + i] = v[i];
        }
        __syncthreads();
        // dot products of this pixel's dL/dF chunk with its K feature rows
        if (Wsum > 0.f) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (id[k] < 0) continue;
                float s = 0.f;
                for (int c = 0; c < cw; c += 8) {
                    float v[8];
                    load8<FT>(feat, id[k], D, c0 + c, v);
#pragma unroll
                    for (int i = 0; i < 8; ++i) s = fmaf(v[i], G[t * kGStride + c + i], s);
                }
                if constexpr (FT == FT_FP8) s *= scale[id[k]];
                dot[k] += s;
            }
        }
        // gradient rows: each half-wave sums one distinct Gaussian's entries
        for (int uu = worker; uu < U; uu += 8) {
            float acc = 0.f;
            const int e1 = lstart[uu + 1];
            for (int e = lstart[uu]; e < e1; ++e) {
                int ent = elist[e];
                int tp = ent / K;
                acc = fmaf(wps[ent], G[tp * kGStride + cl], acc);
            }
            if (cl < cw) unsafeAtomicAdd(&dfeat[(long)uid[uu] * D + c0 + cl], acc);
        }
        __syncthreads();
    }
    // phase 3: gamma_k = (g_k - sum_j w'_j g_j) / W
    if (!inside) return;
    float mean = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) mean = fmaf(wps[t * K + k], dot[k], mean);
#pragma unroll
    for (int k = 0; k < K; ++k)
        dtw[p * K + k] = (Wsum > 0.f && id[k] >= 0) ? (dot[k] - mean) / Wsum : 0.f;
}

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
__global__ __launch_bounds__(256) void quant_fp8_kernel(int n, int D, const float *__restrict__ src,
                                                        uint8_t *__restrict__ dst,
                                                        float *__restrict__ scale) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;   // whole wave leaves together
    const float *x = src + (long)row * D;
    float amax = 0.f;
    for (int c = lane; c < D; c += 64) amax = fmaxf(amax, fabsf(x[c]));
    amax = wave_max(amax);
    // s = 2^floor(log2(amax / 224)): with amax = m 2^E (m in [1, 2)) the exponent is
    // E - 7, less one when m < 1.75
    int e = 0;
    if (amax > 0.f) {
        uint32_t u = __float_as_uint(amax);
        int E = (int)(u >> 23) - 127;
        uint32_t mant = u & 0x7FFFFFu;
        e = E - 7 - (mant < 0x600000u ? 1 : 0);
        if ((u >> 23) == 0) e = -126;      // subnormal amax
        e = max(e, -126);
    }
    const float s = __uint_as_float((uint32_t)(127 + e) << 23);
    const float inv = __uint_as_float((uint32_t)(127 - e) << 23);
    for (int c = lane; c < D; c += 64) dst[(long)row * D + c] = (uint8_t)f32_to_e4m3(x[c] * inv);
    if (lane == 0) scale[row] = s;
}

template <int DT>
__global__ __launch_bounds__(256) void l1_grad_kernel(long n, const void *__restrict__ x,
                                                      const void *__restrict__ tgt, float scale,
                                                      void *__restrict__ grad) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if constexpr (DT == MT_F32) {
        float d = ((const float *)x)[i] - ((const float *)tgt)[i];
        ((float *)grad)[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    } else {
        float d = bf16_to_f32(((const uint16_t *)x)[i]) - bf16_to_f32(((const uint16_t *)tgt)[i]);
        float g = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
        ((uint16_t *)grad)[i] = f32_to_bf16(g);
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

// ---------------------------------------------------------------- dispatch

template <int FT, int MT>
lgs_status fwd_dispatch(int k, long n_pix, int D, const void *feat, const float *scale, const int *ids,
                        const float *tw, void *F, hipStream_t st) {
    unsigned grid = padded_grid((n_pix + kFwdPixPerBlock - 1) / kFwdPixPerBlock);
#define CALL(KK)                                                                                     \
    case KK:                                                                                         \
        hipLaunchKernelGGL((feature_fwd_kernel<KK, FT, MT>), dim3(grid), dim3(256), 0, st, n_pix, D, \
                           feat, scale, ids, tw, F);                                                 \
        break;
    switch (k) { CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(8) CALL(10) CALL(16) }
#undef CALL
    return check_launch("feature_render_fwd");
}

template <int FT, int MT>
lgs_status bwd_dispatch(int k, int W, int H, int views, int D, const void *feat, const float *scale,
                        const int *ids, const float *tw, const void *dF, float *dfeat, float *dtw,
                        hipStream_t st) {
    long tiles = (long)tiles_x(W) * tiles_y(H) * views;
    unsigned grid = padded_grid(tiles);
    size_t lds = (size_t)bwd_lds(k).total;
#define CALL(KK)                                                                                    \
    case KK:                                                                                        \
        if (hipFuncSetAttribute((const void *)feature_bwd_kernel<KK, FT, MT>,                      \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) { \
            set_error("feature_render_bwd: %zu bytes of LDS unavailable", lds);                     \
            return LGS_ERR_UNSUPPORTED;                                                             \
        }                                                                                           \
        hipLaunchKernelGGL((feature_bwd_kernel<KK, FT, MT>), dim3(grid), dim3(256), lds, st, W, H, \
                           views, D, feat, scale, ids, tw, dF, dfeat, dtw);                         \
        break;
    switch (k) { CALL(1) CALL(2) CALL(3) CALL(4) CALL(5) CALL(8) CALL(10) CALL(16) }
#undef CALL
    return check_launch("feature_render_bwd");
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
    long n_pix = (long)width * height * views;
    if (feat_dt == LGS_F32) return fwd_dispatch<FT_F32, MT_F32>(k, n_pix, d, feat, feat_scale, topk_ids, topk_w, F, stream);
    if (feat_dt == LGS_BF16 && map_dt == LGS_BF16)
        return fwd_dispatch<FT_BF16, MT_BF16>(k, n_pix, d, feat, feat_scale, topk_ids, topk_w, F, stream);
    if (feat_dt == LGS_BF16) return fwd_dispatch<FT_BF16, MT_F32>(k, n_pix, d, feat, feat_scale, topk_ids, topk_w, F, stream);
    if (map_dt == LGS_BF16) return fwd_dispatch<FT_FP8, MT_BF16>(k, n_pix, d, feat, feat_scale, topk_ids, topk_w, F, stream);
    return fwd_dispatch<FT_FP8, MT_F32>(k, n_pix, d, feat, feat_scale, topk_ids, topk_w, F, stream);
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
    if (feat_dt == LGS_F32)
        return bwd_dispatch<FT_F32, MT_F32>(k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dL_dF, dL_dfeat, dL_dtopkw, stream);
    if (feat_dt == LGS_BF16 && map_dt == LGS_BF16)
        return bwd_dispatch<FT_BF16, MT_BF16>(k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dL_dF, dL_dfeat, dL_dtopkw, stream);
    if (feat_dt == LGS_BF16)
        return bwd_dispatch<FT_BF16, MT_F32>(k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dL_dF, dL_dfeat, dL_dtopkw, stream);
    if (map_dt == LGS_BF16)
        return bwd_dispatch<FT_FP8, MT_BF16>(k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dL_dF, dL_dfeat, dL_dtopkw, stream);
    return bwd_dispatch<FT_FP8, MT_F32>(k, width, height, views, d, feat, feat_scale, topk_ids, topk_w, dL_dF, dL_dfeat, dL_dtopkw, stream);
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
    unsigned grid = (unsigned)((n + 255) / 256);
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
