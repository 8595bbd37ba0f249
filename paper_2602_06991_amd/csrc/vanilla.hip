// Vanilla feature render: the D-channel feature field alpha-blended exactly as the
// colour of Eq. 1, over every blended Gaussian, F[p] = sum_i w_i f_i with the blend's
// own weights w_i = alpha_i T_i (the dense feature rasterisation that Top-K rendering
// replaces, Sec. 3.2 and Tab. 4), and its adjoint.  It serves as the comparison path.
//
// Both kernels take one 256-thread block per (16x16 tile, 128-channel chunk) and walk
// the tile's depth-sorted list in batches (32 Gaussians in the forward, 16 in the
// adjoint), replaying the blend of each pixel with the forward's arithmetic up to its
// n_contrib, so every weight is the forward's bit for bit.
//
// Forward: per batch the weights W[256 px][32] (split into two BF16 terms, hi and lo)
// and the rows Ft[32][128 ch] go to LDS and the chunk of the map accumulates on the
// matrix cores, F += W Ft (v_mfma_f32_16x16x32_bf16, FP32 accumulators, 64 pixels x
// 128 channels per wave); the map is rounded to BF16 once and stored through LDS in
// whole pixel rows.
//
// Adjoint (given dL/dF = G): per pixel the blend is replayed back to front from T_final
// (as in the blend adjoint); the feature term of the weight gradient is
// e_i = <G, f_i>, so dL/dalpha_i = T_i e_i - (sum_{j>i} w_j e_j) / (1 - alpha_i).  Both
// are linear in the channels, so each 128-channel chunk adds its own share: the chunk
// of every e_i comes from S = G Ft^T on the matrix cores, and the screen-space
// gradients of the chunk are summed over the tile and added with atomics.  The
// feature rows take dFt = W^T G (MFMA, the four waves' partial sums meet in LDS), one
// atomic per element and (tile, batch).
#include "lgs_device.hpp"
#include "tile_map.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

typedef short v_i16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 v_bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kVB = 32;        // Gaussians per batch of the forward (the MFMA K of the map product)
constexpr int kVBB = 16;       // Gaussians per batch of the adjoint (one MFMA row block; its LDS fits two blocks per CU)
constexpr int kVC = 128;       // channels per block
constexpr int kVT = 256;       // threads per block
constexpr int kWS = kVB + 8;   // LDS row stride (BF16) of the weight rows, padded against bank conflicts
constexpr int kFS = kVC + 8;   // LDS row stride (BF16) of the feature rows

enum { VF_BF16 = 1, VF_FP8 = 2 };

// D[4g+r][i] += sum_k A[i][k] B[k][i'] with lane l = 16 g + i: A[i][8g..8g+7],
// B[8g..8g+7][i] (v_mfma_f32_16x16x32_bf16).
__device__ __forceinline__ f32x4 vmfma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v_bf16x8, a), __builtin_bit_cast(v_bf16x8, b),
                                                   c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// E4M3FN code -> BF16 bits (exact: 3 mantissa bits, exponents within BF16's range).
__device__ __forceinline__ uint16_t e4m3_bf16(uint32_t c) { return to_bf16(e4m3_to_f32(c)); }

struct VanArgs {
    int W, H, ntx, nty, D;
    const float2 *mean2d;
    const float *conic;
    const float *opacity;
    const int *sorted_ids;
    const int2 *ranges;
    const int *n_contrib;
};

// Stages 32 rows x 128 channels of the feature table (BF16, or FP8 codes widened to
// BF16 exactly); channels past D and rows past cnt are zero.  Thread t copies 16
// channels of row t / 8.  TRANS: into ft[channel][kTS] (channel-major, for the map's
// B operand), else into ft[row][kFS].
constexpr int kTS = kVB + 8;   // LDS row stride (BF16) of the channel-major rows

template <int FT, bool TRANS, int NR = kVB>
__device__ __forceinline__ void stage_rows32(const VanArgs &a, const void *__restrict__ feat, const int *s_id, int cnt,
                                             int c0, uint16_t *ft) {
    const int t = threadIdx.x;
    const int j = t >> 3, cc = (t & 7) * 16;
    if (j >= NR) return;   // NR rows of 8 threads each
    uint16_t v[16];
    const int c = c0 + cc;
    if (j < cnt && c < a.D) {
        const long row = s_id[j];
        if constexpr (FT == VF_BF16) {
            const u32x4 *src = (const u32x4 *)((const uint16_t *)feat + row * a.D + c);
            const u32x4 x0 = src[0];
            const u32x4 x1 = (c + 8 < a.D) ? src[1] : u32x4{0u, 0u, 0u, 0u};
            *(u32x4 *)&v[0] = x0;
            *(u32x4 *)&v[8] = x1;
        } else {
            const uint8_t *src = (const uint8_t *)feat + row * a.D + c;
            const u32x2 x0 = *(const u32x2 *)src;
            const u32x2 x1 = (c + 8 < a.D) ? *(const u32x2 *)(src + 8) : u32x2{0u, 0u};
            const uint32_t w[4] = {x0.x, x0.y, x1.x, x1.y};
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = e4m3_bf16((w[q >> 2] >> (8 * (q & 3))) & 0xFFu);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = 0;
    }
    if constexpr (TRANS) {
#pragma unroll
        for (int q = 0; q < 16; ++q) ft[(cc + q) * kTS + j] = v[q];
    } else {
        *(u32x4 *)&ft[j * kFS + cc] = *(u32x4 *)&v[0];
        *(u32x4 *)&ft[j * kFS + cc + 8] = *(u32x4 *)&v[8];
    }
}

// ---------------------------------------------------------------- forward

template <int FT>
__global__ __launch_bounds__(kVT, 2) void vanilla_fwd_kernel(VanArgs a, const void *__restrict__ feat,
                                                            const float *__restrict__ scale,
                                                            uint16_t *__restrict__ F) {
    extern __shared__ __align__(16) unsigned char dyn[];
    uint16_t *w_hi = (uint16_t *)dyn;                 // [256][kWS]
    uint16_t *w_lo = w_hi + kVT * kWS;                // [256][kWS]
    uint16_t *ft = w_lo + kVT * kWS;                  // [kVC][kTS] channel-major
    __shared__ int s_id[kVB];
    __shared__ float2 s_xy[kVB];
    __shared__ float4 s_co[kVB];
    __shared__ float s_sc[kVB];
    __shared__ int s_max;
    const int nchunks = (a.D + kVC - 1) / kVC;
    const int ntiles = a.ntx * a.nty;
    const int item = xcd_strips(blockIdx.x);   // strips of items over the XCDs, as the blend kernels
    if (item >= ntiles * nchunks) return;
    const int tile = item / nchunks, chunk = item - tile * nchunks;
    const int c0 = chunk * kVC;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lg = lane >> 4;
    const int x0 = (tile % a.ntx) * kTile, y0 = (tile / a.ntx) * kTile;
    const int px = x0 + (t & 15), py = y0 + (t >> 4);
    const bool valid = px < a.W && py < a.H;
    const long p = (long)py * a.W + px;
    const int2 rg = a.ranges[tile];
    const int last = valid ? a.n_contrib[p] : 0;
    if (t == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, last);
    __syncthreads();
    const int maxl = s_max;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float T = 1.0f;
    f32x4 acc[4][8];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int base = 0; base < maxl; base += kVB) {
        const int cnt = min(kVB, maxl - base);
        __syncthreads();   // the previous batch's operands are consumed
        if (t < cnt) {
            const int r = a.sorted_ids[rg.x + base + t];
            s_id[t] = r;
            s_xy[t] = a.mean2d[r];
            s_co[t] = make_float4(a.conic[3 * r], a.conic[3 * r + 1], a.conic[3 * r + 2], a.opacity[r]);
            s_sc[t] = FT == VF_FP8 ? scale[r] : 1.0f;
        }
        __syncthreads();
        stage_rows32<FT, true>(a, feat, s_id, cnt, c0, ft);
        // the pixel's weights of this batch (the forward's arithmetic), times the FP8 row scale
        for (int j = 0; j < kVB; ++j) {
            float w = 0.f;
            if (j < cnt && base + j < last) {
                const float2 m = s_xy[j];
                const float4 co = s_co[j];
                float dx, dy, raw, ex;
                const float alpha = blend_alpha(fx, fy, m.x, m.y, co.x, co.y, co.z, co.w, dx, dy, raw, ex);
                if (alpha >= kAlphaMin) {
                    w = alpha * T;
                    T = T * (1.0f - alpha);
                }
            }
            const float ws = w * s_sc[j < cnt ? j : 0];
            const uint16_t hi = to_bf16(ws);
            w_hi[t * kWS + j] = hi;
            w_lo[t * kWS + j] = to_bf16(ws - from_bf16(hi));
        }
        __syncthreads();
        // F[64 px of the wave][128 ch] += W[px][32] Ft[32][ch]
        u32x4 b[8];   // B[8g..8g+7][i] = Ft[Gaussian 8g..8g+7][channel 16 nb + i]
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) b[nb] = *(const u32x4 *)&ft[(16 * nb + li) * kTS + 8 * lg];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int row = 64 * wave + 16 * mb + li;
            const u32x4 ah = *(const u32x4 *)&w_hi[row * kWS + 8 * lg];
            const u32x4 al = *(const u32x4 *)&w_lo[row * kWS + 8 * lg];
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                acc[mb][nb] = vmfma(ah, b[nb], acc[mb][nb]);
                acc[mb][nb] = vmfma(al, b[nb], acc[mb][nb]);
            }
        }
    }
    // store: the wave's 64 px x 128 ch block goes through LDS so that each lane writes
    // 16 consecutive bytes of one pixel row
    __syncthreads();
    uint16_t *stage = (uint16_t *)dyn + wave * 64 * kFS;   // [64 px][kFS]
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) stage[(16 * mb + 4 * lg + r) * kFS + 16 * nb + li] = to_bf16(acc[mb][nb][r]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // 64 px x 16 segments of 16 B per wave: 16 rounds of 64 lanes
    for (int q = lane; q < 64 * 16; q += 64) {
        const int pr = q >> 4, seg = q & 15;
        const int pix = 64 * wave + pr;
        const int xx = x0 + (pix & 15), yy = y0 + (pix >> 4);
        const int c = c0 + 8 * seg;
        if (xx < a.W && yy < a.H && c < a.D) {
            const long pp = (long)yy * a.W + xx;
            *(u32x4 *)&F[pp * a.D + c] = *(const u32x4 *)&stage[pr * kFS + 8 * seg];
        }
    }
}

// ---------------------------------------------------------------- adjoint

constexpr int kNV = 6;   // screen-space gradient slots: mean2d 2, conic 3, opacity 1

// Row sums over the 16 lanes of each lane row (every lane takes part).
template <int N>
__device__ __forceinline__ void vrow_sum(float (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0xB1>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x4E>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x141>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x140>(v[q]);
}

template <int FT>
__global__ __launch_bounds__(kVT, 2) void vanilla_bwd_kernel(VanArgs a, const void *__restrict__ feat,
                                                            const float *__restrict__ scale,
                                                            const float *__restrict__ T_final,
                                                            const uint16_t *__restrict__ G,
                                                            float *__restrict__ dfeat, float *__restrict__ g_mean2d,
                                                            float *__restrict__ g_conic, float *__restrict__ g_opac) {
    extern __shared__ __align__(16) unsigned char dyn[];
    // batch area (its start also stages half of the tile's dL/dF chunk at a time)
    uint16_t *ft = (uint16_t *)dyn;                                  // [kVBB][kFS] BF16
    float *s_S = (float *)(dyn + kVBB * kFS * 2);                    // [256][kVBB + 1] FP32
    uint16_t *wt_hi = (uint16_t *)(s_S + kVT * (kVBB + 1));          // [kVBB][kVT + 8] BF16
    uint16_t *wt_lo = wt_hi + kVBB * (kVT + 8);                      // [kVBB][kVT + 8]
    float *s_dF = (float *)(wt_lo + kVBB * (kVT + 8));               // [kVBB][kVC] FP32
    float *s_part = s_dF + kVBB * kVC;                               // [16 rows][kVBB][kNV]
    __shared__ int s_id[kVBB];
    __shared__ float2 s_xy[kVBB];
    __shared__ float4 s_co[kVBB];
    __shared__ float s_sc[kVBB];
    __shared__ int s_max;
    const int nchunks = (a.D + kVC - 1) / kVC;
    const int ntiles = a.ntx * a.nty;
    const int item = xcd_strips(blockIdx.x);   // strips of items over the XCDs, as the blend kernels
    if (item >= ntiles * nchunks) return;
    const int tile = item / nchunks, chunk = item - tile * nchunks;
    const int c0 = chunk * kVC;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lg = lane >> 4;
    const int x0 = (tile % a.ntx) * kTile, y0 = (tile / a.ntx) * kTile;
    const int px = x0 + (t & 15), py = y0 + (t >> 4);
    const bool valid = px < a.W && py < a.H;
    const long p = (long)py * a.W + px;
    const int2 rg = a.ranges[tile];
    const int last = valid ? a.n_contrib[p] : 0;
    float T = valid ? T_final[p] : 1.0f;
    if (t == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, last);
    // the tile's dL/dF chunk [256 px][128 ch] through LDS, half the pixels at a time (BF16,
    // padded rows; zero past the image or D), into registers in the two operand layouts;
    // the waves whose pixels the half holds (two each) take their operands from it
    uint16_t *gs = (uint16_t *)dyn;   // [128][kFS]
    u32x4 ga[4][4];   // S = G Ft^T: A[i][8g..] = G[px 64 w + 16 mb + i][ch 32 ks + 8 g ..]
    u32x4 gb[2][8];   // dFt = W^T G: B[8g..][i] = G[px 64 w + 32 kp + 8 g + q][ch 16 nb + i]
    for (int half = 0; half < 2; ++half) {
        if (half) __syncthreads();   // the first half's operands are loaded
        for (int q = t; q < (kVT / 2) * 16; q += kVT) {
            const int pix = (kVT / 2) * half + (q >> 4), seg = q & 15;
            const int xx = x0 + (pix & 15), yy = y0 + (pix >> 4);
            const int c = c0 + 8 * seg;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (xx < a.W && yy < a.H && c < a.D) v = *(const u32x4 *)&G[((long)yy * a.W + xx) * a.D + c];
            *(u32x4 *)&gs[(q >> 4) * kFS + 8 * seg] = v;
        }
        __syncthreads();
        if ((wave >> 1) != half) continue;
        const int wrow = 64 * (wave & 1);   // the wave's first pixel within the half
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) ga[mb][ks] = *(const u32x4 *)&gs[(wrow + 16 * mb + li) * kFS + 32 * ks + 8 * lg];
#pragma unroll
        for (int kp = 0; kp < 2; ++kp)
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                uint16_t col[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) col[q] = gs[(wrow + 32 * kp + 8 * lg + q) * kFS + 16 * nb + li];
                gb[kp][nb] = *(u32x4 *)col;
            }
    }
    const int maxl = s_max;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    float A = 0.f;
    for (int hi = maxl; hi > 0; hi -= kVBB) {
        const int lo = hi > kVBB ? hi - kVBB : 0;
        const int cnt = hi - lo;
        __syncthreads();   // the previous batch (and the G staging) are consumed
        if (t < cnt) {
            const int r = a.sorted_ids[rg.x + lo + t];
            s_id[t] = r;
            s_xy[t] = a.mean2d[r];
            s_co[t] = make_float4(a.conic[3 * r], a.conic[3 * r + 1], a.conic[3 * r + 2], a.opacity[r]);
            s_sc[t] = FT == VF_FP8 ? scale[r] : 1.0f;
        }
        for (int q = t; q < kVBB * kVC; q += kVT) s_dF[q] = 0.f;
        __syncthreads();
        stage_rows32<FT, false, kVBB>(a, feat, s_id, cnt, c0, ft);
        __syncthreads();
        // S chunk of the batch: the wave's 64 px x kVBB Gaussians
#pragma unroll
        for (int nbg = 0; nbg < kVBB / 16; ++nbg) {
            u32x4 bs[4];   // B[8g..][i] = Ft[Gaussian 16 nbg + i][ch 32 ks + 8 g ..]
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) bs[ks] = *(const u32x4 *)&ft[(16 * nbg + li) * kFS + 32 * ks + 8 * lg];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                f32x4 s = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) s = vmfma(ga[mb][ks], bs[ks], s);
#pragma unroll
                for (int r = 0; r < 4; ++r) s_S[(64 * wave + 16 * mb + 4 * lg + r) * (kVBB + 1) + 16 * nbg + li] = s[r];
            }
        }
        __syncthreads();
        // back-to-front replay of the pixel over the batch
        for (int j = kVBB - 1; j >= 0; --j) {
            float v[kNV] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float w = 0.f;
            bool hit = false;
            if (j < cnt && lo + j < last) {
                const float2 m = s_xy[j];
                const float4 co = s_co[j];
                float dx, dy, raw, ex;
                const float alpha = blend_alpha(fx, fy, m.x, m.y, co.x, co.y, co.z, co.w, dx, dy, raw, ex);
                if (alpha >= kAlphaMin) {
                    hit = true;
                    const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
                    T *= r;                               // transmittance in front of this Gaussian
                    w = alpha * T;
                    const float e = s_S[t * (kVBB + 1) + j] * s_sc[j];
                    const float dal = T * e - A * r;
                    A = fmaf(e, w, A);
                    if (raw <= kAlphaMax) {               // unclamped: alpha = o e^-sigma
                        const float ds = -alpha * dal;
                        v[0] = -ds * (co.x * dx + co.y * dy);
                        v[1] = -ds * (co.y * dx + co.z * dy);
                        v[2] = ds * 0.5f * dx * dx;
                        v[3] = ds * dx * dy;
                        v[4] = ds * 0.5f * dy * dy;
                        v[5] = dal * ex;
                    }
                }
            }
            const uint16_t whi = to_bf16(w);
            wt_hi[j * (kVT + 8) + t] = whi;
            wt_lo[j * (kVT + 8) + t] = to_bf16(w - from_bf16(whi));
            if (__ballot(hit) != 0ull) vrow_sum<kNV>(v);
            if ((t & 15) == 0) {
                float *dst = &s_part[((t >> 4) * kVBB + j) * kNV];
#pragma unroll
                for (int q = 0; q < kNV; ++q) dst[q] = v[q];
            }
        }
        __syncthreads();
        // screen-space gradients of the batch: the 16 row sums per Gaussian and slot in a
        // fixed order, one atomic each
        for (int o = t; o < cnt * kNV; o += kVT) {
            const int j = o / kNV, q = o - j * kNV;
            float sum = 0.f;
#pragma unroll
            for (int r = 0; r < 16; ++r) sum += s_part[(r * kVBB + j) * kNV + q];
            if (sum == 0.f) continue;
            const int rec = s_id[j];
            float *dst = q < 2 ? &g_mean2d[2 * rec + q] : q < 5 ? &g_conic[3 * rec + (q - 2)] : &g_opac[rec];
            unsafeAtomicAdd(dst, sum);
        }
        // dFt[kVBB Gaussians][128 ch] = W^T G over the wave's 64 pixels, partial sums meet in LDS
#pragma unroll
        for (int mbg = 0; mbg < kVBB / 16; ++mbg) {
            u32x4 ah[2], al[2];   // A[i][8g..] = W^T[Gaussian 16 mbg + i][px 64 w + 32 kp + 8 g ..]
#pragma unroll
            for (int kp = 0; kp < 2; ++kp) {
                ah[kp] = *(const u32x4 *)&wt_hi[(16 * mbg + li) * (kVT + 8) + 64 * wave + 32 * kp + 8 * lg];
                al[kp] = *(const u32x4 *)&wt_lo[(16 * mbg + li) * (kVT + 8) + 64 * wave + 32 * kp + 8 * lg];
            }
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                f32x4 d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kp = 0; kp < 2; ++kp) {
                    d = vmfma(ah[kp], gb[kp][nb], d);
                    d = vmfma(al[kp], gb[kp][nb], d);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) atomicAdd(&s_dF[(16 * mbg + 4 * lg + r) * kVC + 16 * nb + li], d[r]);
            }
        }
        __syncthreads();
        for (int q = t; q < cnt * kVC; q += kVT) {
            const int j = q / kVC, c = q - j * kVC;
            const float v = s_dF[q];
            if (c0 + c < a.D && v != 0.f) unsafeAtomicAdd(&dfeat[(long)(s_id[j]) * a.D + c0 + c], v);
        }
    }
}

constexpr size_t kFwdLds = (size_t)2 * kVT * kWS * 2 + (size_t)kVC * kTS * 2;
constexpr size_t kFwdLdsStore = (size_t)4 * 64 * kFS * 2;
constexpr size_t kBwdLds = (size_t)kVBB * kFS * 2 + (size_t)kVT * (kVBB + 1) * 4 + (size_t)2 * kVBB * (kVT + 8) * 2 +
                           (size_t)kVBB * kVC * 4 + (size_t)16 * kVBB * kNV * 4;
constexpr size_t kBwdLdsStage = (size_t)(kVT / 2) * kFS * 2;

lgs_status van_args(const lgs_camera *cam, int d, lgs_dtype feat_dt, const void *feat, const float *feat_scale,
                    lgs_dtype map_dt, const float *mean2d, const float *conic, const float *opacity,
                    const int32_t *sorted_ids, const int32_t *tile_ranges, const int32_t *n_contrib, VanArgs &a) {
    lgs_status st = check_camera(cam);
    if (st) return st;
    LGS_REQUIRE(d > 0 && d % 8 == 0, LGS_ERR_UNSUPPORTED, "d = %d must be a positive multiple of 8", d);
    LGS_REQUIRE((feat_dt == LGS_BF16 || feat_dt == LGS_FP8_E4M3) && map_dt == LGS_BF16, LGS_ERR_UNSUPPORTED,
                "the vanilla feature render takes BF16 or FP8 storage and a BF16 map");
    LGS_REQUIRE(feat && mean2d && conic && opacity && sorted_ids && tile_ranges && n_contrib, LGS_ERR_INVALID_ARG,
                "vanilla feature render: NULL pointer");
    LGS_REQUIRE(feat_dt != LGS_FP8_E4M3 || feat_scale, LGS_ERR_INVALID_ARG, "FP8 features need feat_scale");
    LGS_REQUIRE(aligned16(feat), LGS_ERR_INVALID_ARG, "feat must be 16-byte aligned");
    LGS_REQUIRE(((uintptr_t)mean2d & 7u) == 0 && ((uintptr_t)tile_ranges & 7u) == 0, LGS_ERR_INVALID_ARG,
                "mean2d and tile_ranges must be 8-byte aligned");
    a.W = cam->width;
    a.H = cam->height;
    a.ntx = tiles_x(a.W);
    a.nty = tiles_y(a.H);
    a.D = d;
    a.mean2d = (const float2 *)mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.sorted_ids = sorted_ids;
    a.ranges = (const int2 *)tile_ranges;
    a.n_contrib = n_contrib;
    return LGS_OK;
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_feature_render_vanilla_fwd(const lgs_camera *cam, const float *mean2d, const float *conic,
                                                     const float *opacity, const int32_t *sorted_ids,
                                                     const int32_t *tile_ranges, const int32_t *n_contrib, int32_t d,
                                                     lgs_dtype feat_dt, const void *feat, const float *feat_scale,
                                                     lgs_dtype map_dt, void *F, hipStream_t stream) {
    VanArgs a;
    lgs_status st = van_args(cam, d, feat_dt, feat, feat_scale, map_dt, mean2d, conic, opacity, sorted_ids,
                             tile_ranges, n_contrib, a);
    if (st) return st;
    LGS_REQUIRE(F && aligned16(F), LGS_ERR_INVALID_ARG, "F must be non-NULL and 16-byte aligned");
    const long items = (long)a.ntx * a.nty * ((d + kVC - 1) / kVC);
    const size_t lds = std::max(kFwdLds, kFwdLdsStore);
    if (feat_dt == LGS_BF16)
        hipLaunchKernelGGL(vanilla_fwd_kernel<VF_BF16>, dim3(strip_grid(items)), dim3(kVT), lds, stream, a, feat,
                           feat_scale, (uint16_t *)F);
    else
        hipLaunchKernelGGL(vanilla_fwd_kernel<VF_FP8>, dim3(strip_grid(items)), dim3(kVT), lds, stream, a, feat,
                           feat_scale, (uint16_t *)F);
    return check_launch("feature_render_vanilla_fwd");
}

extern "C" lgs_status lgs_feature_render_vanilla_bwd(const lgs_camera *cam, const float *mean2d, const float *conic,
                                                     const float *opacity, const int32_t *sorted_ids,
                                                     const int32_t *tile_ranges, const float *T_final,
                                                     const int32_t *n_contrib, int32_t d, lgs_dtype feat_dt,
                                                     const void *feat, const float *feat_scale, lgs_dtype map_dt,
                                                     const void *dL_dF, float *dL_dfeat, float *dL_dmean2d,
                                                     float *dL_dconic, float *dL_dopacity, hipStream_t stream) {
    VanArgs a;
    lgs_status st = van_args(cam, d, feat_dt, feat, feat_scale, map_dt, mean2d, conic, opacity, sorted_ids,
                             tile_ranges, n_contrib, a);
    if (st) return st;
    LGS_REQUIRE(T_final && dL_dF && dL_dfeat && dL_dmean2d && dL_dconic && dL_dopacity, LGS_ERR_INVALID_ARG,
                "lgs_feature_render_vanilla_bwd: NULL pointer");
    LGS_REQUIRE(aligned16(dL_dF), LGS_ERR_INVALID_ARG, "dL_dF must be 16-byte aligned");
    const long items = (long)a.ntx * a.nty * ((d + kVC - 1) / kVC);
    const size_t lds = std::max(kBwdLds, kBwdLdsStage);
    if (feat_dt == LGS_BF16)
        hipLaunchKernelGGL(vanilla_bwd_kernel<VF_BF16>, dim3(strip_grid(items)), dim3(kVT), lds, stream, a, feat,
                           feat_scale, T_final, (const uint16_t *)dL_dF, dL_dfeat, dL_dmean2d, dL_dconic, dL_dopacity);
    else
        hipLaunchKernelGGL(vanilla_bwd_kernel<VF_FP8>, dim3(strip_grid(items)), dim3(kVT), lds, stream, a, feat,
                           feat_scale, T_final, (const uint16_t *)dL_dF, dL_dfeat, dL_dmean2d, dL_dconic, dL_dopacity);
    return check_launch("feature_render_vanilla_bwd");
}
