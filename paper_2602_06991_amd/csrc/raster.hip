// Per-tile alpha blending of colour, depth and opacity (Eq. 1) that keeps each
// pixel's K largest blending weights in registers (Eq. 2; recorded during the same
// pass, Sec. 3.2), and its adjoint replayed back to front from the saved final
// transmittance.  One block of 128 threads per 16x16 tile, two pixels per thread
// (rows y and y + 8); the tile's depth-sorted Gaussians are staged through LDS in
// batches (256 forward, 32 backward).
//
// Tiles go to blocks in one of two ways.  When the view count is a multiple of 8, each
// XCD takes a contiguous band (xcd_remap), which is then a set of whole views: a view's
// neighbouring tiles, which share Gaussians, meet in one L2.  Otherwise the tiles go in
// strips of 16 dealt to the XCDs in turn (xcd_strips), so that every XCD gets an even
// share of the image: a frame's rows differ in how many Gaussians they blend, and these
// kernels are bound by instruction issue.  Measured: bands take 0.56 + 1.18 ms for the
// 8 x 640x480 blend and adjoint against 0.72 + 1.42 in strips; strips take 0.50 + 0.97 ms
// at 4 x 1200x680 against 0.61 + 1.23 in bands; one 1200x680 view is even.
#include "lgs_device.hpp"
#include "tile_map.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

// Views are batched: the tiles of view v are tiles v*ntx*nty ... of the grid, its
// pixels v*W*H ... of the per-pixel arrays, and its projected records (mean2d, conic,
// opacity, depth) are records v*n ... ; the sorted lists hold record indices, the
// Top-K lists and colours Gaussian ids (record - v*n).
struct RasterArgs {
    int W, H, ntx, nty, views, n;
    bool bands;   // tile -> block: contiguous bands per XCD (whole views), else strips
    const float2 *mean2d;
    const float *conic;
    const float *opacity;
    const float *rgb;
    const float *depth;
    const int *sorted_ids;
    const int2 *ranges;
    const int *order;   // block -> tile from lgs_tile_order, or null for the fixed mapping
};

struct TilePos {
    int view, tile, x0, y0;   // view, tile index over all views, first pixel column / row
    long pix0;                // first pixel of the view in the per-pixel arrays
    int rec0;                 // first record of the view
};

__device__ __forceinline__ TilePos tile_pos(const RasterArgs &a, int tile) {
    const int per = a.ntx * a.nty;
    TilePos t;
    t.view = tile / per;
    const int lt = tile - t.view * per;
    t.tile = tile;
    t.x0 = (lt % a.ntx) * kTile;
    t.y0 = (lt / a.ntx) * kTile;
    t.pix0 = (long)t.view * a.W * a.H;
    t.rec0 = t.view * a.n;
    return t;
}

// The tile block blockIdx.x renders: from the dispatch order when one is given (an entry
// outside [0, ntiles) runs nothing), else bands or strips over the XCDs.
__device__ __forceinline__ int block_tile(const RasterArgs &a, int ntiles) {
    if (a.order) {
        const int t = a.order[blockIdx.x];
        return (unsigned)t < (unsigned)ntiles ? t : ntiles;
    }
    return a.bands ? xcd_remap(blockIdx.x, gridDim.x) : xcd_strips(blockIdx.x);
}

template <int K>
__device__ __forceinline__ void topk_insert(float (&tw)[K], int (&ti)[K], float w, int id) {
    // strictly larger weights displace; equal weights keep blend order
    if (w > tw[K - 1]) {
        tw[K - 1] = w;
        ti[K - 1] = id;
#pragma unroll
        for (int i = K - 1; i > 0; --i) {
            if (tw[i] > tw[i - 1]) {
                float a = tw[i]; tw[i] = tw[i - 1]; tw[i - 1] = a;
                int b = ti[i]; ti[i] = ti[i - 1]; ti[i - 1] = b;
            }
        }
    }
}

// The forward gives each thread two pixels of the tile, (x, y) and (x, y + 8): the
// Gaussian's LDS records are read once for both.
constexpr int kFwdThreads = 128;

template <int K>
__global__ __launch_bounds__(kFwdThreads) void raster_fwd_kernel(RasterArgs a, float *__restrict__ color,
                                                                 float *__restrict__ depth_map,
                                                                 float *__restrict__ alpha_map,
                                                                 float *__restrict__ T_final,
                                                                 int *__restrict__ n_contrib,
                                                                 int *__restrict__ topk_ids,
                                                                 float *__restrict__ topk_w) {
    __shared__ int s_id[256];
    __shared__ float2 s_xy[256];
    __shared__ float4 s_co[256];   // conic a, b, c, opacity
    __shared__ float4 s_cz[256];   // r, g, b, depth
    const int ntiles = a.ntx * a.nty * a.views;
    const int tile = block_tile(a, ntiles);
    if (tile >= ntiles) return;
    const TilePos tp = tile_pos(a, tile);
    const int t = threadIdx.x;
    const int px = tp.x0 + (t & 15);
    const int py0 = tp.y0 + (t >> 4);
    const float fx = (float)px + 0.5f;
    const int2 rg = a.ranges[tile];
    float fy[2], T[2], C0[2], C1[2], C2[2], Dz[2];
    int last[2];
    bool done[2];
    float tw[2][K];
    int ti[2][K];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int py = py0 + 8 * h;
        fy[h] = (float)py + 0.5f;
        T[h] = 1.0f; C0[h] = C1[h] = C2[h] = Dz[h] = 0.f;
        last[h] = 0;
        done[h] = !(px < a.W && py < a.H);
#pragma unroll
        for (int k = 0; k < K; ++k) { tw[h][k] = 0.0f; ti[h][k] = -1; }
    }
    for (int base = rg.x; base < rg.y; base += 256) {
        if (__syncthreads_count(done[0] && done[1]) == kFwdThreads) break;
        for (int idx = base + t; idx < min(base + 256, rg.y); idx += kFwdThreads) {
            const int r = a.sorted_ids[idx];
            const int g = r - tp.rec0;
            const int q = idx - base;
            s_id[q] = g;
            s_xy[q] = a.mean2d[r];
            s_co[q] = make_float4(a.conic[3 * r], a.conic[3 * r + 1], a.conic[3 * r + 2], a.opacity[r]);
            s_cz[q] = make_float4(a.rgb[3 * g], a.rgb[3 * g + 1], a.rgb[3 * g + 2], a.depth[r]);
        }
        __syncthreads();
        const int cnt = min(256, rg.y - base);
        for (int j = 0; j < cnt && !(done[0] && done[1]); ++j) {
            const float2 m = s_xy[j];
            const float4 co = s_co[j];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (done[h]) continue;
                float dx, dy, raw, ex;
                const float alpha = blend_alpha(fx, fy[h], m.x, m.y, co.x, co.y, co.z, co.w, dx, dy, raw, ex);
                if (alpha < kAlphaMin) continue;
                const float nT = T[h] * (1.0f - alpha);
                if (nT < kTMin) {
                    done[h] = true;
                    continue;
                }
                const float w = alpha * T[h];
                const float4 cz = s_cz[j];
                C0[h] = fmaf(cz.x, w, C0[h]);
                C1[h] = fmaf(cz.y, w, C1[h]);
                C2[h] = fmaf(cz.z, w, C2[h]);
                Dz[h] = fmaf(cz.w, w, Dz[h]);
                T[h] = nT;
                last[h] = base + j - rg.x + 1;
                topk_insert<K>(tw[h], ti[h], w, s_id[j]);
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int py = py0 + 8 * h;
        if (!(px < a.W && py < a.H)) continue;
        const long p = tp.pix0 + (long)py * a.W + px;
        color[3 * p] = C0[h];
        color[3 * p + 1] = C1[h];
        color[3 * p + 2] = C2[h];
        depth_map[p] = Dz[h];
        alpha_map[p] = 1.0f - T[h];
        T_final[p] = T[h];
        n_contrib[p] = last[h];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            topk_ids[p * K + k] = ti[h][k];
            topk_w[p * K + k] = tw[h][k];
        }
    }
}

constexpr int kNG = 10;   // per-Gaussian gradient slots: mean2d 2, conic 3, opacity, rgb 3, depth
constexpr int kNGP = 12;  // the same, padded to whole 16-byte LDS stores
constexpr int kRB = 32;   // Gaussians per LDS batch in the backward

// Sums of N values over each row of 16 lanes, returned to every lane of the row
// (quad_perm 1,0,3,2 and 2,3,0,1, then the 8- and 16-lane mirrors).  Every lane
// must be active.
template <int N>
__device__ __forceinline__ void row_sum_many(float (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0xB1>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x4E>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x141>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x140>(v[q]);
}

// The adjoint gives each thread kPPT pixels of the tile, (x, y + j 16 / kPPT), so the
// per-Gaussian row sums and their LDS traffic serve 16 kPPT pixels per lane row.
constexpr int kPPT = 2;
constexpr int kBwdThreads = 256 / kPPT;
constexpr int kBwdRows = kBwdThreads / 16;   // lane rows of 16 per block

template <int K>
__global__ __launch_bounds__(kBwdThreads) void raster_bwd_kernel(
    RasterArgs a, const float *__restrict__ T_final, const int *__restrict__ n_contrib,
    const int *__restrict__ topk_ids, const float *__restrict__ topk_w, const float *__restrict__ dL_dtopkw,
    const float *__restrict__ dL_dcolor, const float *__restrict__ dL_ddepth,
    const float *__restrict__ dL_dalpha, float *__restrict__ g_mean2d, float *__restrict__ g_conic,
    float *__restrict__ g_opac, float *__restrict__ g_rgb, float *__restrict__ g_depth) {
    __shared__ int s_id[kRB];
    __shared__ float2 s_xy[kRB];
    __shared__ float4 s_co[kRB];
    __shared__ float4 s_cz[kRB];
    __shared__ __align__(16) float s_part[kBwdRows][kRB][kNGP];   // [lane row][Gaussian][slot]
    __shared__ int s_max;
    const int ntiles = a.ntx * a.nty * a.views;
    const int tile = block_tile(a, ntiles);
    if (tile >= ntiles) return;
    const TilePos tp = tile_pos(a, tile);
    const int t = threadIdx.x;
    const int2 rg = a.ranges[tile];
    const int px = tp.x0 + (t & 15);
    const int py0 = tp.y0 + (t >> 4);

    // per-pixel state of the thread's kPPT pixels
    float fy[kPPT], T[kPPT], gC0[kPPT], gC1[kPPT], gC2[kPPT], gD[kPPT], gO[kPPT], A[kPPT];
    int last[kPPT];
    int ti[kPPT][K];
    float gam[kPPT][K];
    // A pixel's Top-K members are the Gaussians whose weight reached its smallest recorded
    // Top-K weight; the weights recomputed here differ from the recorded ones only by the
    // rounding of T (relative 3 n 2^-24 over a list of n), so only a Gaussian whose weight
    // passes wth (that smallest weight, over the slots with a nonzero dL/dw, less 1/64)
    // can be a member that adds a gamma term, and only then are its K ids compared.
    float wth[kPPT];
    const float fx = (float)px + 0.5f;
    int lmax = 0;
#pragma unroll
    for (int h = 0; h < kPPT; ++h) {
        const int py = py0 + (16 / kPPT) * h;
        fy[h] = (float)py + 0.5f;
        T[h] = 1.0f; gC0[h] = gC1[h] = gC2[h] = gD[h] = gO[h] = A[h] = 0.f;
        last[h] = 0;
        wth[h] = __builtin_inff();
#pragma unroll
        for (int k = 0; k < K; ++k) { ti[h][k] = -1; gam[h][k] = 0.f; }
        if (px < a.W && py < a.H) {
            const long p = tp.pix0 + (long)py * a.W + px;
            T[h] = T_final[p];
            last[h] = n_contrib[p];
            gC0[h] = dL_dcolor[3 * p];
            gC1[h] = dL_dcolor[3 * p + 1];
            gC2[h] = dL_dcolor[3 * p + 2];
            gD[h] = dL_ddepth[p];
            gO[h] = dL_dalpha ? dL_dalpha[p] : 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                ti[h][k] = topk_ids[p * K + k];
                gam[h][k] = dL_dtopkw ? dL_dtopkw[p * K + k] : 0.f;
                if (ti[h][k] >= 0 && gam[h][k] != 0.f) wth[h] = fminf(wth[h], topk_w[p * K + k]);
            }
            wth[h] *= 1.0f - 1.0f / 64.0f;
        }
    }
    if (t == 0) s_max = 0;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < kPPT; ++h) lmax = max(lmax, last[h]);
    atomicMax(&s_max, lmax);
    __syncthreads();
    const int maxl = s_max;
    for (int hi = maxl; hi > 0; hi -= kRB) {
        const int lo = hi > kRB ? hi - kRB : 0;
        const int cnt = hi - lo;
        __syncthreads();
        if (t < cnt) {
            const int r = a.sorted_ids[rg.x + lo + t];
            const int g = r - tp.rec0;
            s_id[t] = g;
            s_xy[t] = a.mean2d[r];
            s_co[t] = make_float4(a.conic[3 * r], a.conic[3 * r + 1], a.conic[3 * r + 2], a.opacity[r]);
            s_cz[t] = make_float4(a.rgb[3 * g], a.rgb[3 * g + 1], a.rgb[3 * g + 2], a.depth[r]);
        }
        __syncthreads();
        for (int j = cnt - 1; j >= 0; --j) {
            // -0 is the exact additive identity (x + -0 == x for every x, unlike +0), so the
            // first term of each sum costs no add; the sums (gradients, not replayed
            // decisions) are formed with fused multiply-adds
            float v[kNG];
#pragma unroll
            for (int q = 0; q < kNG; ++q) v[q] = -0.0f;
            bool hit = false;
            const float2 m = s_xy[j];
            const float4 co = s_co[j];
#pragma unroll
            for (int h = 0; h < kPPT; ++h) {
                if (lo + j >= last[h]) continue;
                float dx, dy, raw, ex;
                const float alpha = blend_alpha(fx, fy[h], m.x, m.y, co.x, co.y, co.z, co.w, dx, dy, raw, ex);
                if (alpha < kAlphaMin) continue;
                hit = true;
                const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
                T[h] *= r;                          // transmittance in front of this Gaussian
                const float w = alpha * T[h];
                const float4 cz = s_cz[j];
                float e = fmaf(gC0[h], cz.x, fmaf(gC1[h], cz.y, fmaf(gC2[h], cz.z, fmaf(gD[h], cz.w, gO[h]))));
                if (w >= wth[h]) {
                    const int g = s_id[j];
#pragma unroll
                    for (int k = 0; k < K; ++k) e += (ti[h][k] == g) ? gam[h][k] : 0.f;
                }
                const float dal = fmaf(T[h], e, -A[h] * r);
                A[h] = fmaf(e, w, A[h]);
                v[5] = fmaf(w, gC0[h], v[5]);
                v[6] = fmaf(w, gC1[h], v[6]);
                v[7] = fmaf(w, gC2[h], v[7]);
                v[8] = fmaf(w, gD[h], v[8]);
                if (raw <= kAlphaMax) {             // unclamped: alpha = o e^-sigma
                    const float ds = -alpha * dal;
                    const float hds = 0.5f * ds;
                    v[0] = fmaf(-ds, fmaf(co.x, dx, co.y * dy), v[0]);
                    v[1] = fmaf(-ds, fmaf(co.y, dx, co.z * dy), v[1]);
                    v[2] = fmaf(hds * dx, dx, v[2]);
                    v[3] = fmaf(ds * dx, dy, v[3]);
                    v[4] = fmaf(hds * dy, dy, v[4]);
                    v[9] = fmaf(dal, ex, v[9]);
                }
            }
            // sums over each lane row (16 lanes, 16 kPPT pixels; every lane takes part); the
            // row's first lane files them, and the row sums meet after the batch
            if (__ballot(hit) != 0ull) row_sum_many<kNG>(v);
            if ((t & 15) == 0) {
                float *dst = s_part[t >> 4][j];
                *(float4 *)dst = make_float4(v[0], v[1], v[2], v[3]);
                *(float4 *)(dst + 4) = make_float4(v[4], v[5], v[6], v[7]);
                *(float2 *)(dst + 8) = make_float2(v[8], v[9]);
            }
        }
        __syncthreads();
        // per Gaussian and slot: the row sums in a fixed order, one atomic
        for (int o = t; o < cnt * kNG; o += kBwdThreads) {
            const int j = o / kNG, q = o - j * kNG;
            float sum = 0.f;
#pragma unroll
            for (int r = 0; r < kBwdRows; ++r) sum += s_part[r][j][q];
            if (sum == 0.f) continue;
            const int g = s_id[j];          // Gaussian (colour) and record (screen-space) index
            const long r = (long)tp.rec0 + g;
            float *dst = q < 2 ? &g_mean2d[2 * r + q]
                       : q < 5 ? &g_conic[3 * r + (q - 2)]
                       : q < 8 ? &g_rgb[3 * g + (q - 5)]
                       : q == 8 ? &g_depth[r] : &g_opac[r];
            unsafeAtomicAdd(dst, sum);
        }
    }
}

// Pruning statistics of Sec. 3.3 for one view: every pixel adds one to the Top-K
// count of each Gaussian in its Top-K list, and every blended (pixel, Gaussian) pair
// raises that Gaussian's score S_i = max w (Eq. 5) to its weight.  The blend is replayed
// front to back up to n_contrib with the forward's own arithmetic, so each weight is
// bit-identical to the one the forward blended.  Per Gaussian the block takes a wave
// maximum (weights are >= 0, so the FP32 bits order like integers) and issues one
// atomic max per wave; the counts are gathered per wave and id first as well, so a
// Gaussian in many lists does not take one atomic per pixel.
template <int K>
__global__ __launch_bounds__(kFwdThreads) void prune_stats_kernel(RasterArgs a, const int *__restrict__ n_contrib,
                                                                  const int *__restrict__ topk_ids,
                                                                  int *__restrict__ topk_count,
                                                                  float *__restrict__ max_w) {
    __shared__ int s_id[256];
    __shared__ float2 s_xy[256];
    __shared__ float4 s_co[256];
    __shared__ int s_max;
    const int ntiles = a.ntx * a.nty * a.views;
    const int tile = block_tile(a, ntiles);
    if (tile >= ntiles) return;
    const TilePos tp = tile_pos(a, tile);
    const int t = threadIdx.x, lane = t & 63;
    const int px = tp.x0 + (t & 15);
    const int py0 = tp.y0 + (t >> 4);
    const float fx = (float)px + 0.5f;
    const int2 rg = a.ranges[tile];
    float fy[2], T[2];
    int last[2];
    if (t == 0) s_max = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int py = py0 + 8 * h;
        const bool valid = px < a.W && py < a.H;
        const long p = tp.pix0 + (long)py * a.W + px;
        fy[h] = (float)py + 0.5f;
        T[h] = 1.0f;
        last[h] = valid ? n_contrib[p] : 0;
        for (int k = 0; k < K; ++k) {
            int id = valid ? topk_ids[p * K + k] : -1;
            // one atomic per distinct id of the wave (the loop is uniform over the wave)
            while (true) {
                const uint64_t pend = __ballot(id >= 0);
                if (pend == 0ull) break;
                const int src = (int)__builtin_ctzll(pend);
                const int g = __builtin_amdgcn_readlane(id, src);
                const uint64_t same = __ballot(id == g);
                if (lane == src) atomicAdd(&topk_count[g], (int)__popcll(same));
                if (id == g) id = -1;
            }
        }
    }
    __syncthreads();
    atomicMax(&s_max, max(last[0], last[1]));
    __syncthreads();
    const int maxl = s_max;
    for (int base = 0; base < maxl; base += 256) {
        const int cnt = min(256, maxl - base);
        __syncthreads();
        for (int q = t; q < cnt; q += kFwdThreads) {
            const int r = a.sorted_ids[rg.x + base + q];
            s_id[q] = r - tp.rec0;
            s_xy[q] = a.mean2d[r];
            s_co[q] = make_float4(a.conic[3 * r], a.conic[3 * r + 1], a.conic[3 * r + 2], a.opacity[r]);
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float2 m = s_xy[j];
            const float4 co = s_co[j];
            float wm = 0.f;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (base + j >= last[h]) continue;
                float dx, dy, raw, ex;
                const float alpha = blend_alpha(fx, fy[h], m.x, m.y, co.x, co.y, co.z, co.w, dx, dy, raw, ex);
                if (alpha < kAlphaMin) continue;
                const float w = alpha * T[h];
                T[h] = T[h] * (1.0f - alpha);
                wm = fmaxf(wm, w);
            }
            // every lane takes part in the reduction
            if (__ballot(wm > 0.f) == 0ull) continue;
            wm = fmaxf(wm, dpp_mov<0xB1>(wm));
            wm = fmaxf(wm, dpp_mov<0x4E>(wm));
            wm = fmaxf(wm, dpp_mov<0x141>(wm));
            wm = fmaxf(wm, dpp_mov<0x140>(wm));
            const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wm), 0));
            const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wm), 16));
            const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wm), 32));
            const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wm), 48));
            const float wmax = fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
            if (lane == 0 && wmax > 0.f) atomicMax((int *)max_w + s_id[j], __float_as_int(wmax));
        }
    }
}

template <int K>
void launch_fwd(RasterArgs a, float *color, float *depth_map, float *alpha_map, float *T_final,
                int *n_contrib, int *topk_ids, float *topk_w, hipStream_t st) {
    hipLaunchKernelGGL(raster_fwd_kernel<K>, dim3(strip_grid((long long)a.ntx * a.nty * a.views)), dim3(kFwdThreads), 0,
                       st, a, color, depth_map, alpha_map, T_final, n_contrib, topk_ids, topk_w);
}

template <int K>
void launch_bwd(RasterArgs a, const float *T_final, const int *n_contrib, const int *topk_ids,
                const float *topk_w, const float *dL_dtopkw, const float *dL_dcolor, const float *dL_ddepth,
                const float *dL_dalpha, float *gm, float *gc, float *go, float *grgb, float *gz,
                hipStream_t st) {
    hipLaunchKernelGGL(raster_bwd_kernel<K>, dim3(strip_grid((long long)a.ntx * a.nty * a.views)), dim3(kBwdThreads), 0,
                       st, a, T_final, n_contrib, topk_ids, topk_w, dL_dtopkw, dL_dcolor, dL_ddepth, dL_dalpha,
                       gm, gc, go, grgb, gz);
}

template <int K>
void launch_prune(RasterArgs a, const int *n_contrib, const int *topk_ids, int *count, float *max_w, hipStream_t st) {
    hipLaunchKernelGGL(prune_stats_kernel<K>, dim3(strip_grid((long long)a.ntx * a.nty * a.views)), dim3(kFwdThreads), 0, st,
                       a, n_contrib, topk_ids, count, max_w);
}

#define LGS_K_SWITCH(k, CALL)            \
    switch (k) {                         \
    case 1: CALL(1); break;              \
    case 2: CALL(2); break;              \
    case 3: CALL(3); break;              \
    case 4: CALL(4); break;              \
    case 5: CALL(5); break;              \
    case 8: CALL(8); break;              \
    case 10: CALL(10); break;            \
    case 16: CALL(16); break;            \
    }

// The dispatch order of the tile kernels (lgs_tile_order).  Workgroups go to the XCDs
// in turn, so block b runs on XCD b % 8; the blocks of XCD x keep the tiles the fixed
// mapping gives that XCD (its L2 still holds their neighbours' records), reordered
// so that tiles with more pairs start first and the short ones fill the tail.  The
// weight is the tile's pair count in log-spaced buckets, eight per octave (a counting
// sort in LDS; the order inside a bucket is whatever the atomics give: the tile
// kernels' outputs do not depend on it).  One block per XCD.  weight: null for the
// pair counts, else one weight per tile (tile_weight_kernel).
constexpr int kOrderBins = 257;   // 256 weight buckets, heaviest first, then the padding slots
__global__ __launch_bounds__(1024) void tile_order_kernel(RasterArgs a, int grid, const int *__restrict__ weight,
                                                          int *__restrict__ order) {
    __shared__ int cnt[kOrderBins];
    __shared__ int off[kOrderBins];
    const int x = blockIdx.x, per = grid / 8, ntiles = a.ntx * a.nty * a.views;
    auto tile_of = [&](int i) {
        const int b = x + 8 * i;
        return a.bands ? xcd_remap(b, grid) : xcd_strips(b);
    };
    auto bin_of = [&](int tile) {
        if (tile >= ntiles) return kOrderBins - 1;
        int w;
        if (weight) {
            w = max(weight[tile], 0);
        } else {
            const int2 r = a.ranges[tile];
            w = max(r.y - r.x, 0);
        }
        return 255 - min(255, (int)(8.0f * __log2f((float)w + 1.0f)));
    };
    for (int i = threadIdx.x; i < kOrderBins; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < per; i += blockDim.x) atomicAdd(&cnt[bin_of(tile_of(i))], 1);
    __syncthreads();
    if (threadIdx.x < 64) {   // one wave scans the 256 weight bins, four per lane, then the padding bin
        const int l = threadIdx.x;
        const int c0 = cnt[4 * l], c1 = cnt[4 * l + 1], c2 = cnt[4 * l + 2], c3 = cnt[4 * l + 3];
        const int own = c0 + c1 + c2 + c3;
        int inc = own;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(inc, d);
            if (l >= d) inc += y;
        }
        const int ex = inc - own;
        off[4 * l] = ex;
        off[4 * l + 1] = ex + c0;
        off[4 * l + 2] = ex + c0 + c1;
        off[4 * l + 3] = ex + c0 + c1 + c2;
        if (l == 63) off[kOrderBins - 1] = inc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < per; i += blockDim.x) {
        const int t = tile_of(i);
        order[x + 8 * atomicAdd(&off[bin_of(t)], 1)] = t;
    }
}

// A tile's weight for the adjoint's order: the largest n_contrib over its pixels, the
// length of list its adjoint walks.  One 256-thread block per tile.
__global__ __launch_bounds__(256) void tile_weight_kernel(RasterArgs a, const int *__restrict__ n_contrib,
                                                          int *__restrict__ weight) {
    __shared__ int s_max[4];
    const TilePos tp = tile_pos(a, blockIdx.x);
    const int t = threadIdx.x, px = tp.x0 + (t & 15), py = tp.y0 + (t >> 4);
    int v = (px < a.W && py < a.H) ? n_contrib[tp.pix0 + (long)py * a.W + px] : 0;
    for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d));
    if ((t & 63) == 0) s_max[t >> 6] = v;
    __syncthreads();
    if (t == 0) weight[blockIdx.x] = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
}

// Checks the batched cameras (one image size) and fills the geometry part of RasterArgs.
lgs_status raster_args(const lgs_camera *cams, int views, int n, RasterArgs &a) {
    LGS_REQUIRE(cams, LGS_ERR_INVALID_ARG, "camera array is NULL");
    LGS_REQUIRE(views >= 1 && n >= 0, LGS_ERR_INVALID_ARG, "views = %d, n = %d", views, n);
    for (int v = 0; v < views; ++v) {
        lgs_status st = check_camera(&cams[v]);
        if (st) return st;
        LGS_REQUIRE(cams[v].width == cams[0].width && cams[v].height == cams[0].height, LGS_ERR_INVALID_ARG,
                    "batched views share the image size");
    }
    LGS_REQUIRE((long long)views * n <= 0x7FFFFFFF, LGS_ERR_INVALID_ARG, "too many records");
    a.W = cams[0].width;
    a.H = cams[0].height;
    a.ntx = tiles_x(a.W);
    a.nty = tiles_y(a.H);
    a.views = views;
    a.n = n;
    a.bands = views % 8 == 0;
    a.order = nullptr;
    return LGS_OK;
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_rasterize_topk_fwd_views(const lgs_camera *cams, int32_t views, int32_t k, int32_t n,
                                                   const float *mean2d, const float *conic, const float *opacity,
                                                   const float *rgb, const float *depth, const int32_t *sorted_ids,
                                                   const int32_t *tile_ranges, float *color, float *depth_map,
                                                   float *alpha_map, float *T_final, int32_t *n_contrib,
                                                   int32_t *topk_ids, float *topk_w, const int32_t *tile_order,
                                                   hipStream_t stream) {
    RasterArgs a;
    lgs_status st = raster_args(cams, views, n, a);
    if (st) return st;
    LGS_REQUIRE(k_supported(k), LGS_ERR_UNSUPPORTED, "K = %d is not compiled", k);
    LGS_REQUIRE(mean2d && conic && opacity && rgb && depth && sorted_ids && tile_ranges && color &&
                    depth_map && alpha_map && T_final && n_contrib && topk_ids && topk_w,
                LGS_ERR_INVALID_ARG, "lgs_rasterize_topk_fwd: NULL pointer");
    LGS_REQUIRE(((uintptr_t)mean2d & 7u) == 0 && ((uintptr_t)tile_ranges & 7u) == 0,
                LGS_ERR_INVALID_ARG, "mean2d and tile_ranges must be 8-byte aligned");
    a.mean2d = (const float2 *)mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.rgb = rgb;
    a.depth = depth;
    a.sorted_ids = sorted_ids;
    a.ranges = (const int2 *)tile_ranges;
    a.order = tile_order;
#define CALL_FWD(KK) launch_fwd<KK>(a, color, depth_map, alpha_map, T_final, n_contrib, topk_ids, topk_w, stream)
    LGS_K_SWITCH(k, CALL_FWD)
#undef CALL_FWD
    return check_launch("rasterize_topk_fwd");
}

extern "C" lgs_status lgs_rasterize_topk_fwd(const lgs_camera *cam, int32_t k, const float *mean2d,
                                             const float *conic, const float *opacity,
                                             const float *rgb, const float *depth,
                                             const int32_t *sorted_ids, const int32_t *tile_ranges,
                                             float *color, float *depth_map, float *alpha_map,
                                             float *T_final, int32_t *n_contrib, int32_t *topk_ids,
                                             float *topk_w, const int32_t *tile_order, hipStream_t stream) {
    // one view: the record of Gaussian g is g (n only splits views)
    return lgs_rasterize_topk_fwd_views(cam, 1, k, 0x7FFFFFFF, mean2d, conic, opacity, rgb, depth, sorted_ids,
                                        tile_ranges, color, depth_map, alpha_map, T_final, n_contrib, topk_ids,
                                        topk_w, tile_order, stream);
}

extern "C" lgs_status lgs_rasterize_topk_bwd_views(
    const lgs_camera *cams, int32_t views, int32_t k, int32_t n, const float *mean2d, const float *conic,
    const float *opacity, const float *rgb, const float *depth, const int32_t *sorted_ids,
    const int32_t *tile_ranges, const float *T_final, const int32_t *n_contrib, const int32_t *topk_ids,
    const float *topk_w, const float *dL_dcolor, const float *dL_ddepth, const float *dL_dalpha,
    const float *dL_dtopkw, float *dL_dmean2d, float *dL_dconic, float *dL_dopacity, float *dL_drgb,
    float *dL_ddepth_g, const int32_t *tile_order, hipStream_t stream) {
    RasterArgs a;
    lgs_status st = raster_args(cams, views, n, a);
    if (st) return st;
    LGS_REQUIRE(k_supported(k), LGS_ERR_UNSUPPORTED, "K = %d is not compiled", k);
    LGS_REQUIRE(mean2d && conic && opacity && rgb && depth && sorted_ids && tile_ranges && T_final &&
                    n_contrib && topk_ids && topk_w && dL_dcolor && dL_ddepth && dL_dmean2d &&
                    dL_dconic && dL_dopacity && dL_drgb && dL_ddepth_g,
                LGS_ERR_INVALID_ARG, "lgs_rasterize_topk_bwd: NULL pointer");
    LGS_REQUIRE(((uintptr_t)mean2d & 7u) == 0 && ((uintptr_t)tile_ranges & 7u) == 0,
                LGS_ERR_INVALID_ARG, "mean2d and tile_ranges must be 8-byte aligned");
    a.mean2d = (const float2 *)mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.rgb = rgb;
    a.depth = depth;
    a.sorted_ids = sorted_ids;
    a.ranges = (const int2 *)tile_ranges;
    a.order = tile_order;
#define CALL_BWD(KK)                                                                             \
    launch_bwd<KK>(a, T_final, n_contrib, topk_ids, topk_w, dL_dtopkw, dL_dcolor, dL_ddepth, dL_dalpha, \
                   dL_dmean2d, dL_dconic, dL_dopacity, dL_drgb, dL_ddepth_g, stream)
    LGS_K_SWITCH(k, CALL_BWD)
#undef CALL_BWD
    return check_launch("rasterize_topk_bwd");
}

extern "C" lgs_status lgs_rasterize_topk_bwd(
    const lgs_camera *cam, int32_t k, const float *mean2d, const float *conic, const float *opacity,
    const float *rgb, const float *depth, const int32_t *sorted_ids, const int32_t *tile_ranges,
    const float *T_final, const int32_t *n_contrib, const int32_t *topk_ids, const float *topk_w,
    const float *dL_dcolor, const float *dL_ddepth, const float *dL_dalpha, const float *dL_dtopkw,
    float *dL_dmean2d, float *dL_dconic, float *dL_dopacity, float *dL_drgb, float *dL_ddepth_g,
    const int32_t *tile_order, hipStream_t stream) {
    return lgs_rasterize_topk_bwd_views(cam, 1, k, 0x7FFFFFFF, mean2d, conic, opacity, rgb, depth, sorted_ids,
                                        tile_ranges, T_final, n_contrib, topk_ids, topk_w, dL_dcolor, dL_ddepth,
                                        dL_dalpha, dL_dtopkw, dL_dmean2d, dL_dconic, dL_dopacity, dL_drgb,
                                        dL_ddepth_g, tile_order, stream);
}

extern "C" lgs_status lgs_prune_stats_views(const lgs_camera *cams, int32_t views, int32_t k, int32_t n,
                                            const float *mean2d, const float *conic, const float *opacity,
                                            const int32_t *sorted_ids, const int32_t *tile_ranges,
                                            const int32_t *n_contrib, const int32_t *topk_ids, int32_t *topk_count,
                                            float *max_w, const int32_t *tile_order, hipStream_t stream) {
    RasterArgs a;
    lgs_status st = raster_args(cams, views, n, a);
    if (st) return st;
    LGS_REQUIRE(k_supported(k), LGS_ERR_UNSUPPORTED, "K = %d is not compiled", k);
    LGS_REQUIRE(mean2d && conic && opacity && sorted_ids && tile_ranges && n_contrib && topk_ids && topk_count &&
                    max_w,
                LGS_ERR_INVALID_ARG, "lgs_prune_stats: NULL pointer");
    LGS_REQUIRE(((uintptr_t)mean2d & 7u) == 0 && ((uintptr_t)tile_ranges & 7u) == 0 && ((uintptr_t)max_w & 3u) == 0,
                LGS_ERR_INVALID_ARG, "mean2d and tile_ranges must be 8-byte aligned, max_w 4-byte aligned");
    a.mean2d = (const float2 *)mean2d;
    a.conic = conic;
    a.opacity = opacity;
    a.rgb = nullptr;
    a.depth = nullptr;
    a.sorted_ids = sorted_ids;
    a.ranges = (const int2 *)tile_ranges;
    a.order = tile_order;
#define CALL_PRUNE(KK) launch_prune<KK>(a, n_contrib, topk_ids, topk_count, max_w, stream)
    LGS_K_SWITCH(k, CALL_PRUNE)
#undef CALL_PRUNE
    return check_launch("prune_stats");
}

extern "C" lgs_status lgs_prune_stats(const lgs_camera *cam, int32_t k, const float *mean2d, const float *conic,
                                      const float *opacity, const int32_t *sorted_ids,
                                      const int32_t *tile_ranges, const int32_t *n_contrib,
                                      const int32_t *topk_ids, int32_t *topk_count, float *max_w,
                                      const int32_t *tile_order, hipStream_t stream) {
    return lgs_prune_stats_views(cam, 1, k, 0x7FFFFFFF, mean2d, conic, opacity, sorted_ids, tile_ranges, n_contrib,
                                 topk_ids, topk_count, max_w, tile_order, stream);
}

// The order buffer: the grid's entries, then as many again for the tile weights.
extern "C" int64_t lgs_tile_order_size(int32_t width, int32_t height, int32_t views) {
    if (width <= 0 || height <= 0 || views <= 0) return 0;
    return 2ll * strip_grid((long long)tiles_x(width) * tiles_y(height) * views);
}

extern "C" lgs_status lgs_tile_order(const lgs_camera *cams, int32_t views, const int32_t *tile_ranges,
                                     const int32_t *n_contrib, int32_t *order, hipStream_t stream) {
    RasterArgs a;
    lgs_status st = raster_args(cams, views, 0, a);
    if (st) return st;
    LGS_REQUIRE(tile_ranges && order, LGS_ERR_INVALID_ARG, "lgs_tile_order: NULL pointer");
    LGS_REQUIRE(((uintptr_t)tile_ranges & 7u) == 0, LGS_ERR_INVALID_ARG, "tile_ranges must be 8-byte aligned");
    a.ranges = (const int2 *)tile_ranges;
    const long long grid = strip_grid((long long)a.ntx * a.nty * a.views);
    LGS_REQUIRE(grid % 8 == 0 && grid <= 0x7FFFFFFF, LGS_ERR_INVALID_ARG, "too many tiles");
    const int ntiles = a.ntx * a.nty * a.views;
    int *weight = nullptr;
    if (n_contrib) {
        weight = order + grid;
        hipLaunchKernelGGL(tile_weight_kernel, dim3(ntiles), dim3(256), 0, stream, a, n_contrib, weight);
    }
    hipLaunchKernelGGL(tile_order_kernel, dim3(8), dim3(1024), 0, stream, a, (int)grid, weight, order);
    return check_launch("tile_order");
}
