// Top-K feature rendering (Eq. 3-4, Sec. 3.2) and its adjoint: the device code and the
// launches, included by one compilation unit per Top-K size (feature_k*.hip) so the
// build spreads over several compiler processes.
//
// Every kernel takes one 256-thread block per 16x16 tile (views stacked).  The block
// first forms the union of the tile's Top-K ids (per-wave ballot dedupe, then a bounded
// LDS hash) and orders it by Gaussian id.
//
// MFMA path (BF16 or FP8 storage, BF16 map, K <= 8, unions of at most 32 Gaussians):
// the map and the adjoint are dense per-tile products on the matrix cores.  With Ft the
// union's rows and W the (renormalised) weights, F^T = Ft^T W^T, the dot products
// S^T = Ft G^T, and the gradient rows dFt = W^T G.  Each FP32 weight enters as a pair
// of BF16 terms (hi, lo), so every product is exact in the FP32 accumulator.  The
// channels are taken in slabs of at most 512 (one slab up to D = 512); per slab wave w
// owns a quarter of the slab's 32-channel chunks for all 256 pixels, so its gradient
// rows are complete when the slab ends and each (union row, channel) takes one atomic
// per tile.  Per tile row the weights pass through a three-buffer LDS ring (one
// barrier per row).
//
// Per-pixel path (FP32 storage or map, larger unions, K = 10 or 16): lanes across
// channels, 64 pixels per wave, rows staged in LDS when they fit; the adjoint sums
// w' dL/dF per wave-distinct Gaussian in registers and flushes with coalesced atomics.
//
// The adjoint has three modes: 0 reads a given dL/dF; 1 forms the L1 loss gradient
// from the recomputed map and a target; 2 does as 1 and also stores the map, so the
// render and its adjoint take one pass.
#pragma once

#include <algorithm>
#include <type_traits>

#include "feature_launch.hpp"
#include "lgs_device.hpp"
#include "lgs_host.hpp"
#include "tile_map.hpp"

namespace lgs {
namespace {



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

// ---------------------------------------------------------------- tile union

// Both feature kernels give one 16x16 tile to a 256-thread block.  Wave w owns the
// tile's rows 4w..4w+3 (64 pixels) and streams them one pixel at a time with lanes
// across channels (CPL consecutive channels per lane per pass).
//
// Prologue: lane i loads the Top-K slots of the wave's pixel i.  The wave lists its
// distinct Gaussian ids with a ballot loop (one iteration per distinct id, no
// contention), the four wave lists merge through a small LDS hash table into the
// tile's union, and the union's feature rows are staged once into LDS (at most
// `ucap` of them; rare larger unions read the rest from global memory).  The forward
// then builds each pixel's row from LDS and writes it; the backward adds w'_k dL/dF
// into per-wave register accumulators indexed by the wave-local id index, and adds
// each accumulator to dL/df once, with coalesced atomics.
constexpr int kFB = 256;          // threads per feature block
constexpr int kPixPerWave = 64;
constexpr int kUP = 32;           // union rows of the MFMA path (two 16-row blocks)
constexpr int kUP2 = 64;          // ... and of its large-union form (four blocks; K > 4 only)
constexpr int kCPW = 4;           // 32-channel chunks per wave and channel slab on the MFMA path
constexpr int kSlabCh = 4 * 32 * kCPW;   // channels of one slab: D above this takes several slabs
constexpr int kRowBudget = 32 * 1024;   // LDS bytes for staged rows on the per-pixel path

template <int K> struct TileCfg {
    static constexpr int CPL = K <= 4 ? 8 : (K <= 8 ? 4 : 2);   // channels per lane per pass
    static constexpr int RA = K <= 4 ? 12 : (K <= 8 ? 16 : 24);  // register accumulators per wave
    static constexpr int HS = 256;   // union hash slots: dedups any tile of up to 128 wave-distinct ids
};

template <int FT> struct Bytes { static constexpr int v = FT == FT_F32 ? 4 : FT == FT_BF16 ? 2 : 1; };

// CPL consecutive values (storage format FT) starting at element index `at`.
template <int FT, int CPL>
__device__ __forceinline__ void loadc(const void *__restrict__ base, long at, float (&v)[CPL]) {
    if constexpr (FT == FT_F32) {
        const float *p = (const float *)base + at;
        if constexpr (CPL == 8) {
            f32x4 a = ((const f32x4 *)p)[0], b = ((const f32x4 *)p)[1];
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else if constexpr (CPL == 4) {
            f32x4 a = *(const f32x4 *)p;
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        } else {
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            f32x2 a = *(const f32x2 *)p;
            v[0] = a.x; v[1] = a.y;
        }
    } else if constexpr (FT == FT_BF16) {
        const uint16_t *p = (const uint16_t *)base + at;
        if constexpr (CPL == 8) {
            u32x4 a = *(const u32x4 *)p;
            uint32_t w4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) { v[2 * i] = bf16_to_f32(w4[i] & 0xFFFFu); v[2 * i + 1] = bf16_to_f32(w4[i] >> 16); }
        } else if constexpr (CPL == 4) {
            u32x2 a = *(const u32x2 *)p;
            v[0] = bf16_to_f32(a.x & 0xFFFFu); v[1] = bf16_to_f32(a.x >> 16);
            v[2] = bf16_to_f32(a.y & 0xFFFFu); v[3] = bf16_to_f32(a.y >> 16);
        } else {
            uint32_t a = *(const uint32_t *)p;
            v[0] = bf16_to_f32(a & 0xFFFFu); v[1] = bf16_to_f32(a >> 16);
        }
    } else {
        const uint8_t *p = (const uint8_t *)base + at;
        if constexpr (CPL == 8) {
            u32x2 a = *(const u32x2 *)p;
#pragma unroll
            for (int i = 0; i < 4; ++i) { v[i] = e4m3_to_f32((a.x >> (8 * i)) & 0xFFu); v[4 + i] = e4m3_to_f32((a.y >> (8 * i)) & 0xFFu); }
        } else if constexpr (CPL == 4) {
            uint32_t a = *(const uint32_t *)p;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = e4m3_to_f32((a >> (8 * i)) & 0xFFu);
        } else {
            uint32_t a = *(const uint16_t *)p;
            v[0] = e4m3_to_f32(a & 0xFFu); v[1] = e4m3_to_f32(a >> 8);
        }
    }
}

template <int MT, int CPL>
__device__ __forceinline__ void storec(void *__restrict__ base, long at, const float (&v)[CPL]) {
    if constexpr (MT == MT_F32) {
        float *p = (float *)base + at;
        if constexpr (CPL == 8) {
            f32x4 a = {v[0], v[1], v[2], v[3]}, b = {v[4], v[5], v[6], v[7]};
            __builtin_nontemporal_store(a, (f32x4 *)p);
            __builtin_nontemporal_store(b, (f32x4 *)p + 1);
        } else if constexpr (CPL == 4) {
            f32x4 a = {v[0], v[1], v[2], v[3]};
            __builtin_nontemporal_store(a, (f32x4 *)p);
        } else {
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            f32x2 a = {v[0], v[1]};
            __builtin_nontemporal_store(a, (f32x2 *)p);
        }
    } else {
        uint16_t *p = (uint16_t *)base + at;
        uint32_t w[CPL / 2];
#pragma unroll
        for (int i = 0; i < CPL / 2; ++i)
            w[i] = (uint32_t)f32_to_bf16(v[2 * i]) | ((uint32_t)f32_to_bf16(v[2 * i + 1]) << 16);
        if constexpr (CPL == 8) {
            u32x4 a = {w[0], w[1], w[2], w[3]};
            __builtin_nontemporal_store(a, (u32x4 *)p);
        } else if constexpr (CPL == 4) {
            u32x2 a = {w[0], w[1]};
            __builtin_nontemporal_store(a, (u32x2 *)p);
        } else {
            __builtin_nontemporal_store(w[0], (uint32_t *)p);
        }
    }
}

__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

struct TileGeom {
    int view, tx0, ty0;
};

__device__ __forceinline__ TileGeom tile_geom(int tile, int W, int H) {
    const int ntx = (W + kTile - 1) / kTile, nty = (H + kTile - 1) / kTile;
    TileGeom g;
    g.view = tile / (ntx * nty);
    int tv = tile - g.view * ntx * nty;
    g.tx0 = (tv % ntx) * kTile;
    g.ty0 = (tv / ntx) * kTile;
    return g;
}

// Per-lane state after the prologue: the lane's pixel slots and, for each slot, the
// wave-local index of its Gaussian.
template <int K>
struct Slots {
    int id[K];
    int wl[K];     // wave-local index of the slot's Gaussian (-1: empty)
    int u[K];      // tile union index (-1: empty)
    float wp[K];   // renormalised weight w'_k
    float wf[K];   // weight applied to the stored row: w'_k, times the row scale for FP8
    float W;
};

// The tile's union, at the start of the dynamic LDS.  The first fields live for the
// whole tile; the rest (the hash, the wave lists, the union in hash order) serve the
// union's construction and the per-pixel path, and on the MFMA path they are dead once
// the union is ordered, so the MFMA buffers overlay them (union_keep_bytes).
template <int K, int FT>
struct UnionLds {
    int nw[4];
    int nU;
    // MFMA path (U <= kUP): the union in ascending id order, so both feature
    // kernels order the K dimension of their products identically
    int rank[kUP2];      // hash-order union index -> ascending-id index
    int uid2[kUP2];      // ascending-id index -> Gaussian id
    float uscale2[FT == FT_FP8 ? kUP2 : 1];  // ascending-id index -> FP8 row scale
    // construction and per-pixel path
    int hkey[TileCfg<K>::HS];
    int hval[TileCfg<K>::HS];
    int wlist[4][kPixPerWave * K];   // wave-local distinct ids
    int16_t wmap[4][kPixPerWave * K];   // wave-local index -> tile union index (< 4 * 64 K)
    int uid[4 * kPixPerWave * K];    // tile union index -> Gaussian id
    float uscale[FT == FT_FP8 ? 4 * kPixPerWave * K : 1];  // tile union index -> FP8 row scale
};
// Bytes of the union that outlive its ordering (where the MFMA buffers start), and of
// the whole union (where the per-pixel path's buffers start).
template <int K, int FT>
constexpr size_t union_keep_bytes() {
    using UL = UnionLds<K, FT>;
    return (__builtin_offsetof(UL, hkey) + 15) & ~(size_t)15;
}
template <int K, int FT>
constexpr size_t union_bytes() { return (sizeof(UnionLds<K, FT>) + 15) & ~(size_t)15; }

// Builds the tile union: L.uid[0, U) and, per lane, the slots' union indices.
// Returns the wave's number of distinct ids.
template <int K, int FT>
__device__ __forceinline__ int tile_union(const TileGeom &tg, int W, int H,
                                          const int *__restrict__ ids, const float *__restrict__ tw,
                                          const float *__restrict__ scale, UnionLds<K, FT> &L,
                                          Slots<K> &s, int &U) {
    constexpr int HS = TileCfg<K>::HS;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int x = tg.tx0 + (lane & 15), y = tg.ty0 + wave * 4 + (lane >> 4);
    const bool valid = x < W && y < H;
    const long p = (long)tg.view * W * H + (long)y * W + x;
    float wv[K];
    s.W = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s.id[k] = valid ? ids[p * K + k] : -1;
        wv[k] = valid ? tw[p * K + k] : 0.f;
        s.W += wv[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s.wp[k] = (s.W > 0.f && s.id[k] >= 0) ? wv[k] / s.W : 0.f;
        if (!(s.W > 0.f)) s.id[k] = -1;
        s.wl[k] = -1;
    }
    for (int h = t; h < HS; h += kFB) L.hkey[h] = -1;
    if (t == 0) L.nU = 0;
    // distinct ids of the wave: each iteration takes the first pending slot's id and
    // resolves every slot of every lane that holds it
    int nw = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        while (true) {
            const uint64_t m = __ballot(s.wl[k] < 0 && s.id[k] >= 0);
            if (m == 0ull) break;
            const int lid = rdlane(s.id[k], (int)__builtin_ctzll(m));
#pragma unroll
            for (int k2 = k; k2 < K; ++k2) s.wl[k2] = (s.id[k2] == lid) ? nw : s.wl[k2];
            if (lane == 0) L.wlist[wave][nw] = lid;
            ++nw;
        }
    }
    if (lane == 0) L.nw[wave] = nw;
    __syncthreads();
    const int ntot = L.nw[0] + L.nw[1] + L.nw[2] + L.nw[3];
    if (ntot <= HS / 2) {
        // merge the four lists through the hash table (at most half full, so every
        // probe sequence ends): one dense index per distinct id
        for (int j = lane; j < nw; j += 64) {
            const int g = L.wlist[wave][j];
            uint32_t h = ((uint32_t)g * 2654435761u) & (HS - 1);
            for (int probe = 0; probe < HS; ++probe) {
                const int prev = atomicCAS(&L.hkey[h], -1, g);
                if (prev == -1) {
                    const int u = atomicAdd(&L.nU, 1);
                    L.uid[u] = g;
                    if constexpr (FT == FT_FP8) L.uscale[u] = scale[g];
                    L.hval[h] = u;
                    break;
                }
                if (prev == g) break;
                h = (h + 1) & (HS - 1);
            }
        }
        __syncthreads();
        for (int j = lane; j < nw; j += 64) {
            const int g = L.wlist[wave][j];
            uint32_t h = ((uint32_t)g * 2654435761u) & (HS - 1);
            for (int probe = 0; probe < HS && L.hkey[h] != g; ++probe) h = (h + 1) & (HS - 1);
            L.wmap[wave][j] = (int16_t)L.hval[h];
        }
    } else {
        // very large unions: concatenate the wave lists (a Gaussian seen by several
        // waves gets several rows; only the staging budget notices)
        int off = 0;
        for (int w2 = 0; w2 < wave; ++w2) off += L.nw[w2];
        for (int j = lane; j < nw; j += 64) {
            const int g = L.wlist[wave][j];
            L.uid[off + j] = g;
            if constexpr (FT == FT_FP8) L.uscale[off + j] = scale[g];
            L.wmap[wave][j] = (int16_t)(off + j);
        }
        if (t == 0) L.nU = ntot;
        __syncthreads();
    }
    U = L.nU;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s.u[k] = s.wl[k] >= 0 ? L.wmap[wave][s.wl[k]] : -1;
        s.wf[k] = s.wp[k];
        if constexpr (FT == FT_FP8) s.wf[k] = s.u[k] >= 0 ? s.wp[k] * L.uscale[s.u[k]] : 0.f;
    }
    __syncthreads();   // wmap has been read: its space may be reused
    return nw;
}

// The per-pixel path walks the channels in passes of 64 CPL (one value per lane and
// channel group); per pass it stages the first min(U, ucap) union rows' channels of that
// pass, in their storage format, into `rows` = [ucap][64 CPL]: 16-byte pieces (8-byte
// for FP8 rows).  Staging a pass rather than whole rows lets the same LDS hold 2-4x the
// rows, so large unions rarely fall back to global reads.  All threads take part; the
// barriers around it keep the previous pass's readers and the next pass's writers apart.
template <int K> constexpr int pass_ch() { return 64 * TileCfg<K>::CPL; }

template <int K, int FT>
__device__ __forceinline__ void stage_pass(const UnionLds<K, FT> &L, int U, int D, int ucap, int pass,
                                           const void *__restrict__ feat, unsigned char *rows) {
    typedef typename std::conditional<FT == FT_FP8, u32x2, u32x4>::type piece;
    constexpr int PW = pass_ch<K>();
    constexpr int per = (int)sizeof(piece) / Bytes<FT>::v;   // channels per piece (8, or 4 in FP32)
    const int cb = pass * PW;
    const int pieces = (min(D, cb + PW) - cb) / per;
    const int nr = min(U, ucap);
    __syncthreads();
    for (int q = threadIdx.x; q < nr * pieces; q += kFB) {
        const int r = q / pieces, c = q - r * pieces;
        const piece *src = (const piece *)((const unsigned char *)feat + ((long)L.uid[r] * D + cb) * Bytes<FT>::v) + c;
        ((piece *)(rows + (long)r * PW * Bytes<FT>::v))[c] = *src;
    }
    __syncthreads();
}

// CPL values of union row u at channel c0 of pass `pass`: from LDS (staged) or global memory.
template <int K, int FT, int CPL>
__device__ __forceinline__ void urow(const unsigned char *rows, int ucap, const int *uid, int u, int pass,
                                     const void *__restrict__ feat, int D, int c0, float (&v)[CPL]) {
    if (u < ucap) loadc<FT, CPL>(rows, (long)u * pass_ch<K>() + c0 - pass * pass_ch<K>(), v);
    else loadc<FT, CPL>(feat, (long)uid[u] * D + c0, v);
}

template <int CPL>
__device__ __forceinline__ void flush_row(const float (&a)[CPL], int g, int D, int pass_c0, int lane,
                                          float *__restrict__ dfeat, float *xbuf) {
    // transpose through wave-private LDS so each atomic instruction covers 64
    // consecutive channels
#pragma unroll
    for (int j = 0; j < CPL; ++j) xbuf[lane * CPL + j] = a[j];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float *dst = dfeat + (long)g * D + pass_c0;
    const int span = min(64 * CPL, D - pass_c0);
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int c = j * 64 + lane;
        const float v = xbuf[c];
        if (c < span && v != 0.f) unsafeAtomicAdd(&dst[c], v);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- MFMA tile path
//
// Tiles whose Top-K union has at most kUP Gaussians (BF16 or FP8 storage, BF16 map)
// run both feature kernels as dense per-tile products on the matrix cores:
//   F^T[c][p]  = sum_u Ft[u][c] Wa[p][u]         the feature map (Eq. 4), and its L1 recompute
//   S^T[u][p] += sum_c Ft[u][c] G[p][c]          the dot products g_k = <dL/dF, f_k>
//   dFt[u][c] += sum_p Wd[p][u] G[p][c]          the feature gradient rows sum_p w'_k dL/dF
// Ft holds the union's stored rows (FP8 codes widened to BF16, exactly), Wa the
// renormalised weights w'_k (times the FP8 row scale), Wd the weights w'_k; each is
// zero outside the pixel's K slots.  An FP32 weight w enters as two BF16 terms
// hi = RNE(w), lo = RNE(w - hi), i.e. with 16 significant bits, and every product is
// exact in the FP32 accumulator.
//
// Operand layouts (lane l = 16 g + i): v_mfma_f32_16x16x16_bf16 takes A[i][4g..4g+3]
// and B[4g..4g+3][i]; v_mfma_f32_16x16x32_bf16 takes A[i][8g..8g+7] and
// B[8g..8g+7][i]; both return D[4g..4g+3][i].
//
// Work split: wave w owns a contiguous range of 32-channel chunks for all 256
// pixels of the tile, so its Ft operands stay in registers for the whole tile and
// its gradient rows are complete when the tile ends (one atomic per element and
// tile).  The tile's 16 pixel rows are the MFMA column blocks, processed in turn;
// per row the weights are scattered into a per-wave LDS buffer and read back in
// operand layout.  Within a chunk, channel block b (of two) row m stands for
// channel 8 (m / 4) + 4 b + m % 4, so that after both blocks lane (i, g) holds the
// eight consecutive channels 8g..8g+7 of pixel i: one 16-byte access per lane.
// Partial dot products of the four waves meet in LDS and are summed in a fixed
// order, so dL/dw is deterministic.

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats to packed BF16, round to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    bf16x2_t r = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ uint16_t bits_bf16(float a) { return __builtin_bit_cast(uint16_t, (__bf16)a); }
__device__ __forceinline__ i16x4 as_op4(u32x2 v) { return __builtin_bit_cast(i16x4, v); }
__device__ __forceinline__ i16x8 as_op8(u32x4 v) { return __builtin_bit_cast(i16x8, v); }
__device__ __forceinline__ f32x4 mfma16(i16x4 a, i16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(i16x8 a, i16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(__bf16 __attribute__((ext_vector_type(8))), a),
                                                   __builtin_bit_cast(__bf16 __attribute__((ext_vector_type(8))), b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// Channel of block b, row m within a 32-channel chunk.
__device__ __forceinline__ int blk_ch(int b, int m) { return 8 * (m >> 2) + 4 * b + (m & 3); }

// Weights of one tile row in operand-ready layout, shared by the block's four waves:
// a ring of three such buffers lets one row be read while the next is scattered and
// the one after is cleared, with a single block barrier per row.  NUB union blocks of
// 16 (2, or 4 for the large-union form).  Row strides are padded so that the 16 lanes
// of a read group, which take the same offset in consecutive rows, fall on distinct
// banks (wa: 72 or 136 bytes; wd: 48 bytes with two blocks, unpadded with four, where
// the LDS it would take is needed more).
template <int NUB>
struct MfRingF {
    static constexpr bool WD = false;
    uint16_t wa[2][16][16 * NUB + 4];   // [hi, lo][pixel of the row][union index]
};
template <int NUB>
struct MfRingB {
    static constexpr bool WD = true;
    uint16_t wa[2][16][16 * NUB + 4];
    uint16_t wd[2][16 * NUB][NUB == 2 ? 24 : 16];   // [hi, lo][union index][pixel of the row]
};
// Per-wave LDS: the forward's map row for the wave's channels (16-byte columns
// XOR-swizzled by pixel, so neither the writes nor the reads collide on banks), the
// backward's G of the row's chunks, transposed.
struct MfWaveF {
    uint16_t out[16][128];
};
struct MfWaveB {
    uint16_t gt[kCPW][2][16][16];       // [chunk][channel block][block row][pixel]
};
static_assert(sizeof(MfRingF<2>) % 16 == 0 && sizeof(MfRingB<2>) % 16 == 0 && sizeof(MfRingF<4>) % 16 == 0 &&
                  sizeof(MfRingB<4>) % 16 == 0,
              "ring buffers in 16-byte pieces");
static_assert(sizeof(MfWaveF) == 4096 && sizeof(MfWaveB) == 4096, "wave buffer layout");
// row stride (floats) of the backward's S^T rows: 20 with two union blocks, so the four
// lane groups of a store fall on distinct banks; 16 with four, to fit the wave buffer
template <int NUB> constexpr int sp_stride() { return NUB == 2 ? 20 : 16; }
static_assert(kUP * sp_stride<2>() * 4 <= (int)sizeof(MfWaveB) && kUP2 * sp_stride<4>() * 4 <= (int)sizeof(MfWaveB),
              "S^T rows fit the wave buffer");
// union blocks of the largest MFMA form a kernel of this K runs
__host__ __device__ constexpr int mf_nub_max(int K) { return K > 4 ? 4 : 2; }

// Dynamic LDS of the MFMA path.  Backward: the waves' partial dot products first,
// then the slot table (per pixel and slot: union index, Wa weight, Wd weight), the
// weight ring and the four per-wave buffers.  Forward: the slot table, the ring and
// the wave buffers.  While a channel slab's operands are loaded, half of the union
// rows are staged as BF16 ([16][slab channels], at most 16 KB) over the ring and the
// wave buffers, which are idle then.  Up to K = 4 the partial dot products are kept
// for the whole tile ([4][256][K]) and the slot table holds 32-bit indices and both
// weights.  Above K = 4, to stay at two blocks per CU, the partials of the last two
// rows ([2][4][16][K]) are summed row by row into the tile's dot products ([256][K]),
// and the slot table holds 16-bit indices and, without FP8 row scales (Wa = Wd), one
// weight.
__host__ __device__ inline size_t mf_align(size_t a) { return (a + 15) & ~(size_t)15; }
__host__ __device__ constexpr bool mf_compact(int K) { return K > 4; }
__host__ __device__ inline size_t mf_partials_bytes(int K) {
    return mf_align(mf_compact(K) ? (size_t)(2 * 4 * 16 + kTilePix) * K * 4 : (size_t)4 * kTilePix * K * 4);
}
__host__ __device__ inline size_t mf_slots_bytes(int K, bool fp8) {
    if (!mf_compact(K)) return (size_t)3 * kTilePix * K * 4;
    return mf_align((size_t)kTilePix * K * (2 + 4 * (fp8 ? 2 : 1)));
}
__host__ __device__ inline size_t mf_slots_at(int K, bool bwd) { return bwd ? mf_partials_bytes(K) : 0; }
__host__ __device__ inline size_t mf_ring_at(int K, bool bwd, bool fp8) {
    return mf_slots_at(K, bwd) + mf_slots_bytes(K, fp8);
}
__host__ __device__ inline size_t mf_ring_bytes(int K, bool bwd) {
    return mf_nub_max(K) == 4 ? (bwd ? sizeof(MfRingB<4>) : sizeof(MfRingF<4>))
                              : (bwd ? sizeof(MfRingB<2>) : sizeof(MfRingF<2>));
}
__host__ __device__ inline size_t mf_waves_at(int K, bool bwd, bool fp8) {
    return mf_ring_at(K, bwd, fp8) + 3 * mf_ring_bytes(K, bwd);
}
__host__ __device__ inline size_t mf_lds_bytes(int K, bool bwd, bool fp8) {
    return mf_waves_at(K, bwd, fp8) + 4 * (bwd ? sizeof(MfWaveB) : sizeof(MfWaveF));
}
// the staged rows of a slab fit over the ring and the wave buffers
static_assert(3 * sizeof(MfRingF<2>) + 4 * sizeof(MfWaveF) >= 16 * kSlabCh * 2, "staging area (forward)");
static_assert(3 * sizeof(MfRingB<2>) + 4 * sizeof(MfWaveB) >= 16 * kSlabCh * 2, "staging area (backward)");

template <int K>
struct SlotTable {
    typename std::conditional<mf_compact(K), int16_t, int>::type *u;
    float *wa, *wd;
};
template <int K, bool FP8>
__device__ __forceinline__ SlotTable<K> slot_table(unsigned char *dyn, bool bwd) {
    SlotTable<K> st;
    float *w = (float *)(dyn + mf_slots_at(K, bwd));
    if constexpr (mf_compact(K)) {
        st.wa = w;
        st.wd = FP8 ? w + kTilePix * K : w;
        st.u = (int16_t *)(w + kTilePix * K * (FP8 ? 2 : 1));
    } else {
        st.u = (int *)w;
        st.wa = w + kTilePix * K;
        st.wd = st.wa + kTilePix * K;
    }
    return st;
}

// Prologue of the MFMA path (all 256 threads; U <= kUP2): orders the union by id.
template <int K, int FT>
__device__ __forceinline__ void mf_prologue(UnionLds<K, FT> &L, Slots<K> &s, int U) {
    const int t = threadIdx.x;
    static_assert(4 * kUP2 <= kFB, "four threads per member");
    {   // four threads per member (whole waves, so the shuffles see every lane)
        const int u = t >> 2, q = t & 3;
        const int g = u < U ? L.uid[u] : 0;
        int r = 0;
        for (int v = q; v < U; v += 4) r += L.uid[v] < g ? 1 : 0;   // ids are distinct
        r += __shfl_xor(r, 1);
        r += __shfl_xor(r, 2);
        if (u < U && q == 0) {
            L.rank[u] = r;
            L.uid2[r] = g;
            if constexpr (FT == FT_FP8) L.uscale2[r] = L.uscale[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) s.u[k] = s.u[k] >= 0 ? L.rank[s.u[k]] : -1;
}

// Storage and map formats on the MFMA path.  BF16 rows (and FP8 codes, widened
// exactly) are one BF16 operand; an FP32 row value f is the exact sum of three BF16
// terms t0 = RNE(f), t1 = RNE(f - t0), t2 = f - t0 - t1 (exact for |f| above about
// 2^-100; below, the absolute error is under 2^-133), each multiplied in turn.  With
// three terms or an FP32 map a wave holds two 32-channel chunks per slab instead of
// four, so the operands and the FP32 target rows fit the register budget.
template <int FT, int MT, int NUB = 2>
struct MfForm {
    static constexpr int NT = FT == FT_F32 ? 3 : 1;        // BF16 terms per stored value
    static constexpr bool M32 = MT == MT_F32;              // FP32 map (and target)
    // chunks per wave and slab; the large-union form (four union blocks, rare tiles)
    // holds one, so that its registers stay well below the common form's
    static constexpr int CPW = NUB == 4 ? 1 : ((NT == 3 || M32) ? 2 : 4);
    static_assert(CPW >= 1 && CPW <= kCPW, "wave buffers sized for kCPW chunks");
};

// Channel slabs: the ceil(D / 32) chunks are split into ceil(chunks / (4 CPW)) slabs
// of near-equal size (at most 4 CPW chunks); a tile runs its row loop once per slab
// with that slab's operands in registers.
struct MfSlab {
    int c0, n;   // first chunk, chunk count
};
__device__ __forceinline__ int mf_nslabs(int D, int per_slab) {
    return (((D + 31) >> 5) + per_slab - 1) / per_slab;
}
__device__ __forceinline__ MfSlab mf_slab(int D, int ns, int sl) {
    const int nch = (D + 31) >> 5, per = (nch + ns - 1) / ns;
    MfSlab m;
    m.c0 = sl * per;
    m.n = min(per, nch - m.c0);
    return m;
}

// Stages union rows 16 h .. 16 h + 15 (those below U), channels of the slab, into
// ft = [16][32 slab.n]: BF16 (FP8 codes widened exactly), or FP32 as stored.
template <int K, int FT>
__device__ __forceinline__ void mf_stage_half(const UnionLds<K, FT> &L, int U, int D, int h, const MfSlab &sb,
                                              const void *__restrict__ feat, void *ft) {
    const int cb = sb.c0 * 32, ds = sb.n * 32;
    const int c8 = (min(D, cb + ds) - cb) >> 3;
    const int nr = min(16, U - 16 * h);
    for (int q = threadIdx.x; q < nr * c8; q += kFB) {
        const int r = q / c8, c = (q - r * c8) * 8;
        const long src = (long)L.uid2[16 * h + r] * D + cb + c;
        if constexpr (FT == FT_F32) {
            const u32x4 *a = (const u32x4 *)((const float *)feat + src);
            u32x4 *d = (u32x4 *)((float *)ft + r * ds + c);
            d[0] = a[0];
            d[1] = a[1];
        } else {
            u32x4 o;
            if constexpr (FT == FT_BF16) {
                o = *(const u32x4 *)((const uint16_t *)feat + src);
            } else {
                const u32x2 a = *(const u32x2 *)((const uint8_t *)feat + src);
                float v[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = e4m3_to_f32((a.x >> (8 * i)) & 0xFFu);
                    v[4 + i] = e4m3_to_f32((a.y >> (8 * i)) & 0xFFu);
                }
                o.x = pk_bf16(v[0], v[1]); o.y = pk_bf16(v[2], v[3]);
                o.z = pk_bf16(v[4], v[5]); o.w = pk_bf16(v[6], v[7]);
            }
            *(u32x4 *)((uint16_t *)ft + r * ds + c) = o;
        }
    }
}

// The wave's chunks of the slab: [beg, beg + n) of the ceil(D / 32) chunks.
struct MfChunks {
    int beg, n;
};
__device__ __forceinline__ MfChunks mf_chunks(const MfSlab &sb, int wave) {
    const int cpw = (sb.n + 3) >> 2;
    MfChunks m;
    m.beg = sb.c0 + wave * cpw;
    m.n = max(0, min(cpw, sb.n - wave * cpw));
    return m;
}

// The three BF16 terms of an FP32 value (see MfForm).
__device__ __forceinline__ void split3(float v, short &t0, short &t1, short &t2) {
    const uint16_t a = bits_bf16(v);
    const float r = v - bf16_to_f32(a);
    const uint16_t b = bits_bf16(r);
    t0 = (short)a;
    t1 = (short)b;
    t2 = (short)bits_bf16(r - bf16_to_f32(b));
}

// Register operands of union block h (rows 16 h .. 16 h + 15, staged in ft), zero
// outside the union and past D; term t of NT:
//   opA[t][i][b][h]: lane (i16, g) = Ft[16 h + 4 g + j][chunk + blk_ch(b, i16)], j < 4
//   opC[t][i][h]:    lane (i16, g) = Ft[16 h + i16][chunk + 8 g + j], j < 8
template <int FT, int NT, int CPW, int NUB>
__device__ __forceinline__ void mf_load_ops(const void *ft, int U, int D, int h, const MfSlab &sb,
                                            const MfChunks &mc, int lane, i16x4 (&opA)[NT][CPW][2][NUB],
                                            i16x8 (&opC)[NT][CPW][NUB]) {
    const int i16 = lane & 15, g = lane >> 4;
    const int nr = U - 16 * h;   // staged rows of this block
    const int cb = sb.c0 * 32, ds = sb.n * 32;
    const uint16_t *fb = (const uint16_t *)ft;
    const float *ff = (const float *)ft;
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
        const int c0 = (mc.beg + i) * 32;
        const bool on = i < mc.n;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            i16x4 a[NT];
            const int ch = c0 + blk_ch(b, i16);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * g + j;
                const bool in = on && r < nr && ch < D;
                if constexpr (NT == 1) {
                    a[0][j] = in ? (short)fb[r * ds + ch - cb] : (short)0;
                } else {
                    short t0, t1, t2;
                    split3(in ? ff[r * ds + ch - cb] : 0.f, t0, t1, t2);
                    a[0][j] = t0;
                    a[1][j] = t1;
                    a[2][j] = t2;
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) opA[t][i][b][h] = a[t];
        }
        const int ch = c0 + 8 * g;
        const bool in = on && i16 < nr && ch < D;
        if constexpr (NT == 1) {
            u32x4 v = {0u, 0u, 0u, 0u};
            if (in) v = *(const u32x4 *)(fb + i16 * ds + ch - cb);
            opC[0][i][h] = as_op8(v);
        } else {
            f32x4 v0 = {0.f, 0.f, 0.f, 0.f}, v1 = {0.f, 0.f, 0.f, 0.f};
            if (in) {
                v0 = *(const f32x4 *)(ff + i16 * ds + ch - cb);
                v1 = *(const f32x4 *)(ff + i16 * ds + ch - cb + 4);
            }
            i16x8 c[3];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                short t0, t1, t2;
                split3(j < 4 ? v0[j] : v1[j - 4], t0, t1, t2);
                c[0][j] = t0;
                c[1][j] = t1;
                c[2][j] = t2;
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) opC[t][i][h] = c[t];
        }
    }
}

// Prologue of the MFMA path: the union ordered by id and the slot table.
template <int K, int FT>
__device__ __forceinline__ void mf_begin(UnionLds<K, FT> &L, Slots<K> &s, int U, const SlotTable<K> &st) {
    mf_prologue<K, FT>(L, s, U);
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        st.u[t * K + k] = s.u[k];
        st.wa[t * K + k] = s.u[k] >= 0 ? s.wf[k] : 0.f;
        if constexpr (FT == FT_FP8 || !mf_compact(K)) st.wd[t * K + k] = s.u[k] >= 0 ? s.wp[k] : 0.f;
    }
}

// The slab's operands, through the staging area `ft` (over the ring and the wave
// buffers: every wave must be done with them, hence the barrier first).  Union blocks
// past U get zero operands.
template <int K, int FT, int NT, int CPW, int NUB>
__device__ __forceinline__ void mf_load_slab(const UnionLds<K, FT> &L, int U, int D, const void *__restrict__ feat,
                                             void *ft, const MfSlab &sb, const MfChunks &mc, int lane,
                                             i16x4 (&opA)[NT][CPW][2][NUB], i16x8 (&opC)[NT][CPW][NUB]) {
#pragma unroll
    for (int h = 0; h < NUB; ++h) {
        if (h > 0 && 16 * h >= U) {   // uniform over the block
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    opA[t][i][0][h] = (i16x4){0, 0, 0, 0};
                    opA[t][i][1][h] = (i16x4){0, 0, 0, 0};
                    opC[t][i][h] = (i16x8){0, 0, 0, 0, 0, 0, 0, 0};
                }
            continue;
        }
        __syncthreads();
        mf_stage_half<K, FT>(L, U, D, h, sb, feat, ft);
        __syncthreads();
        mf_load_ops<FT, NT, CPW, NUB>(ft, U, D, h, sb, mc, lane, opA, opC);
    }
    __syncthreads();
}

// The weight ring (all 256 threads take part in clearing and scattering).
template <typename RB>
__device__ __forceinline__ void ring_clear(RB &rb) {
    constexpr int n16 = (int)sizeof(RB) / 16;
#pragma unroll
    for (int q = 0; q < (n16 + kFB - 1) / kFB; ++q) {
        const int i = q * kFB + (int)threadIdx.x;
        if (i < n16) ((u32x4 *)&rb)[i] = (u32x4){0u, 0u, 0u, 0u};
    }
}

// Scatters tile row `row`'s slots (16 pixels x K) into a cleared ring buffer, each
// FP32 weight as hi = RNE(w) and lo = RNE(w - hi).
template <int K, typename RB>
__device__ __forceinline__ void ring_scatter(int row, const SlotTable<K> &st, RB &rb) {
    const int t = threadIdx.x;
    if (t < 16 * K) {
        const int x = t & 15, k = t >> 4, p = row * 16 + x;
        const int u = st.u[p * K + k];
        if (u >= 0) {
            const float a = st.wa[p * K + k];
            rb.wa[0][x][u] = bits_bf16(a);
            rb.wa[1][x][u] = bits_bf16(a - bf16_to_f32(bits_bf16(a)));
            if constexpr (RB::WD) {
                const float d = st.wd[p * K + k];
                rb.wd[0][u][x] = bits_bf16(d);
                rb.wd[1][u][x] = bits_bf16(d - bf16_to_f32(bits_bf16(d)));
            }
        }
    }
}

// Operands of one row from its ring buffer, for union blocks s < NUB:
//   wa[s][h]: lane (i16, g) = Wa_h[pixel i16][16 s + 4 g + j], j < 4     (16x16x16 B)
//   wd[s]:    lane (i16, g) = Wd_{g/2}[pixel 8 (g % 2) + j][16 s + i16]    (16x16x32 A)
template <int NUB, typename RB>
__device__ __forceinline__ void ring_read(const RB &rb, int lane, i16x4 (&wa)[NUB][2], i16x8 (&wd)[NUB]) {
    const int i16 = lane & 15, g = lane >> 4;
#pragma unroll
    for (int s = 0; s < NUB; ++s) {
#pragma unroll
        for (int h = 0; h < 2; ++h) wa[s][h] = *(const i16x4 *)&rb.wa[h][i16][16 * s + 4 * g];
        if constexpr (RB::WD) wd[s] = *(const i16x8 *)&rb.wd[g >> 1][16 * s + i16][8 * (g & 1)];
    }
}

// Ring schedule: before the rows, buffers 0 and 1 are cleared and row 0 scattered
// into buffer 0.  At row r, after the block barrier: read buffer r % 3, scatter row
// r + 1 into buffer (r + 1) % 3 (cleared during row r - 1) and clear buffer
// (r + 2) % 3 (last read during row r - 1).
template <int K, typename RB>
__device__ __forceinline__ void ring_start(RB *ring, const SlotTable<K> &st) {
    ring_clear(ring[0]);
    ring_clear(ring[1]);
    __syncthreads();
    ring_scatter<K>(0, st, ring[0]);
}
template <int K, int NUB, typename RB>
__device__ __forceinline__ void ring_row(RB *ring, const SlotTable<K> &st, int row, int lane, i16x4 (&wa)[NUB][2],
                                         i16x8 (&wd)[NUB]) {
    __syncthreads();
    const int b = row % 3;
    ring_read<NUB>(ring[b], lane, wa, wd);
    if (row + 1 < 16) ring_scatter<K>(row + 1, st, ring[b == 2 ? 0 : b + 1]);
    ring_clear(ring[b == 0 ? 2 : b - 1]);
}

// Map block (chunk i, channel block b) of the current row: lane (i16, g) gets
// F[pixel i16][chunk + 8 g + 4 b + r], r < 4.  Forward and backward run this same
// sequence, so the recomputed map is bit-identical to the stored one.
template <int NT, int CPW, int NUB>
__device__ __forceinline__ f32x4 mf_map(const i16x4 (&opA)[NT][CPW][2][NUB], int i, int b,
                                        const i16x4 (&wa)[NUB][2], int nub) {
    f32x4 F = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < NUB; ++h) {
        if (h > 0 && h >= nub) break;   // block 0 unconditionally (straight-line MFMAs)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            F = mfma16(opA[t][i][b][h], wa[h][0], F);
            F = mfma16(opA[t][i][b][h], wa[h][1], F);
        }
    }
    return F;
}

// Sign of the L1 feature loss gradient for two packed BF16 map values against the
// target: -1, 0 or +1 per value, packed as BF16 (the loss scale is applied to the
// sums).  d = F - F^ is exact; scaling it by 2^140 lifts every nonzero difference
// of two BF16 values (at least 2^-133) to 2^7 or more before the clamp to [-1, 1].
__device__ __forceinline__ uint32_t l1_sign2(uint32_t f, uint32_t t) {
    const float d0 = __uint_as_float(f << 16) - __uint_as_float(t << 16);
    const float d1 = __uint_as_float(f & 0xFFFF0000u) - __uint_as_float(t & 0xFFFF0000u);
    const float s0 = __builtin_amdgcn_fmed3f(__builtin_ldexpf(d0, 140), -1.f, 1.f);
    const float s1 = __builtin_amdgcn_fmed3f(__builtin_ldexpf(d1, 140), -1.f, 1.f);
    return pk_bf16(s0, s1);
}
// The same for FP32 map values (the rounded difference keeps the sign of the exact one).
__device__ __forceinline__ float l1_sign(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }
__device__ __forceinline__ u32x4 l1_sign8(f32x4 F0, f32x4 F1, u32x4 T0, u32x4 T1) {
    const f32x4 t0 = __builtin_bit_cast(f32x4, T0), t1 = __builtin_bit_cast(f32x4, T1);
    u32x4 G;
    G.x = pk_bf16(l1_sign(F0[0] - t0[0]), l1_sign(F0[1] - t0[1]));
    G.y = pk_bf16(l1_sign(F0[2] - t0[2]), l1_sign(F0[3] - t0[3]));
    G.z = pk_bf16(l1_sign(F1[0] - t1[0]), l1_sign(F1[1] - t1[1]));
    G.w = pk_bf16(l1_sign(F1[2] - t1[2]), l1_sign(F1[3] - t1[3]));
    return G;
}

template <int K, int FT, int MT, int NUB>
__device__ __forceinline__ void mf_forward(const TileGeom &tg, int W, int H, int D, int U,
                                           const void *__restrict__ feat, void *__restrict__ F,
                                           UnionLds<K, FT> &L, Slots<K> &s, unsigned char *dyn) {
    typedef MfForm<FT, MT, NUB> Fm;
    constexpr int NT = Fm::NT, CPW = Fm::CPW;
    static_assert(NUB <= mf_nub_max(K), "the LDS layout holds this form's ring");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const SlotTable<K> st = slot_table<K, FT == FT_FP8>(dyn, false);
    MfRingF<NUB> *ring = (MfRingF<NUB> *)(dyn + mf_ring_at(K, false, FT == FT_FP8));
    MfWaveF &mw = ((MfWaveF *)(dyn + mf_waves_at(K, false, FT == FT_FP8)))[wave];
    mf_begin<K, FT>(L, s, U, st);
    const int nub = (U + 15) >> 4;   // union blocks in use
    const int i16 = lane & 15, g = lane >> 4;
    const int rows = min(16, H - tg.ty0);
    const int ns = mf_nslabs(D, 4 * CPW);
    for (int sl = 0; sl < ns; ++sl) {
        const MfSlab sb = mf_slab(D, ns, sl);
        const MfChunks mc = mf_chunks(sb, wave);
        i16x4 opA[NT][CPW][2][NUB];
        i16x8 opC[NT][CPW][NUB];
        mf_load_slab<K, FT, NT, CPW, NUB>(L, U, D, feat, ring, sb, mc, lane, opA, opC);
        ring_start<K>(ring, st);
        for (int row = 0; row < rows; ++row) {
            i16x4 wa[NUB][2];
            i16x8 wd[NUB];
            ring_row<K, NUB>(ring, st, row, lane, wa, wd);
            // the row's map values go through LDS (16-byte pieces XOR-swizzled by pixel)
            // so that every store instruction writes whole pixel rows: 16 lanes x 16
            // bytes per pixel, four pixels per instruction
            const long rowpix = (long)tg.view * W * H + (long)(tg.ty0 + row) * W + tg.tx0;
            const int piece = lane & 15;
            if constexpr (!Fm::M32) {
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    if (i >= mc.n) break;
                    const f32x4 F0 = mf_map<NT, CPW, NUB>(opA, i, 0, wa, nub);
                    const f32x4 F1 = mf_map<NT, CPW, NUB>(opA, i, 1, wa, nub);
                    u32x4 o = {pk_bf16(F0[0], F0[1]), pk_bf16(F0[2], F0[3]), pk_bf16(F1[0], F1[1]),
                               pk_bf16(F1[2], F1[3])};
                    *(u32x4 *)&mw.out[i16][8 * ((4 * i + g) ^ i16)] = o;
                }
                wave_lds_sync();
                const int ch = mc.beg * 32 + 8 * piece;   // 8 channels per piece
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int px = 4 * q + (lane >> 4);
                    if (tg.tx0 + px < W && piece < 4 * mc.n && ch < D)
                        *(u32x4 *)((uint16_t *)F + (rowpix + px) * D + ch) =
                            *(const u32x4 *)&mw.out[px][8 * (piece ^ px)];
                }
            } else {
                float(*out)[64] = (float(*)[64])mw.out;   // [pixel][64 channels]
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    if (i >= mc.n) break;
                    const f32x4 F0 = mf_map<NT, CPW, NUB>(opA, i, 0, wa, nub);
                    const f32x4 F1 = mf_map<NT, CPW, NUB>(opA, i, 1, wa, nub);
                    const int pc = 8 * i + 2 * g;
                    *(f32x4 *)&out[i16][4 * (pc ^ i16)] = F0;
                    *(f32x4 *)&out[i16][4 * ((pc + 1) ^ i16)] = F1;
                }
                wave_lds_sync();
                const int ch = mc.beg * 32 + 4 * piece;   // 4 channels per piece
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int px = 4 * q + (lane >> 4);
                    if (tg.tx0 + px < W && piece < 8 * mc.n && ch < D)
                        *(f32x4 *)((float *)F + (rowpix + px) * D + ch) = *(const f32x4 *)&out[px][4 * (piece ^ px)];
                }
            }
            wave_lds_sync();
        }
    }
}

// Backward of the MFMA path.  L1: dF holds the target map and G = l1_scale
// sign(F - F^) is formed from the recomputed map (the products take the sign, the
// sums the scale); otherwise dF holds dL/dF (BF16 map only).  SF (with L1): the map
// is also stored to Fo, so one pass renders and differentiates.
template <int K, int FT, int MT, int NUB, bool L1, bool SF, int R, bool MULTI>
__device__ __forceinline__ void mf_backward(const TileGeom &tg, int W, int H, int D, int U,
                                            const void *__restrict__ feat, const void *__restrict__ dF,
                                            float gs, float *__restrict__ dfeat, float *__restrict__ dtw,
                                            void *__restrict__ Fo, UnionLds<K, FT> &L, Slots<K> &s,
                                            unsigned char *dyn) {
    typedef MfForm<FT, MT, NUB> Fm;
    constexpr int NT = Fm::NT, CPW = Fm::CPW, TW = Fm::M32 ? 2 : 1;   // target pieces per chunk
    constexpr int SP = sp_stride<NUB>();
    static_assert(NUB <= mf_nub_max(K), "the LDS layout holds this form's ring");
    static_assert(L1 || !SF, "the map is stored only on the L1 path");
    static_assert(L1 || !Fm::M32, "dL/dF enters the products as BF16");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the waves' partial dot products, [4][256][K] (K <= 4), or those of the last two
    // rows [2][4][16][K] and the tile's sums [256][K]; slabs after the first add theirs
    constexpr bool RS = mf_compact(K);
    float *sred = (float *)dyn;
    float *sring = (float *)dyn;
    float *gsum = sring + 2 * 4 * 16 * K;
    const SlotTable<K> st = slot_table<K, FT == FT_FP8>(dyn, true);
    MfRingB<NUB> *ring = (MfRingB<NUB> *)(dyn + mf_ring_at(K, true, FT == FT_FP8));
    MfWaveB &mw = ((MfWaveB *)(dyn + mf_waves_at(K, true, FT == FT_FP8)))[wave];
    // row r's four partials meet after the barrier of row r + 1, in a fixed order (the
    // first slab stores the sums, later slabs add theirs)
    auto sum_row = [&](int r, bool first) {
        const int t = threadIdx.x;
        if (t < 16 * K) {
            const int i = t & 15, k = t >> 4;
            const float *b = sring + (size_t)(r & 1) * 4 * 16 * K;
            float v = b[(0 * 16 + i) * K + k] + b[(1 * 16 + i) * K + k];
            v += b[(2 * 16 + i) * K + k];
            v += b[(3 * 16 + i) * K + k];
            float &d = gsum[(r * 16 + i) * K + k];
            d = first ? v : d + v;
        }
    };
    mf_begin<K, FT>(L, s, U, st);
    const int nub = (U + 15) >> 4;   // union blocks in use
    const int i16 = lane & 15, g = lane >> 4;
    const int x = tg.tx0 + i16;
    const int rows = min(16, H - tg.ty0);
    const float gscale = L1 ? gs : 1.f;   // the L1 path accumulates sign(F - F^)
    auto row_at = [&](int row) { return ((long)tg.view * W * H + (long)(tg.ty0 + row) * W + tg.tx0) * D; };
    const int ns = mf_nslabs(D, 4 * CPW);
    // one slab's row loop; the first slab is peeled out of the loop over the others.
    // MULTI: the launch's D takes several slabs; the one-slab kernel has no loop at all,
    // which keeps its register allocation free of the loop's live ranges
    auto slab = [&](int sl, auto first_tag) __attribute__((always_inline)) {
        constexpr bool FIRST = decltype(first_tag)::value;
        const MfSlab sb = mf_slab(D, ns, sl);
        const MfChunks mc = mf_chunks(sb, wave);
        i16x4 opA[NT][CPW][2][NUB];
        i16x8 opC[NT][CPW][NUB];
        mf_load_slab<K, FT, NT, CPW, NUB>(L, U, D, feat, ring, sb, mc, lane, opA, opC);
        ring_start<K>(ring, st);

        f32x4 acc[CPW][2][NUB];   // [chunk][channel block][union block]
#pragma unroll
        for (int i = 0; i < CPW; ++i)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < NUB; ++v) acc[i][b][v] = (f32x4){0.f, 0.f, 0.f, 0.f};

        // dL/dF (or the target) of R - 1 rows ahead, in an R-deep register ring; lane
        // (i16, g) reads channels 8g..8g+7 of each chunk for pixel i16 (one 16-byte
        // piece in BF16, two in FP32).  The loads carry no branches: each is a uniform
        // row base plus a per-lane offset fixed for the tile, where a lane whose pixel or
        // channels lie outside reads the row's first element (rows past the image read
        // the last row).  Such values meet only zero weights and zero operands; the L1
        // gradient is always finite, dL/dF is masked.
        u32x4 tb[R][CPW][TW];
        uint32_t loff[CPW];
        bool lon[CPW];
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int ch = (mc.beg + i) * 32 + 8 * g;
            lon[i] = x < W && i < mc.n && ch < D;
            loff[i] = lon[i] ? (uint32_t)(i16 * D + ch) : 0u;
        }
        auto fetch = [&](int row, u32x4 (&dst)[CPW][TW]) {
            const long base = row_at(min(row, rows - 1));
#pragma unroll
            for (int i = 0; i < CPW; ++i) {
                if constexpr (Fm::M32) {
                    const float *p = (const float *)dF + base + loff[i];
                    dst[i][0] = *(const u32x4 *)p;
                    dst[i][TW - 1] = *(const u32x4 *)(p + 4);
                } else {
                    dst[i][0] = *(const u32x4 *)((const uint16_t *)dF + base + loff[i]);
                }
            }
        };
#pragma unroll
        for (int r = 0; r < R - 1; ++r) fetch(r, tb[r]);

        // every wave walks all 16 rows and all CPW chunks: rows past the image and
        // chunks past D carry zero weights and zero operands
#pragma unroll 1
        for (int row0 = 0; row0 < 16; row0 += R) {
#pragma unroll
            for (int h = 0; h < R; ++h) {
                const int row = row0 + h;
                fetch(row + R - 1, tb[(h + R - 1) % R]);
                i16x4 wa[NUB][2];
                i16x8 wd[NUB];
                ring_row<K, NUB>(ring, st, row, lane, wa, wd);
                if constexpr (RS)
                    if (row > 0) sum_row(row - 1, FIRST);
                f32x4 sacc[NUB];
#pragma unroll
                for (int v = 0; v < NUB; ++v) sacc[v] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    u32x4 G;
                    if constexpr (L1) {
                        const f32x4 F0 = mf_map<NT, CPW, NUB>(opA, i, 0, wa, nub);
                        const f32x4 F1 = mf_map<NT, CPW, NUB>(opA, i, 1, wa, nub);
                        if constexpr (!Fm::M32) {
                            u32x4 Fp = {pk_bf16(F0[0], F0[1]), pk_bf16(F0[2], F0[3]), pk_bf16(F1[0], F1[1]),
                                        pk_bf16(F1[2], F1[3])};
                            __asm__ volatile("" : "+v"(Fp.x), "+v"(Fp.y), "+v"(Fp.z), "+v"(Fp.w));
                            // the stored map: the target's layout, so the same per-lane offsets
                            if constexpr (SF)
                                if (row < rows && lon[i]) *(u32x4 *)((uint16_t *)Fo + row_at(row) + loff[i]) = Fp;
                            const u32x4 T = tb[h][i][0];
                            G.x = l1_sign2(Fp.x, T.x);
                            G.y = l1_sign2(Fp.y, T.y);
                            G.z = l1_sign2(Fp.z, T.z);
                            G.w = l1_sign2(Fp.w, T.w);
                        } else {
                            if constexpr (SF)
                                if (row < rows && lon[i]) {
                                    float *p = (float *)Fo + row_at(row) + loff[i];
                                    *(f32x4 *)p = F0;
                                    *(f32x4 *)(p + 4) = F1;
                                }
                            G = l1_sign8(F0, F1, tb[h][i][0], tb[h][i][TW - 1]);
                        }
                    } else {
                        G = (row < rows && lon[i]) ? tb[h][i][0] : (u32x4){0u, 0u, 0u, 0u};
                    }
                    // keep G packed: its halves are stored as they are, not re-derived
                    __asm__ volatile("" : "+v"(G.x), "+v"(G.y), "+v"(G.z), "+v"(G.w));
                    // dot products over the chunk's 32 channels
#pragma unroll
                    for (int v = 0; v < NUB; ++v) {
                        if (v > 0 && v >= nub) break;
#pragma unroll
                        for (int t = 0; t < NT; ++t) sacc[v] = mfma32(opC[t][i][v], as_op8(G), sacc[v]);
                    }
                    // G transposed: block b row 4g + r <- this lane's channel 8g + 4b + r
                    mw.gt[i][0][4 * g + 0][i16] = (uint16_t)(G.x & 0xFFFFu);
                    mw.gt[i][0][4 * g + 1][i16] = (uint16_t)(G.x >> 16);
                    mw.gt[i][0][4 * g + 2][i16] = (uint16_t)(G.y & 0xFFFFu);
                    mw.gt[i][0][4 * g + 3][i16] = (uint16_t)(G.y >> 16);
                    mw.gt[i][1][4 * g + 0][i16] = (uint16_t)(G.z & 0xFFFFu);
                    mw.gt[i][1][4 * g + 1][i16] = (uint16_t)(G.z >> 16);
                    mw.gt[i][1][4 * g + 2][i16] = (uint16_t)(G.w & 0xFFFFu);
                    mw.gt[i][1][4 * g + 3][i16] = (uint16_t)(G.w >> 16);
                }
                wave_lds_sync();
                // gradient rows: B operand [hi pixels; lo pixels] x 16 block rows, i.e. G of
                // pixels 8 (g % 2) + j
#pragma unroll
                for (int i = 0; i < CPW; ++i)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const i16x8 g2 = *(const i16x8 *)&mw.gt[i][b][i16][8 * (g & 1)];
#pragma unroll
                        for (int v = 0; v < NUB; ++v) {
                            if (v > 0 && v >= nub) break;
                            acc[i][b][v] = mfma32(wd[v], g2, acc[i][b][v]);
                        }
                    }
                wave_lds_sync();
                // this wave's share of S^T for the row -> its K slots, through LDS (rows of
                // SP floats)
                float *spb = (float *)&mw;   // [16 NUB][SP], over the G buffer
#pragma unroll
                for (int v = 0; v < NUB; ++v)
#pragma unroll
                    for (int r = 0; r < 4; ++r) spb[(16 * v + 4 * g + r) * SP + i16] = sacc[v][r];
                wave_lds_sync();
                const int p = row * 16 + i16;
                for (int k = g; k < K; k += 4) {
                    const int u = st.u[p * K + k];
                    const float val = u >= 0 ? gscale * spb[u * SP + i16] : 0.f;
                    if constexpr (RS) {
                        sring[(((row & 1) * 4 + wave) * 16 + i16) * K + k] = val;
                    } else {
                        float &d = sred[(wave * kTilePix + p) * K + k];
                        d = FIRST ? val : d + val;
                    }
                }
                wave_lds_sync();
            }
        }
        if constexpr (RS) {
            __syncthreads();
            sum_row(15, FIRST);
        }

        // gradient rows: lane (i16, g) holds dFt[16 v + 4 g + r][chunk + blk_ch(b, i16)]
#pragma unroll
        for (int v = 0; v < NUB; ++v) {
            if (v >= nub) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = 16 * v + 4 * g + r;
                if (u >= U) continue;
                float *dst = dfeat + (long)L.uid2[u] * D;
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    if (i >= mc.n) break;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int ch = (mc.beg + i) * 32 + blk_ch(b, i16);
                        const float val = gscale * acc[i][b][v][r];
                        if (ch < D && val != 0.f) unsafeAtomicAdd(dst + ch, val);
                    }
                }
            }
        }
    };
    slab(0, std::true_type{});
    if constexpr (MULTI)
        for (int sl = 1; sl < ns; ++sl) slab(sl, std::false_type{});
    __syncthreads();
    // gamma_k = (g_k - sum_j w'_j g_j) / W for the thread's own pixel
    const int t = threadIdx.x;
    const int px = tg.tx0 + (t & 15), py = tg.ty0 + (t >> 4);
    if (px >= W || py >= H) return;
    const long p = (long)tg.view * W * H + (long)py * W + px;
    // the pixel's slots come back from the slot table (its union indices, and w'_k in wd,
    // 0 for an empty slot), so they need no registers through the slab loop
    float gk[K], mean = 0.f;
    int uk[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uk[k] = st.u[t * K + k];
        float v;
        if constexpr (RS) {
            v = gsum[t * K + k];
        } else {
            v = sred[(0 * kTilePix + t) * K + k] + sred[(1 * kTilePix + t) * K + k];
            v += sred[(2 * kTilePix + t) * K + k];
            v += sred[(3 * kTilePix + t) * K + k];
        }
        if constexpr (FT == FT_FP8) v *= uk[k] >= 0 ? L.uscale2[uk[k]] : 0.f;
        gk[k] = uk[k] >= 0 ? v : 0.f;
        mean = fmaf(st.wd[t * K + k], gk[k], mean);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) dtw[p * K + k] = uk[k] >= 0 ? (gk[k] - mean) / s.W : 0.f;
}

// ---------------------------------------------------------------- forward

// The wave's pixels.  STAGED: every union row of the tile is in LDS, so the loop
// issues no global loads at all and its stores never have to be waited for.
template <int K, int FT, int MT, bool STAGED>
__device__ __forceinline__ void fwd_pixels(const TileGeom &tg, int W, int H, int D, int U, int ucap,
                                           const void *__restrict__ feat, void *__restrict__ F,
                                           const Slots<K> &sl, const UnionLds<K, FT> &L,
                                           unsigned char *rows, int wave, int lane) {
    constexpr int CPL = TileCfg<K>::CPL, PW = pass_ch<K>();
    const int passes = (D + PW - 1) / PW;
    for (int pass = 0; pass < passes; ++pass) {
        stage_pass<K, FT>(L, U, D, ucap, pass, feat, rows);
        const int c0 = pass * PW + lane * CPL;
        const bool lane_on = c0 < D;
        for (int i = 0; i < kPixPerWave; ++i) {
            const int x = tg.tx0 + (i & 15), y = tg.ty0 + wave * 4 + (i >> 4);
            if (x >= W || y >= H) continue;
            const long p = (long)tg.view * W * H + (long)y * W + x;
            float out[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) out[j] = 0.f;
            if constexpr (STAGED) {
                // branch-free: an empty slot reads row 0 with weight 0, a lane past D
                // reads the pass's first channel and stores nothing; all K reads issue together
                const int cc = lane_on ? lane * CPL : 0;
                float v[K][CPL];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int u = rdlane(sl.u[k], i);
                    loadc<FT, CPL>(rows, (long)(u < 0 ? 0 : u) * PW + cc, v[k]);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float wf = rdlane(sl.wf[k], i);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) out[j] = fmaf(wf, v[k][j], out[j]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int u = rdlane(sl.u[k], i);
                    if (u < 0 || !lane_on) continue;
                    const float wf = rdlane(sl.wf[k], i);
                    float v[CPL];
                    urow<K, FT, CPL>(rows, ucap, L.uid, u, pass, feat, D, c0, v);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) out[j] = fmaf(wf, v[j], out[j]);
                }
            }
            if (lane_on) storec<MT, CPL>(F, p * D + c0, out);
        }
    }
}

// Tiles take the MFMA path when the union fits (at most kUP Gaussians, or kUP2 for K > 4), K <= 8, and,
// in the adjoint, dL/dF is exact in BF16: a BF16 map, or the L1 loss, whose gradient
// enters as sign(F - F^) with the scale applied to the sums.  MODE -1: the forward.
template <int K, int FT, int MT, int MODE>
struct MfOk {
    static constexpr bool v = K <= 8 && (MODE < 0 || MT == MT_BF16 || MODE >= 1);
};

template <int K, int FT, int MT>
__global__ __launch_bounds__(kFB) void feature_fwd_kernel(int W, int H, int views, int D, int ucap,
                                                          const void *__restrict__ feat,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ ids,
                                                          const float *__restrict__ tw,
                                                          void *__restrict__ F) {
    extern __shared__ __align__(16) unsigned char lds[];
    UnionLds<K, FT> &L = *reinterpret_cast<UnionLds<K, FT> *>(lds);
    unsigned char *dyn = lds + union_bytes<K, FT>();   // the per-pixel path's staged rows
    const int ntiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile) * views;
    const int tile = xcd_strips(blockIdx.x);
    if (tile >= ntiles) return;
    const TileGeom tg = tile_geom(tile, W, H);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Slots<K> sl;
    int U;
    tile_union<K, FT>(tg, W, H, ids, tw, scale, L, sl, U);
    if constexpr (MfOk<K, FT, MT, -1>::v) {
        if (U <= kUP) {
            mf_forward<K, FT, MT, 2>(tg, W, H, D, U, feat, F, L, sl, lds + union_keep_bytes<K, FT>());
            return;
        }
        if constexpr (mf_nub_max(K) == 4) {
            if (U <= kUP2) {
                mf_forward<K, FT, MT, 4>(tg, W, H, D, U, feat, F, L, sl, lds + union_keep_bytes<K, FT>());
                return;
            }
        }
    }
    if (U >= 1 && U <= ucap) fwd_pixels<K, FT, MT, true>(tg, W, H, D, U, ucap, feat, F, sl, L, dyn, wave, lane);
    else fwd_pixels<K, FT, MT, false>(tg, W, H, D, U, ucap, feat, F, sl, L, dyn, wave, lane);
}

// ---------------------------------------------------------------- backward

// The wave's pixels for one channel pass after another.  STAGED: every union row of
// the tile is in LDS, so the only global traffic in the loop is dL/dF (or the target).
template <int K, int FT, int MT, bool L1, bool SF, bool STAGED>
__device__ __forceinline__ void bwd_pixels(const TileGeom &tg, int W, int H, int D, int U, int ucap,
                                           const void *__restrict__ feat, const void *__restrict__ dF,
                                           float l1_scale, float *__restrict__ dfeat, void *__restrict__ Fo,
                                           const Slots<K> &sl, const UnionLds<K, FT> &L,
                                           unsigned char *rows, int nw,
                                           float (*sdot)[K], float *xbuf, int wave, int lane) {
    constexpr int CPL = TileCfg<K>::CPL, RA = TileCfg<K>::RA, PW = pass_ch<K>();
    const float gs = MT == MT_F32 ? l1_scale : bf16_to_f32(f32_to_bf16(l1_scale));
    constexpr int MS = MT == MT_F32 ? FT_F32 : FT_BF16;
    const int passes = (D + PW - 1) / PW;
    for (int pass = 0; pass < passes; ++pass) {
        stage_pass<K, FT>(L, U, D, ucap, pass, feat, rows);
        const int c0 = pass * PW + lane * CPL;
        const bool lane_on = c0 < D;
        float acc[RA][CPL];
#pragma unroll
        for (int r = 0; r < RA; ++r)
#pragma unroll
            for (int j = 0; j < CPL; ++j) acc[r][j] = 0.f;
        // dL/dF (or the target) one pixel ahead of its use
        auto want = [&](int i) {
            const int x = tg.tx0 + (i & 15), y = tg.ty0 + wave * 4 + (i >> 4);
            return x < W && y < H && rdlane(sl.W, i) > 0.f;
        };
        auto fetch = [&](int i, float (&dst)[CPL]) {
            const int x = tg.tx0 + (i & 15), y = tg.ty0 + wave * 4 + (i >> 4);
#pragma unroll
            for (int j = 0; j < CPL; ++j) dst[j] = 0.f;
            if (want(i) && lane_on)
                loadc<MS, CPL>(dF, ((long)tg.view * W * H + (long)y * W + x) * D + c0, dst);
        };
        float nxt[CPL];
        fetch(0, nxt);
        for (int i = 0; i < kPixPerWave; ++i) {
            float cur[CPL];
#pragma unroll
            for (int j = 0; j < CPL; ++j) cur[j] = nxt[j];
            if (i + 1 < kPixPerWave) fetch(i + 1, nxt);
            if constexpr (SF) {
                // pixels without contributors still get their (zero) map entries
                const int x = tg.tx0 + (i & 15), y = tg.ty0 + wave * 4 + (i >> 4);
                if (x < W && y < H && !(rdlane(sl.W, i) > 0.f) && lane_on) {
                    float z[CPL];
#pragma unroll
                    for (int j = 0; j < CPL; ++j) z[j] = 0.f;
                    storec<MT, CPL>(Fo, ((long)tg.view * W * H + (long)y * W + x) * D + c0, z);
                }
            }
            if (!want(i)) continue;
            int wl[K];
            float wp[K], v[K][CPL];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                wl[k] = rdlane(sl.wl[k], i);
                wp[k] = rdlane(sl.wp[k], i);
#pragma unroll
                for (int j = 0; j < CPL; ++j) v[k][j] = 0.f;
                const int u = rdlane(sl.u[k], i);
                if constexpr (STAGED) {
                    // branch-free (see the forward); empty slots carry weight 0 and
                    // their dot product is never used
                    loadc<FT, CPL>(rows, (long)(u < 0 ? 0 : u) * PW + (lane_on ? lane * CPL : 0), v[k]);
                    if (!lane_on) {
#pragma unroll
                        for (int j = 0; j < CPL; ++j) v[k][j] = 0.f;
                    }
                } else if (u >= 0 && lane_on) {
                    urow<K, FT, CPL>(rows, ucap, L.uid, u, pass, feat, D, c0, v[k]);
                }
            }
            float G[CPL];
            if constexpr (L1) {
                float Fv[CPL];
#pragma unroll
                for (int j = 0; j < CPL; ++j) Fv[j] = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (wl[k] < 0) continue;
                    const float wf = rdlane(sl.wf[k], i);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) Fv[j] = fmaf(wf, v[k][j], Fv[j]);
                }
                float fm[CPL];
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    fm[j] = MT == MT_F32 ? Fv[j] : bf16_to_f32(f32_to_bf16(Fv[j]));
                    const float d = lane_on ? fm[j] - cur[j] : 0.f;
                    G[j] = d > 0.f ? gs : (d < 0.f ? -gs : 0.f);
                }
                if constexpr (SF) {
                    const int x = tg.tx0 + (i & 15), y = tg.ty0 + wave * 4 + (i >> 4);
                    if (lane_on) storec<MT, CPL>(Fo, ((long)tg.view * W * H + (long)y * W + x) * D + c0, fm);
                }
            } else {
#pragma unroll
                for (int j = 0; j < CPL; ++j) G[j] = cur[j];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float part = 0.f;
#pragma unroll
                for (int j = 0; j < CPL; ++j) part = fmaf(G[j], v[k][j], part);
                if constexpr (FT == FT_FP8) {
                    const int u = rdlane(sl.u[k], i);
                    part *= (u >= 0 ? L.uscale[u] : 0.f);
                }
                const float g = wave_sum(part);
                if (lane == 0) sdot[i][k] += g;
                if (wl[k] < 0) continue;
                if (wl[k] < RA) {
#pragma unroll
                    for (int r = 0; r < RA; ++r) {
                        if (r != wl[k]) continue;
#pragma unroll
                        for (int j = 0; j < CPL; ++j) acc[r][j] = fmaf(wp[k], G[j], acc[r][j]);
                    }
                } else {
                    // beyond the register accumulators: straight to global memory
                    float a[CPL];
#pragma unroll
                    for (int j = 0; j < CPL; ++j) a[j] = wp[k] * G[j];
                    flush_row<CPL>(a, L.wlist[wave][wl[k]], D, pass * 64 * CPL, lane, dfeat, xbuf);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RA; ++r)
            if (r < nw) flush_row<CPL>(acc[r], L.wlist[wave][r], D, pass * 64 * CPL, lane, dfeat, xbuf);
    }
}

// MODE 0: dF holds dL/dF (map dtype).  MODE 1: dF holds the target map F^ and
// dL/dF = l1_scale * sign(F - F^) is formed on the fly from F recomputed exactly as
// the forward kernel computes and rounds it.  MODE 2: as 1, and that F is stored to
// Fo, bit-identical to the forward kernel's map (render and adjoint in one pass).
constexpr int kRing = 1;   // rows of dL/dF in flight on the MFMA path, besides the one in use

template <int K, int CPL>
constexpr size_t fallback_extra() { return (size_t)4 * kPixPerWave * K * 4 + (size_t)4 * 64 * CPL * 4; }

// Two blocks per CU: registers are capped at 256 per lane.
template <int K, int FT, int MT, int MODE, bool MULTI>
__global__ __launch_bounds__(kFB, 2) void feature_bwd_kernel(int W, int H, int views, int D, int ucap,
                                                          const void *__restrict__ feat,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ ids,
                                                          const float *__restrict__ tw,
                                                          const void *__restrict__ dF, float l1_scale,
                                                          float *__restrict__ dfeat,
                                                          float *__restrict__ dtw, void *__restrict__ Fo) {
    constexpr int CPL = TileCfg<K>::CPL;
    constexpr bool L1 = MODE >= 1, SF = MODE == 2;
    extern __shared__ __align__(16) unsigned char lds[];
    UnionLds<K, FT> &L = *reinterpret_cast<UnionLds<K, FT> *>(lds);
    unsigned char *dyn = lds + union_bytes<K, FT>();   // the per-pixel path's buffers
    const int ntiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile) * views;
    const int tile = xcd_strips(blockIdx.x);
    if (tile >= ntiles) return;
    const TileGeom tg = tile_geom(tile, W, H);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Slots<K> sl;
    int U;
    const int nw = tile_union<K, FT>(tg, W, H, ids, tw, scale, L, sl, U);
    if constexpr (MfOk<K, FT, MT, MODE>::v) {
        // gs: the loss scale as the unfused path's L1 gradient holds it (in the map's
        // format); formed inside each branch, where it costs no register across the union
        // build (formed before the branches, the one-pass kernel spilled)
        if (U <= kUP) {
            const float gs = MT == MT_F32 ? l1_scale : bf16_to_f32(f32_to_bf16(l1_scale));
            mf_backward<K, FT, MT, 2, L1, SF, kRing + 1, MULTI>(tg, W, H, D, U, feat, dF, gs, dfeat, dtw, Fo, L,
                                                                sl, lds + union_keep_bytes<K, FT>());
            return;
        }
        // unions of 33..64 (K > 4): four union blocks, one chunk per wave and slab, so
        // D takes several slabs and the loop over them
        if constexpr (mf_nub_max(K) == 4) {
            if (U <= kUP2) {
                const float gs = MT == MT_F32 ? l1_scale : bf16_to_f32(f32_to_bf16(l1_scale));
                mf_backward<K, FT, MT, 4, L1, SF, kRing + 1, true>(tg, W, H, D, U, feat, dF, gs, dfeat, dtw, Fo,
                                                                   L, sl, lds + union_keep_bytes<K, FT>());
                return;
            }
        }
    }
    // per-pixel path: staged rows, then the dot products and the transpose buffers
    float(*s_dot)[kPixPerWave][K] = (float(*)[kPixPerWave][K])(dyn + kRowBudget);
    float(*s_x)[64 * CPL] = (float(*)[64 * CPL])(dyn + kRowBudget + (size_t)4 * kPixPerWave * K * 4);
    float *xbuf = s_x[wave];
#pragma unroll
    for (int k = 0; k < K; ++k) s_dot[wave][lane][k] = 0.f;
    if (U >= 1 && U <= ucap)
        bwd_pixels<K, FT, MT, L1, SF, true>(tg, W, H, D, U, ucap, feat, dF, l1_scale, dfeat, Fo, sl, L, dyn, nw,
                                           s_dot[wave], xbuf, wave, lane);
    else
        bwd_pixels<K, FT, MT, L1, SF, false>(tg, W, H, D, U, ucap, feat, dF, l1_scale, dfeat, Fo, sl, L, dyn, nw,
                                            s_dot[wave], xbuf, wave, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // gamma_k = (g_k - sum_j w'_j g_j) / W for the lane's own pixel
    const int x = tg.tx0 + (lane & 15), y = tg.ty0 + wave * 4 + (lane >> 4);
    if (x >= W || y >= H) return;
    const long p = (long)tg.view * W * H + (long)y * W + x;
    float g[K], mean = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        g[k] = s_dot[wave][lane][k];
        mean = fmaf(sl.wp[k], g[k], mean);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        dtw[p * K + k] = (sl.W > 0.f && sl.id[k] >= 0) ? (g[k] - mean) / sl.W : 0.f;
}

// ---------------------------------------------------------------- launches

// Staged union rows per block: as many as fit in `budget` bytes (at least 0).
// Staged union rows per block on the per-pixel path: one pass's channels of as many rows
// as fit in `budget` bytes.
inline int pick_ucap(int pass_channels, int sf, int budget) { return budget / (pass_channels * sf); }

}  // namespace

template <int K, int FT, int MT>
lgs_status feature_fwd_launch(int W, int H, int views, int D, const void *feat, const float *scale,
                              const int *ids, const float *tw, void *F, hipStream_t st) {
    const unsigned grid = strip_grid((long)tiles_x(W) * tiles_y(H) * views);
    const int rb = pass_ch<K>() * Bytes<FT>::v;   // staged bytes per row and pass
    const size_t ub = union_bytes<K, FT>();
    // MFMA-capable kernels give the per-pixel path (unions beyond kUP) whatever rows
    // fit beside the union in the MFMA path's LDS, so that both paths keep their
    // blocks per CU
    size_t lds;
    int ucap;
    if (MfOk<K, FT, MT, -1>::v) {
        lds = union_keep_bytes<K, FT>() + mf_lds_bytes(K, false, FT == FT_FP8);
        ucap = lds > ub ? (int)((lds - ub) / rb) : 0;
        lds = std::max(lds, ub);
    } else {
        ucap = pick_ucap(pass_ch<K>(), Bytes<FT>::v, kRowBudget);
        lds = ub + (size_t)ucap * rb;
    }
    hipLaunchKernelGGL((feature_fwd_kernel<K, FT, MT>), dim3(grid), dim3(kFB), lds, st, W, H, views, D, ucap,
                       feat, scale, ids, tw, F);
    return check_launch("feature_render_fwd");
}

template <int K, int FT, int MT, int MODE>
lgs_status feature_bwd_launch(int W, int H, int views, int D, const void *feat, const float *scale,
                              const int *ids, const float *tw, const void *dF, float l1_scale, float *dfeat,
                              float *dtw, void *Fo, hipStream_t st) {
    const unsigned grid = strip_grid((long)tiles_x(W) * tiles_y(H) * views);
    const int ucap = pick_ucap(pass_ch<K>(), Bytes<FT>::v, kRowBudget);
    size_t lds = union_bytes<K, FT>() + kRowBudget + fallback_extra<K, TileCfg<K>::CPL>();
    if (MfOk<K, FT, MT, MODE>::v)
        lds = std::max(lds, union_keep_bytes<K, FT>() + mf_lds_bytes(K, true, FT == FT_FP8));
    // D beyond one channel slab takes the kernel with the loop over slabs
    if constexpr (MfOk<K, FT, MT, MODE>::v) {
        if (D > 4 * 32 * MfForm<FT, MT>::CPW) {
            hipLaunchKernelGGL((feature_bwd_kernel<K, FT, MT, MODE, true>), dim3(grid), dim3(kFB), lds, st, W, H,
                               views, D, ucap, feat, scale, ids, tw, dF, l1_scale, dfeat, dtw, Fo);
            return check_launch("feature_render_bwd");
        }
    }
    hipLaunchKernelGGL((feature_bwd_kernel<K, FT, MT, MODE, false>), dim3(grid), dim3(kFB), lds, st, W, H, views, D,
                       ucap, feat, scale, ids, tw, dF, l1_scale, dfeat, dtw, Fo);
    return check_launch("feature_render_bwd");
}

}  // namespace lgs

// Explicit instantiations of every storage / map / mode form for one K.
#define LGS_FEATURE_FORMS(K, FT, MT)                                                                     \
    template lgs_status feature_fwd_launch<K, FT, MT>(LGS_FEATURE_FWD_PARAMS);                           \
    template lgs_status feature_bwd_launch<K, FT, MT, 0>(LGS_FEATURE_BWD_PARAMS);                        \
    template lgs_status feature_bwd_launch<K, FT, MT, 1>(LGS_FEATURE_BWD_PARAMS);                        \
    template lgs_status feature_bwd_launch<K, FT, MT, 2>(LGS_FEATURE_BWD_PARAMS);
#define LGS_FEATURE_INSTANTIATE(K)                                                                       \
    namespace lgs {                                                                                      \
    LGS_FEATURE_FORMS(K, FT_F32, MT_F32)                                                                 \
    LGS_FEATURE_FORMS(K, FT_BF16, MT_BF16)                                                               \
    LGS_FEATURE_FORMS(K, FT_BF16, MT_F32)                                                                \
    LGS_FEATURE_FORMS(K, FT_FP8, MT_BF16)                                                                \
    LGS_FEATURE_FORMS(K, FT_FP8, MT_F32)                                                                 \
    }
