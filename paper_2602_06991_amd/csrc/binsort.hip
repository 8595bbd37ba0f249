// Tile binning and depth sort of the tile-based rasterizer (Sec. 3.1 follows 3DGS).
//
// Instead of one radix sort of 64-bit (tile | depth) keys over every (tile, Gaussian)
// pair, the Gaussians are sorted once by their 32-bit depth key (N items), the pairs
// are then written out in that depth order, and a stable sort by the tile index alone
// (ceil(log2 tiles) bits) finishes the (tile, depth, id) order.  Equal depth keys
// keep id order because every pass is stable and the first starts in id order.
//
// Every sort pass is an LSD radix pass with 8-bit digits in three launches:
// per-block digit histograms, a per-digit scan over blocks, and a stable scatter.
// The scatter ranks equal digits within a wave with ballots, orders the block's items
// by digit in LDS, and then writes each digit's run of the block with consecutive
// lanes, so the stores of a wave cover a few runs instead of up to 64 buckets.
#include "lgs_device.hpp"
#include "lgs_host.hpp"

#include <mutex>

namespace lgs {
namespace {

constexpr int kSortThreads = 256;
// Items per thread of a sort pass: 4 (1024 items per block, so the 0.5-2 M items of
// one frame still spread over hundreds of blocks), or 16 (4096 per block) from
// kBigPass items on, where fewer, fuller blocks write longer runs per digit.
constexpr int kSortIpt = 4;
constexpr int kSortIptBig = 16;
constexpr int kSortItems = kSortThreads * kSortIpt;   // the smallest block: sizes the histogram
constexpr long kBigPass = 1L << 22;
constexpr int kScanItems = 4096;
// Depth key of a record that touches no tile: sorts last, and the depth sort's first
// pass drops it (a positive depth's bit pattern never has the sign bit).
constexpr uint32_t kDropKey = 0xFFFFFFFFu;

// Exclusive scan of one value per thread over a 256-thread block.
template <typename T>
__device__ T block_exscan256(T v, T *lds, T &total) {
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        T x = t >= off ? lds[t - off] : (T)0;
        __syncthreads();
        lds[t] += x;
        __syncthreads();
    }
    T inc = lds[t];
    total = lds[255];
    __syncthreads();
    return inc - v;
}

__global__ __launch_bounds__(256) void depth_keys_kernel(int n, const float *__restrict__ depth,
                                                         const int *__restrict__ touched,
                                                         uint32_t *__restrict__ keys,
                                                         int *__restrict__ vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // positive depths order like their bit patterns; culled Gaussians go last
    keys[i] = touched[i] > 0 ? __float_as_uint(depth[i]) : kDropKey;
    vals[i] = i;
}

// The item count of a pass is n, or min(n, *n_dev) when the count lives on the device.
__device__ __forceinline__ int items_of(int n, const long long *n_dev) {
    return n_dev ? (int)min((long long)n, *n_dev) : n;
}

// Lanes of the wave (among those with `valid`) whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bb = __ballot(on);
        m &= on ? bb : ~bb;
    }
    return m;
}

// Digit counts of one block of IPT * 256 items, written digit-major (hist[d * nb + b]).
// When every valid lane of a wave holds the same digit (the top byte of nearby depths),
// the first of them adds the wave's count at once, so such keys do not serialise on one
// LDS counter; otherwise each lane adds its own (spread digits rarely collide, and the
// test costs two ballots where grouping equal digits costs eight).
template <int IPT>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                                  int n, const long long *__restrict__ n_dev,
                                                                  int shift, bool drop, int nb,
                                                                  int *__restrict__ hist) {
    __shared__ int h[256];
    const int t = threadIdx.x, lane = t & 63;
    n = items_of(n, n_dev);
    h[t] = 0;
    __syncthreads();
    const long base = (long)blockIdx.x * (kSortThreads * IPT);
    uint32_t k[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const long i = base + r * kSortThreads + t;
        k[r] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = base + r * kSortThreads + t < n && !(drop && k[r] == kDropKey);
        const uint32_t d = (k[r] >> shift) & 255u;
        const uint64_t vm = __ballot(valid);
        if (vm == 0ull) continue;   // the same for the whole wave
        const int first = (int)__builtin_ctzll(vm);
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, first);
        if (__ballot(valid && d == d0) == vm) {
            if (lane == first) atomicAdd(&h[d0], (int)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1);
        }
    }
    __syncthreads();
    hist[t * nb + blockIdx.x] = h[t];
}

// One block per digit: exclusive scan of that digit's per-block counts, in place.
__global__ __launch_bounds__(256) void radix_scan_digits_kernel(int *__restrict__ hist, int nb,
                                                                int *__restrict__ totals) {
    __shared__ int lds[256];
    int d = blockIdx.x;
    int *row = hist + (long)d * nb;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        int i = b0 + threadIdx.x;
        int v = i < nb ? row[i] : 0;
        int tot;
        int ex = block_exscan256(v, lds, tot);
        if (i < nb) row[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[d] = carry;
}

// Stable scatter of one block of IPT * 256 items.  Wave w takes the block's items
// [64 IPT w, 64 IPT (w + 1)) in order, 64 per round, so (wave, round, lane) order is
// input order.  Per round the lanes of a digit group take consecutive offsets after
// the wave's running count of that digit (the group's lowest lane advances it).
// The block's items are then placed in LDS in (digit, input) order and written out
// with thread t on items t, t + 256, ...: consecutive lanes write consecutive slots of
// a digit's run.
template <int IPT>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ kin, const int *__restrict__ vin, int n, const long long *__restrict__ n_dev,
    int shift, bool drop, long long *__restrict__ n_out, int nb, const int *__restrict__ hist,
    const int *__restrict__ totals, uint32_t *__restrict__ kout, int *__restrict__ vout) {
    constexpr int kItems = kSortThreads * IPT;
    n = items_of(n, n_dev);
    const long b0 = (long)blockIdx.x * kItems;
    if (b0 >= n) return;   // the whole block: past the items
    __shared__ uint32_t s_key[kItems];
    __shared__ int s_val[kItems];
    __shared__ int s_cnt[4][256];   // per wave and digit: running count, then the wave's first slot
    __shared__ int s_dst[256];      // per digit: global slot of block slot 0 of the digit's run
    __shared__ int s_scan[256];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int cnt = (int)min((long)kItems, n - b0);
    for (int w = 0; w < 4; ++w) s_cnt[w][t] = 0;
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[IPT];
    int val[IPT], off[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int j = wave * 64 * IPT + r * 64 + lane;
        const bool valid = j < cnt;
        key[r] = valid ? kin[b0 + j] : 0u;
        val[r] = valid ? vin[b0 + j] : 0;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const bool valid = wave * 64 * IPT + r * 64 + lane < cnt && !(drop && key[r] == kDropKey);
        const uint32_t d = (key[r] >> shift) & 255u;
        const uint64_t m = digit_peers(d, valid);
        const int lead = m ? __builtin_ctzll(m) : 0;
        int before = 0;
        if (valid && lane == lead) before = atomicAdd(&s_cnt[wave][d], __popcll(m));
        before = __shfl(before, lead);
        off[r] = before + __popcll(m & lt);
    }
    __syncthreads();
    int kept;   // the block's items that take part (all but dropped ones)
    {
        // digit t: the block's first slot of the digit, each wave's first slot within it,
        // and the global slot the block's run of the digit starts at
        const int c0 = s_cnt[0][t], c1 = s_cnt[1][t], c2 = s_cnt[2][t], c3 = s_cnt[3][t];
        const int start = block_exscan256(c0 + c1 + c2 + c3, s_scan, kept);
        s_cnt[0][t] = start;
        s_cnt[1][t] = start + c0;
        s_cnt[2][t] = start + c0 + c1;
        s_cnt[3][t] = start + c0 + c1 + c2;
        int all;
        const int gstart = block_exscan256(totals[t], s_scan, all);
        s_dst[t] = gstart + hist[t * nb + blockIdx.x] - start;
        if (n_out && blockIdx.x == 0 && t == 0) *n_out = all;   // the items the pass kept
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        if (wave * 64 * IPT + r * 64 + lane < cnt && !(drop && key[r] == kDropKey)) {
            const int p = s_cnt[wave][(key[r] >> shift) & 255u] + off[r];
            s_key[p] = key[r];
            s_val[p] = val[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const int i = r * kSortThreads + t;
        if (i < kept) {
            const uint32_t k = s_key[i];
            const int dst = s_dst[(k >> shift) & 255u] + i;
            kout[dst] = k;
            vout[dst] = s_val[i];
        }
    }
}

// ---------------------------------------------------------------- int64 scan

// Pair counts in depth order; the entries past the kept records (n_kept) count zero.
__global__ __launch_bounds__(256) void gather_counts_kernel(int n, const long long *__restrict__ n_kept,
                                                            const int *__restrict__ order,
                                                            const int *__restrict__ touched,
                                                            long long *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = i < items_of(n, n_kept) ? touched[order[i]] : 0;
}

__global__ __launch_bounds__(256) void scan_partial_kernel(const long long *__restrict__ in, long n,
                                                           long long *__restrict__ sums) {
    __shared__ long long lds[256];
    long base = (long)blockIdx.x * kScanItems;
    long long s = 0;
    for (int j = 0; j < kScanItems / 256; ++j) {
        long i = base + j * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    long long tot;
    block_exscan256(s, lds, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(long long *__restrict__ sums, int nb,
                                                        long long *__restrict__ total) {
    __shared__ long long lds[256];
    long long carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        int i = b0 + threadIdx.x;
        long long v = i < nb ? sums[i] : 0;
        long long tot;
        long long ex = block_exscan256(v, lds, tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Thread t scans 16 consecutive items of the block's 4096.  The items pass through LDS
// so that every global load and store is coalesced (item k at k + k / 16: one pad
// word per 16 keeps a thread's run off its neighbours' banks).
constexpr int kScanPer = kScanItems / 256;
__device__ __forceinline__ int scan_slot(int k) { return k + k / kScanPer; }

__global__ __launch_bounds__(256) void scan_final_kernel(const long long *__restrict__ in, long n,
                                                         const long long *__restrict__ sums,
                                                         long long *__restrict__ out) {
    __shared__ long long lds[256];
    __shared__ long long stage[kScanItems + kScanItems / kScanPer];
    const int t = threadIdx.x;
    const long base = (long)blockIdx.x * kScanItems;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int k = j * 256 + t;
        stage[scan_slot(k)] = base + k < n ? in[base + k] : 0;
    }
    __syncthreads();
    long long v[kScanPer];
    long long s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = stage[scan_slot(t * kScanPer + j)];
        s += v[j];
    }
    long long tot;
    long long run = block_exscan256(s, lds, tot) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        stage[scan_slot(t * kScanPer + j)] = run;   // only this thread reads these slots back
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int k = j * 256 + t;
        if (base + k < n) out[base + k] = stage[scan_slot(k)];
    }
}

// Writes the (tile, id) pairs of 256 consecutive Gaussians (depth order) per block.
// The block's pairs are dealt out evenly over its threads: pair q belongs to the
// last Gaussian whose first pair is at or before q (binary search in LDS), so a
// Gaussian covering hundreds of tiles does not hold up its wave.
// Records of several views are binned together: record r belongs to view r / n_view,
// whose tiles take keys view * T + tile, so one stable sort orders (view, tile).
__global__ __launch_bounds__(256) void duplicate_kernel(int n, const long long *__restrict__ n_kept,
                                                        const int *__restrict__ order,
                                                        const long long *__restrict__ offs,
                                                        const int4 *__restrict__ rect,
                                                        const int *__restrict__ touched, int ntx,
                                                        int n_view, int T, long long max_pairs,
                                                        uint32_t *__restrict__ tile_keys,
                                                        int *__restrict__ ids) {
    __shared__ int s_start[256];
    __shared__ int s_g[256];
    __shared__ int s_key0[256];   // the key of the record's first tile: view * T + y0 * ntx + x0
    __shared__ int s_rw[256];     // its box width in tiles, and the width's reciprocal
    __shared__ float s_inv[256];
    __shared__ long long s_base;
    __shared__ int s_total;
    n = items_of(n, n_kept);   // the records the depth sort kept
    const int t = threadIdx.x;
    const int s = blockIdx.x * 256 + t;
    int g = -1, c = 0;
    long long o = 0;
    int4 r = make_int4(0, 0, 1, 1);
    if (s < n) {
        g = order[s];
        c = max(touched[g], 0);
        o = offs[s];
        if (c > 0) r = rect[g];
    }
    if (t == 0) {
        s_base = o;   // the block's first Gaussian always exists
        s_total = 0;
    }
    __syncthreads();
    const int start = s < n ? (int)(o - s_base) : 0x7FFFFFFF;
    s_start[t] = start;
    s_g[t] = g;
    s_key0[t] = g >= 0 ? (g / n_view) * T + r.y * ntx + r.x : 0;
    s_rw[t] = r.z - r.x;
    s_inv[t] = 1.0f / (float)(r.z - r.x);
    if (s < n) atomicMax(&s_total, start + c);
    __syncthreads();
    const int total = s_total;
    const long long base = s_base;
    const int lim = (int)min((long long)total, max_pairs - base);   // never past the buffers
    // four pairs per thread and round, their owner searches interleaved (eight
    // fixed steps each: the largest j with s_start[j] <= q; s_start[0] = 0)
    constexpr int kU = 4;
    for (int q0 = t; q0 < lim; q0 += kU * 256) {
        int lo[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) lo[u] = 0;
#pragma unroll
        for (int step = 128; step > 0; step >>= 1)
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (s_start[lo[u] + step] <= q0 + u * 256) lo[u] += step;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int q = q0 + u * 256;
            if (q >= lim) break;
            const int j = lo[u];
            const int k = q - s_start[j];   // the pair's tile within the record's box, row by row
            const int rw = s_rw[j];
            // dy = k / rw: the float product is within 0.5 of it for k < 2^22 (a box of at
            // most a view's tiles), the integer steps make it exact for any k
            int dy = (int)((float)k * s_inv[j]);
            while (dy * rw > k) --dy;
            while ((dy + 1) * rw <= k) ++dy;
            tile_keys[base + q] = (uint32_t)(s_key0[j] + dy * ntx + (k - dy * rw));
            ids[base + q] = s_g[j];
        }
    }
}

__global__ __launch_bounds__(256) void zero_ranges_kernel(int n2, int *__restrict__ ranges) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n2) ranges[i] = 0;
}

// Run boundaries of the sorted tile keys; keys outside [0, T) (a caller's box past the
// tile grid) mark nothing.
// Each thread takes four consecutive keys (one 16-byte load; keys 16-byte aligned) and
// their two neighbours.
__global__ __launch_bounds__(256) void mark_ranges_kernel(int m, const long long *__restrict__ m_dev,
                                                          const uint32_t *__restrict__ keys, uint32_t T,
                                                          int *__restrict__ ranges) {
    m = items_of(m, m_dev);
    const long i0 = ((long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= m) return;
    uint32_t k[6];   // keys i0 - 1 .. i0 + 4 (the ends are only read inside [0, m))
    k[0] = i0 > 0 ? keys[i0 - 1] : 0u;
    if (i0 + 4 <= m) {
        const uint4 v = *(const uint4 *)(keys + i0);
        k[1] = v.x; k[2] = v.y; k[3] = v.z; k[4] = v.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < m ? keys[i0 + j] : 0u;
    }
    k[5] = i0 + 4 < m ? keys[i0 + 4] : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const long i = i0 + j;
        const uint32_t kk = k[1 + j];
        if (i >= m || kk >= T) continue;
        if (i == 0 || k[j] != kk) ranges[2 * kk] = (int)i;
        if (i == m - 1 || k[2 + j] != kk) ranges[2 * kk + 1] = (int)(i + 1);
    }
}

// ---------------------------------------------------------------- host side

struct Layout {
    size_t dk0, dv0, dk1, dv1, cnt, offs, sums, total, kept, hist, totals, pk0, pk1, pv1, bytes;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_of(long n, long max_pairs) {
    Layout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t o = at;
        at = align256(at + bytes);
        return o;
    };
    long items = n > max_pairs ? n : max_pairs;
    long nb_sort = (items + kSortItems - 1) / kSortItems;
    long nb_scan = (n + kScanItems - 1) / kScanItems;
    L.dk0 = take(4 * (size_t)n);
    L.dv0 = take(4 * (size_t)n);
    L.dk1 = take(4 * (size_t)n);
    L.dv1 = take(4 * (size_t)n);
    L.cnt = take(8 * (size_t)n);
    L.offs = take(8 * (size_t)n);
    L.sums = take(8 * (size_t)(nb_scan + 1));
    L.total = take(8);
    L.kept = take(8);
    L.hist = take(4 * 256 * (size_t)(nb_sort + 1));
    L.totals = take(4 * 256);
    L.pk0 = take(4 * (size_t)max_pairs);
    L.pk1 = take(4 * (size_t)max_pairs);
    L.pv1 = take(4 * (size_t)max_pairs);
    L.bytes = at;
    return L;
}

// One stable LSD pass over bits [shift, shift + 8) of n items (min(n, *n_dev) if
// n_dev is given: the grid is sized for n).
template <int IPT>
void radix_launch(const uint32_t *kin, const int *vin, uint32_t *kout, int *vout, int n, const long long *n_dev,
                  int shift, bool drop, long long *n_out, int *hist, int *totals, hipStream_t st) {
    const int nb = (int)(((long)n + kSortThreads * IPT - 1) / (kSortThreads * IPT));
    hipLaunchKernelGGL(radix_hist_kernel<IPT>, dim3(nb), dim3(kSortThreads), 0, st, kin, n, n_dev, shift, drop, nb,
                       hist);
    hipLaunchKernelGGL(radix_scan_digits_kernel, dim3(256), dim3(256), 0, st, hist, nb, totals);
    hipLaunchKernelGGL(radix_scatter_kernel<IPT>, dim3(nb), dim3(kSortThreads), 0, st, kin, vin, n, n_dev, shift,
                       drop, n_out, nb, hist, totals, kout, vout);
}

// drop: items keyed kDropKey leave the sort (n_out, if given, receives the kept count).
lgs_status radix_pass(const uint32_t *kin, const int *vin, uint32_t *kout, int *vout, int n,
                      const long long *n_dev, int shift, int *hist, int *totals, hipStream_t st,
                      bool drop = false, long long *n_out = nullptr) {
    if (n >= kBigPass)
        radix_launch<kSortIptBig>(kin, vin, kout, vout, n, n_dev, shift, drop, n_out, hist, totals, st);
    else
        radix_launch<kSortIpt>(kin, vin, kout, vout, n, n_dev, shift, drop, n_out, hist, totals, st);
    return check_launch("radix pass");
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_bin_sort_workspace(int32_t n, int32_t width, int32_t height,
                                             int64_t max_pairs, size_t *bytes) {
    LGS_REQUIRE(bytes, LGS_ERR_INVALID_ARG, "bytes is NULL");
    LGS_REQUIRE(n >= 0 && width > 0 && height > 0 && max_pairs >= 0 && max_pairs <= 0x7FFFFFFF,
                LGS_ERR_INVALID_ARG, "lgs_bin_sort_workspace: bad sizes");
    *bytes = layout_of(n, max_pairs).bytes;
    return LGS_OK;
}

namespace lgs {
namespace {

// The binning of lgs_bin_sort over the workspace `workspace` (ws_bytes usable bytes),
// for `views` views of n_view records each (views * n_view = n records, view-major).
lgs_status bin_sort_on(const lgs_camera *cam, int32_t views, int32_t n_view, const float *depth,
                       const int32_t *tile_rect, const int32_t *tiles_touched, void *workspace, size_t ws_bytes,
                       int64_t max_pairs, int32_t *sorted_ids, int32_t *tile_ranges, int64_t *n_pairs,
                       hipStream_t stream) {
    lgs_status st = check_camera(cam);
    if (st) return st;
    LGS_REQUIRE(views >= 1 && n_view >= 0 && (long long)views * n_view <= 0x7FFFFFFF && max_pairs >= 0 &&
                    max_pairs <= 0x7FFFFFFF,
                LGS_ERR_INVALID_ARG, "lgs_bin_sort: bad sizes");
    LGS_REQUIRE(tile_ranges, LGS_ERR_INVALID_ARG, "tile_ranges is NULL");
    const int n = views * n_view;
    const int ntx = tiles_x(cam->width), nty = tiles_y(cam->height);
    const int T1 = ntx * nty;                 // tiles of one view
    LGS_REQUIRE((long long)views * T1 <= (1LL << 29), LGS_ERR_INVALID_ARG, "too many tiles");
    const int T = views * T1;                 // tiles of all views
    if (n == 0) {
        hipLaunchKernelGGL(zero_ranges_kernel, dim3((2 * T + 255) / 256), dim3(256), 0, stream,
                           2 * T, tile_ranges);
        if (n_pairs) *n_pairs = 0;
        return check_launch("bin_sort zero");
    }
    LGS_REQUIRE(depth && tile_rect && tiles_touched && workspace && (sorted_ids || max_pairs == 0),
                LGS_ERR_INVALID_ARG, "lgs_bin_sort: NULL pointer");
    LGS_REQUIRE(((uintptr_t)workspace & 255u) == 0, LGS_ERR_INVALID_ARG,
                "workspace must be 256-byte aligned");
    LGS_REQUIRE(aligned16(tile_rect), LGS_ERR_INVALID_ARG, "tile_rect must be 16-byte aligned");
    Layout L = layout_of(n, max_pairs);
    LGS_REQUIRE(ws_bytes >= L.bytes, LGS_ERR_INVALID_ARG, "workspace too small: %zu < %zu", ws_bytes,
                L.bytes);
    char *ws = (char *)workspace;
    uint32_t *dk0 = (uint32_t *)(ws + L.dk0), *dk1 = (uint32_t *)(ws + L.dk1);
    int *dv0 = (int *)(ws + L.dv0), *dv1 = (int *)(ws + L.dv1);
    long long *cnt = (long long *)(ws + L.cnt), *offs = (long long *)(ws + L.offs);
    long long *sums = (long long *)(ws + L.sums), *total = (long long *)(ws + L.total);
    long long *kept = (long long *)(ws + L.kept);
    int *hist = (int *)(ws + L.hist), *totals = (int *)(ws + L.totals);

    // 1. sort Gaussians by depth key (4 passes of 8 bits), ending in dk0/dv0; the first
    // pass drops the records that touch no tile, the later ones sort the kept count
    unsigned g1 = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(depth_keys_kernel, dim3(g1), dim3(256), 0, stream, n, depth, tiles_touched,
                       dk0, dv0);
    for (int pass = 0; pass < 4; ++pass) {
        bool even = (pass & 1) == 0;
        st = radix_pass(even ? dk0 : dk1, even ? dv0 : dv1, even ? dk1 : dk0, even ? dv1 : dv0, n,
                        pass == 0 ? nullptr : kept, 8 * pass, hist, totals, stream, pass == 0,
                        pass == 0 ? kept : nullptr);
        if (st) return st;
    }
    // 2. pair offsets in depth order
    hipLaunchKernelGGL(gather_counts_kernel, dim3(g1), dim3(256), 0, stream, n, kept, dv0, tiles_touched,
                       cnt);
    int nbs = (n + kScanItems - 1) / kScanItems;
    hipLaunchKernelGGL(scan_partial_kernel, dim3(nbs), dim3(256), 0, stream, cnt, (long)n, sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, stream, sums, nbs, total);
    hipLaunchKernelGGL(scan_final_kernel, dim3(nbs), dim3(256), 0, stream, cnt, (long)n, sums, offs);
    st = check_launch("bin_sort scan");
    if (st) return st;
    // the pair count: read back once (n_pairs given), or left on the device, where the
    // remaining launches take it from (grids sized for max_pairs)
    long long M = max_pairs;
    const long long *M_dev = nullptr;
    if (n_pairs) {
        st = check_hip(hipMemcpyAsync(&M, total, sizeof(M), hipMemcpyDeviceToHost, stream), "pair count copy");
        if (st) return st;
        st = check_hip(hipStreamSynchronize(stream), "pair count sync");
        if (st) return st;
        *n_pairs = M;
        if (M > max_pairs) {
            set_error("lgs_bin_sort: %lld pairs exceed max_pairs %lld", M, (long long)max_pairs);
            return LGS_ERR_CAPACITY;
        }
    } else {
        M_dev = total;
    }
    hipLaunchKernelGGL(zero_ranges_kernel, dim3((2 * T + 255) / 256), dim3(256), 0, stream, 2 * T,
                       tile_ranges);
    if (M == 0) return check_launch("bin_sort zero");
    // 3. duplicate into (tile, id) pairs in depth order, then stable sort by tile
    int tile_bits = 0;
    while ((1 << tile_bits) < T) ++tile_bits;
    int passes = (tile_bits + 7) / 8;
    uint32_t *pk0 = (uint32_t *)(ws + L.pk0), *pk1 = (uint32_t *)(ws + L.pk1);
    int *pv1 = (int *)(ws + L.pv1);
    // the last pass must land in sorted_ids: start there if the pass count is even
    int *pv0 = sorted_ids;
    uint32_t *kcur = pk0, *knext = pk1;
    int *vcur = (passes % 2 == 0) ? pv0 : pv1, *vnext = (passes % 2 == 0) ? pv1 : pv0;
    hipLaunchKernelGGL(duplicate_kernel, dim3(g1), dim3(256), 0, stream, n, kept, dv0, offs,
                       (const int4 *)tile_rect, tiles_touched, ntx, n_view > 0 ? n_view : 1, T1,
                       (long long)max_pairs, kcur, vcur);
    st = check_launch("bin_sort duplicate");
    if (st) return st;
    for (int pass = 0; pass < passes; ++pass) {
        st = radix_pass(kcur, vcur, knext, vnext, (int)M, M_dev, 8 * pass, hist, totals, stream);
        if (st) return st;
        uint32_t *tk = kcur; kcur = knext; knext = tk;
        int *tv = vcur; vcur = vnext; vnext = tv;
    }
    hipLaunchKernelGGL(mark_ranges_kernel, dim3((unsigned)((M + 1023) / 1024)), dim3(256), 0, stream,
                       (int)M, M_dev, kcur, (uint32_t)T, tile_ranges);
    return check_launch("bin_sort ranges");
}

}  // namespace
}  // namespace lgs

extern "C" lgs_status lgs_bin_sort(const lgs_camera *cam, int32_t n, const float *depth,
                                   const int32_t *tile_rect, const int32_t *tiles_touched,
                                   void *workspace, size_t ws_bytes, int64_t max_pairs,
                                   int32_t *sorted_ids, int32_t *tile_ranges, int64_t *n_pairs,
                                   hipStream_t stream) {
    return bin_sort_on(cam, 1, n, depth, tile_rect, tiles_touched, workspace, ws_bytes, max_pairs, sorted_ids,
                       tile_ranges, n_pairs, stream);
}

extern "C" lgs_status lgs_bin_sort_views(const lgs_camera *cams, int32_t views, int32_t n, const float *depth,
                                         const int32_t *tile_rect, const int32_t *tiles_touched, void *workspace,
                                         size_t ws_bytes, int64_t max_pairs, int32_t *sorted_ids,
                                         int32_t *tile_ranges, int64_t *n_pairs, hipStream_t stream) {
    LGS_REQUIRE(cams && views >= 1, LGS_ERR_INVALID_ARG, "lgs_bin_sort_views: no cameras");
    for (int v = 1; v < views; ++v)
        LGS_REQUIRE(cams[v].width == cams[0].width && cams[v].height == cams[0].height, LGS_ERR_INVALID_ARG,
                    "batched views share the image size");
    return bin_sort_on(cams, views, n, depth, tile_rect, tiles_touched, workspace, ws_bytes, max_pairs, sorted_ids,
                       tile_ranges, n_pairs, stream);
}

extern "C" lgs_status lgs_bin_sort_count(int32_t n, int64_t max_pairs, const void *workspace, int64_t *n_pairs,
                                         hipStream_t stream) {
    LGS_REQUIRE(n_pairs && workspace, LGS_ERR_INVALID_ARG, "lgs_bin_sort_count: NULL pointer");
    LGS_REQUIRE(n >= 0 && max_pairs >= 0 && max_pairs <= 0x7FFFFFFF, LGS_ERR_INVALID_ARG,
                "lgs_bin_sort_count: bad sizes");
    if (n == 0) {
        *n_pairs = 0;
        return LGS_OK;
    }
    const Layout L = layout_of(n, max_pairs);
    long long M = 0;
    lgs_status st = check_hip(hipMemcpyAsync(&M, (const char *)workspace + L.total, sizeof(M),
                                             hipMemcpyDeviceToHost, stream), "pair count copy");
    if (st) return st;
    st = check_hip(hipStreamSynchronize(stream), "pair count sync");
    if (st) return st;
    *n_pairs = M;
    if (M > max_pairs) {
        set_error("lgs_bin_sort: %lld pairs exceed max_pairs %lld", M, (long long)max_pairs);
        return LGS_ERR_CAPACITY;
    }
    return LGS_OK;
}

// ---------------------------------------------------------------- allocation-free variant
//
// lgs_bin_sort_noalloc bins exactly as lgs_bin_sort, with its workspace in a static
// device array instead of caller memory.  Each GPU the library runs on holds its own
// copy of the array from the module's load until the process ends.  In host code the
// array's name is only a host-side stand-in, never a device address: the device address
// is looked up once per device with hipGetSymbolAddress and used from then on.

namespace lgs {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first call per
// device (with that device current) and kept.
lgs_status scratch_of_current_device(void **out) {
    int dev = -1;
    lgs_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    LGS_REQUIRE(dev >= 0 && dev < kMaxDevices, LGS_ERR_INVALID_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st) return st;
        LGS_REQUIRE(p != nullptr, LGS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LGS_OK;
}

}  // namespace
}  // namespace lgs

extern "C" lgs_status lgs_bin_sort_noalloc(const lgs_camera *cam, int32_t n, const float *depth,
                                           const int32_t *tile_rect, const int32_t *tiles_touched,
                                           int64_t max_pairs, int32_t *sorted_ids, int32_t *tile_ranges,
                                           int64_t *n_pairs, hipStream_t stream) {
    lgs_status st = check_camera(cam);
    if (st) return st;
    LGS_REQUIRE(n_pairs, LGS_ERR_INVALID_ARG, "lgs_bin_sort_noalloc: n_pairs (host) is required");
    LGS_REQUIRE(n >= 0 && max_pairs >= 0 && max_pairs <= 0x7FFFFFFF, LGS_ERR_INVALID_ARG,
                "lgs_bin_sort_noalloc: bad sizes");
    const size_t need = layout_of(n, max_pairs).bytes;
    LGS_REQUIRE(need <= kScratchBytes, LGS_ERR_INVALID_ARG,
                "lgs_bin_sort_noalloc: n = %d with max_pairs = %lld needs %zu bytes of scratch; the static "
                "scratch holds %zu (use lgs_bin_sort with a workspace)",
                n, (long long)max_pairs, need, kScratchBytes);
    void *ws = nullptr;
    st = scratch_of_current_device(&ws);
    if (st) return st;
    return bin_sort_on(cam, 1, n, depth, tile_rect, tiles_touched, ws, kScratchBytes, max_pairs, sorted_ids,
                       tile_ranges, n_pairs, stream);
}
