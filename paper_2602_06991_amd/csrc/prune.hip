// Weighted survival sampling of the semantic-geometric consistency pruning (Sec. 3.3,
// Eq. 6).  Candidates are the Gaussians with few Top-K selections; of them a fixed
// share survives, drawn without replacement with probabilities proportional to the
// geometric importance S_i.  The draw uses exponential keys: with E_i ~ Exp(1) drawn
// by the caller, the candidates with the smallest E_i / S_i are exactly a weighted
// sample without replacement (each successive pick takes candidate i with probability
// S_i over the S of those left; the first pick is Eq. 6 itself).
//
// Keys are the quotients rounded to FP32 and compared as their bit patterns
// (non-negative, so the bits order like the values); S_i = 0 gives +inf.  The m-th
// smallest key is found by an MSB-first radix select over four 8-bit digits (a
// histogram launch and a one-block digit pick per digit, all on the device), and equal
// keys at the threshold are kept in index order, counted by a block scan.
#include "lgs_device.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

constexpr int kSelItems = 1024;   // items per block of the tie count and marking
constexpr uint32_t kInfKey = 0x7F800000u;

// state words: 0 candidates, 1 m, 2 key prefix chosen so far, 3 how many of the
// candidates holding that prefix still survive; then the digit histogram [256]
constexpr int kStCand = 0, kStM = 1, kStPrefix = 2, kStLeft = 3, kStHist = 4, kStWords = kStHist + 256;

// The key is the correctly rounded FP32 quotient e / s (IEEE division, which hipcc
// emits for FP32 '/' by default and the build requests explicitly), so every
// implementation that rounds the exact quotient once to FP32 gets the same key bits.
__device__ __forceinline__ uint32_t sel_key(float e, float s) {
    return s > 0.f ? __float_as_uint(e / s) : kInfKey;
}

__global__ __launch_bounds__(256) void sel_reset_kernel(int *__restrict__ st) {
    for (int i = threadIdx.x; i < kStWords; i += 256) st[i] = 0;
}

__global__ __launch_bounds__(256) void sel_count_kernel(int n, const int *__restrict__ count, int below,
                                                        int *__restrict__ st) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int c = 0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) c += count[i] < below;
    if (c) atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0 && s) atomicAdd(&st[kStCand], s);
}

// m = floor(keep_ratio * candidates), exactly: keep_ratio = sig 2^-sh with an integer
// significand sig < 2^24 and sh >= 23 (keep_ratio <= 1), so the product is the 64-bit
// integer sig * c shifted right by sh (c < 2^31, the product < 2^55).
__global__ void sel_setup_kernel(uint32_t sig, int sh, int *__restrict__ st) {
    if (threadIdx.x != 0) return;
    const unsigned long long prod = (unsigned long long)sig * (unsigned long long)(uint32_t)st[kStCand];
    const int m = sh >= 64 ? 0 : (int)(prod >> sh);
    st[kStM] = m;
    st[kStLeft] = m;
    st[kStPrefix] = 0;
}

// Histogram of digit (key >> shift) & 255 over the candidates whose higher digits
// equal the chosen prefix.
__global__ __launch_bounds__(256) void sel_hist_kernel(int n, const int *__restrict__ count, int below,
                                                       const float *__restrict__ maxw,
                                                       const float *__restrict__ expo, int shift,
                                                       int *__restrict__ st) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t prefix = (uint32_t)st[kStPrefix];
    const bool top = shift == 24;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        if (count[i] >= below) continue;
        const uint32_t k = sel_key(expo[i], maxw[i]);
        if (!top && (k >> (shift + 8)) != (prefix >> (shift + 8))) continue;
        atomicAdd(&h[(k >> shift) & 255u], 1);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&st[kStHist + threadIdx.x], h[threadIdx.x]);
}

// One block: the digit whose bucket holds the remaining survivor count's boundary.
__global__ __launch_bounds__(256) void sel_pick_kernel(int shift, int *__restrict__ st) {
    __shared__ int sc[256];
    const int t = threadIdx.x;
    const int c = st[kStHist + t];
    sc[t] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? sc[t - off] : 0;
        __syncthreads();
        sc[t] += x;
        __syncthreads();
    }
    const int before = sc[t] - c;
    const int left = st[kStLeft];
    __syncthreads();
    st[kStHist + t] = 0;   // cleared for the next digit
    if (left > 0 && before < left && left <= before + c) {
        st[kStPrefix] = (int)((uint32_t)st[kStPrefix] | ((uint32_t)t << shift));
        st[kStLeft] = left - before;
    }
}

// Per block of kSelItems indices: how many candidates hold exactly the threshold key.
__global__ __launch_bounds__(256) void sel_ties_kernel(int n, const int *__restrict__ count, int below,
                                                       const float *__restrict__ maxw,
                                                       const float *__restrict__ expo,
                                                       const int *__restrict__ st, int *__restrict__ ties) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    const uint32_t kt = (uint32_t)st[kStPrefix];
    int c = 0;
    for (int r = 0; r < kSelItems / 256; ++r) {
        const long i = (long)blockIdx.x * kSelItems + r * 256 + threadIdx.x;
        if (i < n && count[i] < below && sel_key(expo[i], maxw[i]) == kt) ++c;
    }
    if (c) atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) ties[blockIdx.x] = s;
}

// One block: exclusive scan of the per-block tie counts, in place.
__global__ __launch_bounds__(256) void sel_ties_scan_kernel(int nb, int *__restrict__ ties) {
    __shared__ int sc[256];
    const int t = threadIdx.x;
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int v = b0 + t < nb ? ties[b0 + t] : 0;
        sc[t] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int x = t >= off ? sc[t - off] : 0;
            __syncthreads();
            sc[t] += x;
            __syncthreads();
        }
        if (b0 + t < nb) ties[b0 + t] = carry + sc[t] - v;
        carry += sc[255];
        __syncthreads();
    }
}

// survive[i] = 1 for non-candidates, for candidates below the threshold key, and for
// the first `left` candidates (by index) at the threshold key.
__global__ __launch_bounds__(256) void sel_mark_kernel(int n, const int *__restrict__ count, int below,
                                                       const float *__restrict__ maxw,
                                                       const float *__restrict__ expo,
                                                       const int *__restrict__ st, const int *__restrict__ ties,
                                                       uint8_t *__restrict__ survive) {
    __shared__ int sc[256];
    const int t = threadIdx.x;
    const uint32_t kt = (uint32_t)st[kStPrefix];
    const int m = st[kStM], left = st[kStLeft];
    // the thread's four consecutive indices, so the tie rank follows index order
    const long i0 = (long)blockIdx.x * kSelItems + 4L * t;
    uint8_t cand[4];
    uint32_t key[4];
    int tie = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long i = i0 + r;
        cand[r] = i < n && count[i] < below;
        key[r] = cand[r] ? sel_key(expo[i], maxw[i]) : 0u;
        tie += cand[r] && key[r] == kt;
    }
    sc[t] = tie;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int x = t >= off ? sc[t - off] : 0;
        __syncthreads();
        sc[t] += x;
        __syncthreads();
    }
    int rank = ties[blockIdx.x] + sc[t] - tie;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long i = i0 + r;
        if (i >= n) break;
        uint8_t keep = 1;
        if (cand[r]) {
            if (m == 0) keep = 0;
            else if (key[r] < kt) keep = 1;
            else if (key[r] == kt) keep = rank++ < left;
            else keep = 0;
        }
        survive[i] = keep;
    }
}

struct SelLayout {
    size_t state, ties, bytes;
    long nb;
};

SelLayout sel_layout(long n) {
    SelLayout L;
    L.nb = (n + kSelItems - 1) / kSelItems;
    L.state = 0;
    L.ties = 256 * ((4 * kStWords + 255) / 256);
    L.bytes = L.ties + 4 * (size_t)(L.nb > 0 ? L.nb : 1);
    return L;
}

inline unsigned sel_grid(long n) { return (unsigned)std::max(1L, std::min(1024L, (n + 4095) / 4096)); }

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_prune_select_workspace(int32_t n, size_t *bytes) {
    LGS_REQUIRE(bytes && n >= 0, LGS_ERR_INVALID_ARG, "lgs_prune_select_workspace: bad arguments");
    *bytes = sel_layout(n).bytes;
    return LGS_OK;
}

extern "C" lgs_status lgs_prune_select(int32_t n, const int32_t *topk_count, const float *max_w,
                                       int32_t count_below, const float *expo, float keep_ratio,
                                       void *workspace, size_t ws_bytes, uint8_t *survive, hipStream_t stream) {
    LGS_REQUIRE(n >= 0, LGS_ERR_INVALID_ARG, "lgs_prune_select: n < 0");
    LGS_REQUIRE(keep_ratio >= 0.f && keep_ratio <= 1.f, LGS_ERR_INVALID_ARG,
                "lgs_prune_select: keep_ratio must lie in [0, 1]");
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(topk_count && max_w && expo && workspace && survive, LGS_ERR_INVALID_ARG,
                "lgs_prune_select: NULL pointer");
    const SelLayout L = sel_layout(n);
    LGS_REQUIRE(ws_bytes >= L.bytes, LGS_ERR_INVALID_ARG, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    LGS_REQUIRE(((uintptr_t)workspace & 255u) == 0, LGS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    int *st = (int *)((char *)workspace + L.state);
    int *ties = (int *)((char *)workspace + L.ties);
    // keep_ratio = sig 2^-sh exactly (a normal float is (2^23 + mantissa) 2^(e - 150), a
    // subnormal one mantissa 2^-149)
    const uint32_t bits = __builtin_bit_cast(uint32_t, keep_ratio);
    const uint32_t ex = (bits >> 23) & 0xFFu, man = bits & 0x7FFFFFu;
    const uint32_t sig = ex ? (man | 0x800000u) : man;
    const int sh = ex ? 150 - (int)ex : 149;
    const unsigned g = sel_grid(n);
    hipLaunchKernelGGL(sel_reset_kernel, dim3(1), dim3(256), 0, stream, st);
    hipLaunchKernelGGL(sel_count_kernel, dim3(g), dim3(256), 0, stream, n, topk_count, count_below, st);
    hipLaunchKernelGGL(sel_setup_kernel, dim3(1), dim3(64), 0, stream, sig, sh, st);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(sel_hist_kernel, dim3(g), dim3(256), 0, stream, n, topk_count, count_below, max_w, expo,
                           shift, st);
        hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, stream, shift, st);
    }
    hipLaunchKernelGGL(sel_ties_kernel, dim3((unsigned)L.nb), dim3(256), 0, stream, n, topk_count, count_below,
                       max_w, expo, st, ties);
    hipLaunchKernelGGL(sel_ties_scan_kernel, dim3(1), dim3(256), 0, stream, (int)L.nb, ties);
    hipLaunchKernelGGL(sel_mark_kernel, dim3((unsigned)L.nb), dim3(256), 0, stream, n, topk_count, count_below,
                       max_w, expo, st, ties, survive);
    return check_launch("prune_select");
}
