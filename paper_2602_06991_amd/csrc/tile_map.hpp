// Tile -> block map in strips over the XCDs, used by the blend kernels (unless the views
// come in eights), the pruning statistics, the vanilla feature render and the Top-K
// feature kernels; xcd_remap of lgs_device.hpp gives contiguous bands instead.
#pragma once
#include "lgs_device.hpp"

namespace lgs {

// For kernels whose tiles differ in work: strips of kStrip consecutive tiles, the strips
// dealt to the XCDs in turn (XCD x takes strips x, x + 8, ...).  Neighbours along a strip
// still meet in one L2, while every XCD gets an even share of the image; one contiguous
// range per XCD left the XCDs with up to 1.2x the mean work in the blend, and the
// feature kernels' tiles differ too (union sizes, the two MFMA forms).  Bijective on
// grids of strip_grid() blocks.
constexpr int kStrip = 16;
__device__ __forceinline__ int xcd_strips(int b) {
    const int x = b & 7, l = b >> 3;
    return ((l / kStrip) * 8 + x) * kStrip + (l % kStrip);
}
__host__ __device__ inline unsigned strip_grid(long long blocks) {
    const long long s = 8LL * kStrip;
    return (unsigned)(((blocks + s - 1) / s) * s);
}

}  // namespace lgs
