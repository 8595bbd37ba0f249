// Launch functions of the Top-K feature kernels, one explicit instantiation set per
// Top-K size in feature_k*.hip; the entry points in feature.hip dispatch to them.
#pragma once

#include <hip/hip_runtime.h>

#include "lgs.h"

namespace lgs {

enum { FT_F32 = 0, FT_BF16 = 1, FT_FP8 = 2 };   // feature storage
enum { MT_F32 = 0, MT_BF16 = 1 };                // feature map

#define LGS_FEATURE_FWD_PARAMS                                                                           \
    int, int, int, int, const void *, const float *, const int *, const float *, void *, hipStream_t
#define LGS_FEATURE_BWD_PARAMS                                                                           \
    int, int, int, int, const void *, const float *, const int *, const float *, const void *, float,    \
        float *, float *, void *, hipStream_t

// Render (Eq. 3-4) of views x W x H pixels into F (map dtype MT).
template <int K, int FT, int MT>
lgs_status feature_fwd_launch(int W, int H, int views, int D, const void *feat, const float *scale,
                              const int *ids, const float *tw, void *F, hipStream_t st);

// Adjoint; MODE 0: dF is dL/dF; 1: dF is the L1 target; 2: as 1 and the map goes to Fo.
template <int K, int FT, int MT, int MODE>
lgs_status feature_bwd_launch(int W, int H, int views, int D, const void *feat, const float *scale,
                              const int *ids, const float *tw, const void *dF, float l1_scale, float *dfeat,
                              float *dtw, void *Fo, hipStream_t st);

}  // namespace lgs
