/*
 * lgs.h - C ABI of the MI355X (gfx950) Top-K Gaussian-splatting renderer.
 *
 * The library renders colour, depth and opacity by front-to-back alpha blending
 * (Eq. 1 of LangGS-SLAM, arXiv 2602.06991, Sec. 3.1), keeps per pixel the K
 * Gaussians with the largest blending weights (Eq. 2, Sec. 3.2), renders the
 * D-dimensional language-feature map from those K alone (Eq. 3-4), and provides
 * the adjoint of every step for the joint optimisation of Sec. 3.4.
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless marked (host).  Arrays are row-major and
 *    contiguous.  Per-pixel arrays are indexed p = y * width + x ("pixel-major").
 *  - The caller owns every buffer.  The library never allocates device memory (its
 *    scratch lives in the workspaces the caller passes to lgs_bin_sort and
 *    lgs_prune_select) and never frees caller memory.
 *  - Every call is asynchronous on `stream` (it may be NULL, the default stream),
 *    except lgs_bin_sort (unless asked not to) and lgs_bin_sort_count, which read the
 *    pair count back to the host.
 *  - Gradient outputs ACCUMULATE (+=) unless stated; the caller zeroes them.
 *  - Arguments are validated on the host before any launch.  A failing call
 *    returns a negative lgs_status, launches nothing and leaves outputs untouched;
 *    lgs_last_error() then describes it.  No C++ exception crosses the ABI.
 *  - Calls are reentrant when they use distinct buffers and workspaces.
 *
 * Geometry conventions (readings of Sec. 3.1, which follows the 3DGS rasterizer):
 *  - Gaussians: mean (3), log-scale (3), rotation quaternion (w, x, y, z; need not be
 *    unit), opacity logit (o = sigmoid), RGB colour (3, no spherical harmonics).
 *  - Camera: world->camera [R|t] with OpenCV axes (x right, y down, z forward),
 *    pinhole fx, fy, cx, cy; pixel (x, y) has its centre at (x + 1/2, y + 1/2).
 *  - Depth key: the FP32 value fmaf(R22, mz, fmaf(R21, my, fmaf(R20, mx, t2))),
 *    correctly rounded at each step.  It is also the z used for the depth map.
 *  - Culled (never rendered, zero gradient): a non-finite parameter, an all-zero
 *    quaternion, a log-scale above 10, an opacity logit below -ln(254) (opacity
 *    under 1/255), or a depth key <= 0.2.
 *  - Projection: Sigma2D = J R Sigma R^T J^T + 0.3 I with the lateral position in J
 *    clamped to 1.3x the half field of view; conic = Sigma2D^-1 stored as (a, b, c)
 *    with sigma(d) = a dx^2/2 + b dx dy + c dy^2/2 for d = pixel centre - mean2D.
 *  - Blend: alpha = min(0.99, o exp(-sigma)); a Gaussian with alpha < 1/255 is
 *    skipped; blending stops BEFORE a Gaussian that would take the transmittance
 *    T (1 - alpha) below 1e-4.  Ties of the depth key blend in id order.
 *  - Top-K (Eq. 2): the K largest weights w = alpha T among the blended Gaussians,
 *    slot 0 the largest; equal weights keep blend order (smaller depth key, then
 *    smaller id).  Unused slots hold id -1 and weight 0.
 *  - Tiles are 16 x 16 pixels; results do not depend on the tiling.
 */
#ifndef LGS_H
#define LGS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LGS_ABI_VERSION 2
#define LGS_TILE 16

typedef enum {
    LGS_OK = 0,
    LGS_ERR_INVALID_ARG = -1,   /* null or misaligned pointer, bad size */
    LGS_ERR_UNSUPPORTED = -2,   /* K, D or dtype combination not compiled */
    LGS_ERR_CAPACITY = -3,      /* pair buffer too small; *n_pairs holds the need */
    LGS_ERR_HIP = -4            /* a HIP runtime call or launch failed */
} lgs_status;

typedef enum {
    LGS_F32 = 0,        /* IEEE binary32 */
    LGS_BF16 = 1,       /* bfloat16, round-to-nearest-even from FP32 */
    LGS_FP8_E4M3 = 2    /* OCP E4M3FN code + one FP32 scale per Gaussian row */
} lgs_dtype;

/* Host struct.  Rt: world->camera [R|t], 3x4 row-major. */
typedef struct {
    float Rt[12];
    float fx, fy, cx, cy;
    int32_t width, height;
} lgs_camera;

/* ABI version of the loaded library (LGS_ABI_VERSION at build time). */
int lgs_abi_version(void);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char *lgs_last_error(void);

/* Supported Top-K sizes, as a host array of *count entries (static storage). */
const int32_t *lgs_supported_k(int32_t *count);

/*
 * Projection (Sec. 3.1; the EWA splat of 3DGS), one thread per Gaussian.
 * In:  means[n*3], log_scales[n*3], quats[n*4] (w,x,y,z), opacity_logits[n], rgb[n*3].
 * Out: mean2d[n*2] (pixels), conic[n*3] (a,b,c), depth[n] (the depth key),
 *      opacity[n], tile_rect[n*4] = half-open tile box (tx0, ty0, tx1, ty1) that
 *      holds every pixel where alpha >= 1/255 (plus a one-pixel margin),
 *      tiles_touched[n] = (tx1-tx0)*(ty1-ty0), 0 for culled Gaussians.
 * Errors: INVALID_ARG for n < 0, a null pointer with n > 0, or a camera with
 * non-positive size or focal length.
 */
lgs_status lgs_project_fwd(const lgs_camera *cam, int32_t n,
                           const float *means, const float *log_scales, const float *quats,
                           const float *opacity_logits, const float *rgb,
                           float *mean2d, float *conic, float *depth, float *opacity,
                           int32_t *tile_rect, int32_t *tiles_touched, hipStream_t stream);

/*
 * Workspace bytes lgs_bin_sort needs for n Gaussians, an image of width x height and
 * room for max_pairs (tile, Gaussian) pairs.  *bytes is a host pointer.
 */
lgs_status lgs_bin_sort_workspace(int32_t n, int32_t width, int32_t height, int64_t max_pairs,
                                  size_t *bytes);

/*
 * Tile binning and depth sort (the tile-based rasterizer of 3DGS that Sec. 3.1
 * follows).  Every Gaussian is duplicated into each tile of its tile_rect; the pairs
 * are ordered by (tile, depth key, Gaussian id) with an on-device radix sort.
 * Out: sorted_ids[max_pairs] (the first *n_pairs are valid),
 *      tile_ranges[tiles*2] = [start, end) of every tile's run in sorted_ids,
 *      tiles = ceil(width/16) * ceil(height/16), tile index ty * ceil(width/16) + tx.
 * *n_pairs (host) receives the pair count.  If it exceeds max_pairs the call
 * returns LGS_ERR_CAPACITY with *n_pairs set to the need and the outputs
 * untouched: grow the buffers and call again.  This call synchronises `stream`
 * once to read the count.  workspace: ws_bytes >= lgs_bin_sort_workspace(...),
 * 256-byte aligned.
 * n_pairs may be NULL: the call is then fully asynchronous.  The count stays in the
 * workspace and the launches after the count take it from there (their grids are
 * sized for max_pairs); if the count exceeds max_pairs the outputs hold only the
 * first max_pairs pairs and are not a valid binning.  lgs_bin_sort_count reads the
 * count back later and reports that case.
 */
lgs_status lgs_bin_sort(const lgs_camera *cam, int32_t n, const float *depth,
                        const int32_t *tile_rect, const int32_t *tiles_touched,
                        void *workspace, size_t ws_bytes, int64_t max_pairs,
                        int32_t *sorted_ids, int32_t *tile_ranges, int64_t *n_pairs,
                        hipStream_t stream);

/*
 * The pair count of the last lgs_bin_sort on this workspace (same n and max_pairs),
 * for calls made with n_pairs = NULL.  Synchronises `stream`; *n_pairs is a host
 * pointer.  Returns LGS_ERR_CAPACITY if the count exceeded max_pairs (that call's
 * outputs are then not valid: grow the buffers and bin again).
 */
lgs_status lgs_bin_sort_count(int32_t n, int64_t max_pairs, const void *workspace, int64_t *n_pairs,
                              hipStream_t stream);

/*
 * Allocation-free variant of lgs_bin_sort, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same binning and outputs, with the workspace in a static device array
 * of the library (64 MiB per GPU, held from the library's load on that GPU until the
 * process ends) instead of caller memory.  It calls no allocator.
 * Limit: the workspace lgs_bin_sort_workspace(n, width, height, max_pairs) would report
 * must fit in 64 MiB (about 32 n + 12 max_pairs bytes), else INVALID_ARG before any
 * launch.  *n_pairs (host) is required: the call synchronises `stream` once to read
 * the pair count, and returns LGS_ERR_CAPACITY with *n_pairs set to the need (outputs
 * untouched) when it exceeds max_pairs.  Every call on one GPU shares that GPU's array
 * and overwrites it; calls that overlap on one GPU (other host threads, other streams)
 * race and must be serialised by the caller.  Nothing in the array needs to start at
 * zero: every word a call reads is written by that call first.
 */
lgs_status lgs_bin_sort_noalloc(const lgs_camera *cam, int32_t n, const float *depth,
                                const int32_t *tile_rect, const int32_t *tiles_touched,
                                int64_t max_pairs, int32_t *sorted_ids, int32_t *tile_ranges,
                                int64_t *n_pairs, hipStream_t stream);

/*
 * Colour/depth/opacity alpha blending (Eq. 1) that records the Top-K (Eq. 2) ids
 * and weights of every pixel during the same pass (Sec. 3.2, implementation).
 * In:  the projection outputs, rgb[n*3], and the lgs_bin_sort outputs.
 * Out: color[P*3], depth_map[P], alpha_map[P] (= 1 - T_final), T_final[P],
 *      n_contrib[P] (entries of the tile's sorted run up to and including the last
 *      blended Gaussian; the backward replays from there), topk_ids[P*k],
 *      topk_w[P*k] (raw weights w), with P = width * height.
 * tile_order: NULL (fixed tile mapping) or lgs_tile_order's output for these
 *      tile_ranges (dispatch order only: the outputs are the same bits).
 * Errors: UNSUPPORTED if k is not one of lgs_supported_k().
 */
lgs_status lgs_rasterize_topk_fwd(const lgs_camera *cam, int32_t k,
                                  const float *mean2d, const float *conic, const float *opacity,
                                  const float *rgb, const float *depth,
                                  const int32_t *sorted_ids, const int32_t *tile_ranges,
                                  float *color, float *depth_map, float *alpha_map,
                                  float *T_final, int32_t *n_contrib,
                                  int32_t *topk_ids, float *topk_w, const int32_t *tile_order,
                                  hipStream_t stream);

/*
 * Top-K feature render (Eq. 3-4): W = sum_k w_k, F[p] = sum_k (w_k / W) f[id_k],
 * F[p] = 0 where W = 0; FP32 accumulation, one rounding at the store.
 * feat[n*d] in feat_dt (FP32, BF16 or FP8 codes with feat_scale[n]: value =
 * code * scale); F[n_pix*d] in map_dt (FP32 or BF16).  Pixels are stacked views of
 * width x height images; n_pix = width * height * views.
 * Supported: (F32 -> F32), (BF16 -> BF16), (BF16 -> F32), (FP8 -> BF16), (FP8 -> F32).
 * d must be a positive multiple of 8; feat and F 16-byte aligned.
 */
lgs_status lgs_feature_render_fwd(int32_t width, int32_t height, int32_t views, int32_t k,
                                  int32_t d, lgs_dtype feat_dt, const void *feat,
                                  const float *feat_scale, const int32_t *topk_ids,
                                  const float *topk_w, lgs_dtype map_dt, void *F,
                                  hipStream_t stream);

/*
 * Adjoint of the feature render.  For every pixel with W > 0:
 *   g_k = <dL_dF[p], f_k>,  gamma_k = (g_k - sum_j w'_j g_j) / W,
 *   dL_dfeat[id_k] += (w_k / W) dL_dF[p]   (FP32, accumulated),
 *   dL_dtopkw[p*k + k'] = gamma_k          (overwritten; 0 where W = 0 or unused).
 * Same dtype and layout rules as the forward; dL_dF is in map_dt.
 */
lgs_status lgs_feature_render_bwd(int32_t width, int32_t height, int32_t views, int32_t k,
                                  int32_t d, lgs_dtype feat_dt, const void *feat,
                                  const float *feat_scale, const int32_t *topk_ids,
                                  const float *topk_w, lgs_dtype map_dt, const void *dL_dF,
                                  float *dL_dfeat, float *dL_dtopkw, hipStream_t stream);

/*
 * Feature adjoint fused with the L1 feature loss of Eq. 9: identical to
 * lgs_feature_render_bwd with dL/dF = scale * sign(F - F_target) (sign(0) = 0, the
 * scale rounded to map_dt), where F is recomputed from the Top-K rows exactly as
 * lgs_feature_render_fwd computes and rounds it.  Reads the target map instead of a
 * materialised dL/dF, so the loss gradient never travels through HBM.
 * F_target[n_pix*d] is in map_dt, 16-byte aligned.
 */
lgs_status lgs_feature_render_bwd_l1(int32_t width, int32_t height, int32_t views, int32_t k,
                                     int32_t d, lgs_dtype feat_dt, const void *feat,
                                     const float *feat_scale, const int32_t *topk_ids,
                                     const float *topk_w, lgs_dtype map_dt, const void *F_target,
                                     float scale, float *dL_dfeat, float *dL_dtopkw,
                                     hipStream_t stream);

/*
 * The feature render (Eq. 3-4) and its adjoint under the L1 feature loss of Eq. 9
 * in one pass over the Top-K records.  The outputs equal those of
 * lgs_feature_render_fwd followed by lgs_feature_render_bwd_l1 on the same inputs:
 * F is bit-identical to the forward's map, dL_dtopkw and the accumulated dL_dfeat
 * are those of the L1 adjoint.  The map is computed once and is both stored and
 * compared with the target, so one launch does the work of two.
 * Out: F[n_pix*d] (map_dt, overwritten), dL_dfeat[n*d] (FP32, accumulated),
 *      dL_dtopkw[n_pix*k] (overwritten).  In: F_target[n_pix*d] (map_dt).
 * Same dtype and layout rules as the forward; F and F_target are 16-byte aligned and
 * must not overlap (INVALID_ARG otherwise).
 */
lgs_status lgs_feature_render_fwd_bwd_l1(int32_t width, int32_t height, int32_t views, int32_t k,
                                         int32_t d, lgs_dtype feat_dt, const void *feat,
                                         const float *feat_scale, const int32_t *topk_ids,
                                         const float *topk_w, lgs_dtype map_dt, void *F,
                                         const void *F_target, float scale, float *dL_dfeat,
                                         float *dL_dtopkw, hipStream_t stream);

/*
 * Vanilla feature render, the comparison path of Top-K rendering (Sec. 3.2, Tab. 4):
 * the D-channel feature blended exactly as the colour of Eq. 1 over EVERY blended
 * Gaussian, F[p] = sum_i w_i f_i with the blend's weights w_i = alpha_i T_i (no
 * renormalisation, no Top-K).  One view.  In: the projection and binning outputs and
 * the n_contrib of lgs_rasterize_topk_fwd on the same inputs (the blend is replayed
 * with the forward's arithmetic up to n_contrib, so the weights are the forward's bit
 * for bit); feat[n*d] BF16, or FP8 codes with feat_scale[n].  Out: F[P*d] BF16 (FP32
 * accumulation, one rounding), P = width * height.  d a positive multiple of 8, feat
 * and F 16-byte aligned.  Errors: UNSUPPORTED for FP32 storage or an FP32 map.
 */
lgs_status lgs_feature_render_vanilla_fwd(const lgs_camera *cam, const float *mean2d, const float *conic,
                                          const float *opacity, const int32_t *sorted_ids,
                                          const int32_t *tile_ranges, const int32_t *n_contrib, int32_t d,
                                          lgs_dtype feat_dt, const void *feat, const float *feat_scale,
                                          lgs_dtype map_dt, void *F, hipStream_t stream);

/*
 * Adjoint of the vanilla feature render for a given dL_dF[P*d] (BF16): accumulates
 *   dL_dfeat[id_i] += w_i dL/dF[p]                     (FP32, per Gaussian row),
 * and the feature term of the blend adjoint, with e_i = <dL/dF[p], f_i>,
 *   dL/dalpha_i = T_i e_i - (sum_{j>i} w_j e_j) / (1 - alpha_i),
 * carried to dL_dmean2d[n*2], dL_dconic[n*3], dL_dopacity[n] (+=, the same screen-space
 * gradients lgs_rasterize_topk_bwd accumulates for colour and depth, so calling both
 * gives the whole adjoint).  T_final and n_contrib from lgs_rasterize_topk_fwd.
 */
lgs_status lgs_feature_render_vanilla_bwd(const lgs_camera *cam, const float *mean2d, const float *conic,
                                          const float *opacity, const int32_t *sorted_ids,
                                          const int32_t *tile_ranges, const float *T_final,
                                          const int32_t *n_contrib, int32_t d, lgs_dtype feat_dt,
                                          const void *feat, const float *feat_scale, lgs_dtype map_dt,
                                          const void *dL_dF, float *dL_dfeat, float *dL_dmean2d,
                                          float *dL_dconic, float *dL_dopacity, hipStream_t stream);

/*
 * Adjoint of the blend (Eq. 1) including the Top-K weight path, replayed back to
 * front per pixel from T_final and n_contrib.  dL_dalpha and dL_dtopkw may be NULL.
 * T_final, n_contrib, topk_ids and topk_w are lgs_rasterize_topk_fwd's outputs for the
 * same inputs (the recorded weights tell which Gaussians can be Top-K members).
 * Accumulates per-Gaussian screen-space gradients:
 *   dL_dmean2d[n*2], dL_dconic[n*3] (w.r.t. a, b, c), dL_dopacity[n], dL_drgb[n*3],
 *   dL_ddepth_g[n] (w.r.t. the depth z of each Gaussian).
 * tile_order: as for lgs_rasterize_topk_fwd.
 */
lgs_status lgs_rasterize_topk_bwd(const lgs_camera *cam, int32_t k,
                                  const float *mean2d, const float *conic, const float *opacity,
                                  const float *rgb, const float *depth,
                                  const int32_t *sorted_ids, const int32_t *tile_ranges,
                                  const float *T_final, const int32_t *n_contrib,
                                  const int32_t *topk_ids, const float *topk_w,
                                  const float *dL_dcolor, const float *dL_ddepth,
                                  const float *dL_dalpha, const float *dL_dtopkw,
                                  float *dL_dmean2d, float *dL_dconic, float *dL_dopacity,
                                  float *dL_drgb, float *dL_ddepth_g, const int32_t *tile_order,
                                  hipStream_t stream);

/*
 * Adjoint of the projection: chain rule from the screen-space gradients to the
 * Gaussian parameters, accumulated into dL_dmeans[n*3], dL_dlog_scales[n*3],
 * dL_dquats[n*4] and dL_dopacity_logits[n].  Culled Gaussians receive nothing.
 */
lgs_status lgs_project_bwd(const lgs_camera *cam, int32_t n,
                           const float *means, const float *log_scales, const float *quats,
                           const float *opacity_logits, const float *rgb,
                           const float *dL_dmean2d, const float *dL_dconic,
                           const float *dL_dopacity, const float *dL_ddepth_g,
                           float *dL_dmeans, float *dL_dlog_scales, float *dL_dquats,
                           float *dL_dopacity_logits, hipStream_t stream);

/*
 * Camera-pose gradient of the rendering loss, for the rendering-loss pose refinement
 * of the mapping step (Sec. 4.1), together with (optionally) the parameter gradients
 * of lgs_project_bwd from the same screen-space gradients.  The pose is perturbed on
 * the left, [R|t] <- exp(xi^) [R|t] with xi = (rho, phi): to first order
 * R <- (I + [phi]x) R and t <- (I + [phi]x) t + rho.  Accumulates
 *   dL_dpose[6] += (dL/drho, dL/dphi)  (FP32, device; one block sum per component and
 *                                       block, added with atomics: the summation order
 *                                       varies from run to run),
 * and, when dL_dmeans, dL_dlog_scales, dL_dquats and dL_dopacity_logits are all given,
 * the same parameter gradients as lgs_project_bwd (all four NULL: pose only).
 * Culled Gaussians contribute nothing.  Errors: INVALID_ARG for a NULL dL_dpose or
 * input, or a partial set of parameter-gradient outputs.
 */
lgs_status lgs_project_bwd_pose(const lgs_camera *cam, int32_t n,
                                const float *means, const float *log_scales, const float *quats,
                                const float *opacity_logits, const float *rgb,
                                const float *dL_dmean2d, const float *dL_dconic,
                                const float *dL_dopacity, const float *dL_ddepth_g,
                                float *dL_dmeans, float *dL_dlog_scales, float *dL_dquats,
                                float *dL_dopacity_logits, float *dL_dpose, hipStream_t stream);

/*
 * Batched views (Sec. 3.4: one mapping step renders several keyframes of the same
 * size).  The geometry calls below take `views` cameras (a host array, at most 16, all
 * of one width x height) and run every view in one launch.  Layout:
 *  - a projected RECORD is (view, Gaussian): record v*n + g holds Gaussian g seen from
 *    view v, so mean2d[views*n*2], conic[views*n*3], depth[views*n], opacity[views*n],
 *    tile_rect[views*n*4], tiles_touched[views*n] and the screen-space gradients
 *    dL_dmean2d, dL_dconic, dL_dopacity, dL_ddepth_g are all record-indexed;
 *  - tiles of view v are tiles v*T ... (v+1)*T - 1 (T = tiles of one view), so
 *    tile_ranges has views*T*2 entries and sorted_ids holds record indices ordered by
 *    (view, tile, depth key, Gaussian id): the binning sorts the view into the key;
 *  - per-pixel arrays stack the views: pixel p of view v is entry v*width*height + p;
 *  - per-Gaussian arrays (rgb, dL_drgb, the parameter gradients, Top-K ids) are
 *    indexed by Gaussian and accumulate over the views.
 * Each call with views = 1 equals its single-view counterpart bit for bit (the
 * single-view calls are this case).  Errors: INVALID_ARG for views outside [1, 16],
 * cameras of different sizes, or more than 2^31 - 1 records.
 */
lgs_status lgs_project_fwd_views(const lgs_camera *cams, int32_t views, int32_t n,
                                 const float *means, const float *log_scales, const float *quats,
                                 const float *opacity_logits, const float *rgb,
                                 float *mean2d, float *conic, float *depth, float *opacity,
                                 int32_t *tile_rect, int32_t *tiles_touched, hipStream_t stream);

/* Binning of views*n records (workspace: lgs_bin_sort_workspace(views * n, ...); for
 * lgs_bin_sort_count pass views * n as n).  Same count and capacity rules as
 * lgs_bin_sort. */
lgs_status lgs_bin_sort_views(const lgs_camera *cams, int32_t views, int32_t n, const float *depth,
                              const int32_t *tile_rect, const int32_t *tiles_touched,
                              void *workspace, size_t ws_bytes, int64_t max_pairs,
                              int32_t *sorted_ids, int32_t *tile_ranges, int64_t *n_pairs,
                              hipStream_t stream);

/* Blend + Top-K of every view; n is the Gaussian count (records per view). */
lgs_status lgs_rasterize_topk_fwd_views(const lgs_camera *cams, int32_t views, int32_t k, int32_t n,
                                        const float *mean2d, const float *conic, const float *opacity,
                                        const float *rgb, const float *depth,
                                        const int32_t *sorted_ids, const int32_t *tile_ranges,
                                        float *color, float *depth_map, float *alpha_map,
                                        float *T_final, int32_t *n_contrib,
                                        int32_t *topk_ids, float *topk_w, const int32_t *tile_order,
                                        hipStream_t stream);

/* Blend adjoint of every view: record-indexed screen-space gradients, per-Gaussian
 * dL_drgb summed over the views (all accumulated). */
lgs_status lgs_rasterize_topk_bwd_views(const lgs_camera *cams, int32_t views, int32_t k, int32_t n,
                                        const float *mean2d, const float *conic, const float *opacity,
                                        const float *rgb, const float *depth,
                                        const int32_t *sorted_ids, const int32_t *tile_ranges,
                                        const float *T_final, const int32_t *n_contrib,
                                        const int32_t *topk_ids, const float *topk_w,
                                        const float *dL_dcolor, const float *dL_ddepth,
                                        const float *dL_dalpha, const float *dL_dtopkw,
                                        float *dL_dmean2d, float *dL_dconic, float *dL_dopacity,
                                        float *dL_drgb, float *dL_ddepth_g, const int32_t *tile_order,
                                        hipStream_t stream);

/*
 * Dispatch order of the blend and its adjoint (the per-tile work of Eq. 1-2 and its
 * adjoint; a scheduling aid that changes no result).  A tile's cost grows with its
 * sorted run, and runs differ by an order of magnitude across a frame, so with tiles
 * in raster order a few long ones finish last on an otherwise idle GPU.  This writes,
 * on the device, an order in which each XCD's tiles start longest run first (weights
 * in log-spaced buckets, eight per octave), from the tile_ranges of lgs_bin_sort /
 * lgs_bin_sort_views for the same cameras and views.  The weight is the tile's pair
 * count, or, when n_contrib (lgs_rasterize_topk_fwd's output, P entries) is given, the
 * largest n_contrib over the tile's pixels: the length of list the adjoint walks, the
 * better weight for the adjoint where early termination leaves most of a run unused.
 * order[lgs_tile_order_size(width, height, views)] int32, caller-owned; its first
 * lgs_tile_order_size / 2 entries are the order (entry b is the tile workgroup b
 * renders; values >= the tile count are padding), the rest holds the tile weights.  Pass it as
 * tile_order to lgs_rasterize_topk_fwd(_views) and lgs_rasterize_topk_bwd(_views); a
 * NULL tile_order keeps the fixed mapping.  The blend's outputs are the same bits
 * either way; the adjoint's atomic sums may round in another order, as they may between
 * any two runs.  The order is valid as long as tile_ranges is; a tile_order not
 * written by this call for the same tiles is undefined (entries outside the tile
 * range are skipped, so such an order can drop tiles but not fault).
 * Errors: INVALID_ARG for NULL pointers, a misaligned tile_ranges or bad cameras.
 */
int64_t lgs_tile_order_size(int32_t width, int32_t height, int32_t views);
lgs_status lgs_tile_order(const lgs_camera *cams, int32_t views, const int32_t *tile_ranges,
                          const int32_t *n_contrib, int32_t *order, hipStream_t stream);

/* Projection adjoint of every view: the parameter gradients summed over the views (one
 * thread per Gaussian adds its views in order and writes once: deterministic), and,
 * if dL_dpose is given, each view's camera-pose gradient into dL_dpose[views*6] (as
 * lgs_project_bwd_pose).  The four parameter-gradient outputs are given together or
 * all NULL; at least one output is required. */
lgs_status lgs_project_bwd_views(const lgs_camera *cams, int32_t views, int32_t n,
                                 const float *means, const float *log_scales, const float *quats,
                                 const float *opacity_logits, const float *rgb,
                                 const float *dL_dmean2d, const float *dL_dconic,
                                 const float *dL_dopacity, const float *dL_ddepth_g,
                                 float *dL_dmeans, float *dL_dlog_scales, float *dL_dquats,
                                 float *dL_dopacity_logits, float *dL_dpose, hipStream_t stream);

/* Pruning statistics over every view of a batched forward, accumulated as in
 * lgs_prune_stats. */
lgs_status lgs_prune_stats_views(const lgs_camera *cams, int32_t views, int32_t k, int32_t n,
                                 const float *mean2d, const float *conic, const float *opacity,
                                 const int32_t *sorted_ids, const int32_t *tile_ranges,
                                 const int32_t *n_contrib, const int32_t *topk_ids, int32_t *topk_count,
                                 float *max_w, const int32_t *tile_order, hipStream_t stream);

/*
 * Statistics of the semantic-geometric consistency pruning (Sec. 3.3, Eq. 5) for one
 * view, from that view's forward outputs (same geometry inputs, n_contrib and
 * topk_ids of lgs_rasterize_topk_fwd with the same k):
 *   topk_count[g] += number of pixels whose Top-K list holds Gaussian g (its Top-K
 *                    participation);
 *   max_w[g] = max(max_w[g], w) over every pixel where g is blended, w = alpha T its
 *              blending weight (the geometric importance S_g of Eq. 5).
 * Both accumulate over calls, so calling once per keyframe gives the counts and maxima
 * over all keyframes; the caller zeroes them first (max_w entries must be >= 0).
 * The weights are recomputed with the forward's own arithmetic and equal its weights
 * bit for bit.  topk_count[n] int32, max_w[n] FP32 (4-byte aligned).
 * tile_order: NULL or lgs_tile_order's output for these tile_ranges (with n_contrib, the
 * weight that fits this replay); the counts and maxima are the same either way (integer
 * adds and maxima of non-negative floats do not depend on their order).
 */
lgs_status lgs_prune_stats(const lgs_camera *cam, int32_t k, const float *mean2d, const float *conic,
                           const float *opacity, const int32_t *sorted_ids, const int32_t *tile_ranges,
                           const int32_t *n_contrib, const int32_t *topk_ids, int32_t *topk_count,
                           float *max_w, const int32_t *tile_order, hipStream_t stream);

/*
 * Workspace bytes of lgs_prune_select for n Gaussians.  *bytes is a host pointer.
 */
lgs_status lgs_prune_select_workspace(int32_t n, size_t *bytes);

/*
 * Survival sampling of the consistency pruning (Sec. 3.3, Eq. 6).  The candidate set
 * G_prune is every Gaussian with topk_count[i] < count_below (low Top-K participation);
 * of its c members, m = floor(keep_ratio * c) (the exact product, taken in integer
 * arithmetic) survive, drawn without replacement with probabilities proportional to
 * S_i = max_w[i]: with the caller's exponential variates expo[i] (E_i >= 0, i.i.d.
 * Exp(1) for a fair draw) the survivors are the m candidates with the smallest key
 * E_i / S_i (the correctly rounded FP32 quotient; +inf when S_i = 0), equal keys taken
 * in index order.  The first survivor is then
 * candidate i with probability S_i / sum_j S_j, which is Eq. 6.
 * Out: survive[n] (uint8, overwritten): 1 for every non-candidate and every drawn
 * candidate, 0 for the candidates to remove.  workspace: ws_bytes >=
 * lgs_prune_select_workspace(n), 256-byte aligned.  keep_ratio in [0, 1]; the paper
 * keeps half (0.5).  Asynchronous: the whole draw runs on the device.
 */
lgs_status lgs_prune_select(int32_t n, const int32_t *topk_count, const float *max_w, int32_t count_below,
                            const float *expo, float keep_ratio, void *workspace, size_t ws_bytes,
                            uint8_t *survive, hipStream_t stream);

/*
 * Storage quantization of the feature table (the precision forms of the renderer):
 * dst_dt = BF16: round-to-nearest-even; dst_dt = FP8_E4M3: per row, scale
 * s = 2^floor(log2(amax / 224)) (s = 1 for an all-zero row) so x / s is exact and
 * amax / s lies in [224, 448), then round-to-nearest-even E4M3FN codes of x / s,
 * saturating at +-448.  dst_scale[n] is written for FP8 only.
 */
lgs_status lgs_quantize_features(int32_t n, int32_t d, const float *src, lgs_dtype dst_dt,
                                 void *dst, float *dst_scale, hipStream_t stream);

/*
 * L1 loss gradient (Eq. 9 and the L1 terms of Eq. 8): grad[i] = scale * sign(x[i] -
 * target[i]), sign(0) = 0, over n elements of dtype dt (F32 or BF16, all three
 * arrays the same dtype, 16-byte aligned).  For BF16 the scale is rounded to BF16.
 */
lgs_status lgs_l1_grad(int64_t n, lgs_dtype dt, const void *x, const void *target, float scale,
                       void *grad, hipStream_t stream);

/*
 * Sparse clearing of the dense feature-gradient table dL/df [n][d] between steps (caller
 * work of a training step).  The feature adjoint writes only rows of Gaussians in a
 * pixel's Top-K list (a pixel's feature depends on its K rows alone, Eq. 3-4), so a table
 * that is zero except for the rows named in the last step's Top-K lists can be cleared
 * by zeroing those rows:
 *   step s:  lgs_zero_marked_rows(gen = s - 1), then lgs_mark_topk_rows(step s's
 *            topk_ids, gen = s) (never before the zeroing: a row named in both steps would
 *            keep its old values), then the feature adjoint
 * row_gen[n] (int32, caller memory) holds each row's last generation; start with the
 * table all zero and row_gen below every generation used (e.g. INT32_MIN).
 *
 * lgs_mark_topk_rows: row_gen[g] = gen for every id g in [0, n) among the n_slots entries
 *   of topk_ids (slots holding -1 are skipped).
 * lgs_zero_marked_rows: zeroes row g of table (FP32, d a multiple of 4, 16-byte aligned)
 *   wherever row_gen[g] == gen; other rows are not touched.
 */
lgs_status lgs_mark_topk_rows(int64_t n_slots, const int32_t *topk_ids, int32_t n, int32_t gen, int32_t *row_gen,
                              hipStream_t stream);
lgs_status lgs_zero_marked_rows(int32_t n, int32_t d, int32_t gen, const int32_t *row_gen, float *table,
                                hipStream_t stream);

/*
 * Refresh of the storage form (the quantizers of lgs_quantize_features) for the rows the
 * feature kernels will read.  A pixel's feature reads only the K rows of its Top-K list
 * (Eq. 3-4), so after lgs_mark_topk_rows has stamped the step's Top-K rows with gen, the
 * store is complete for that step's feature render and adjoint once these rows are
 * converted from the FP32 master table; the other rows of dst are not touched and may
 * hold older values.
 *
 * Quantizes row g of src [n][d] (FP32, d a multiple of 8, 16-byte aligned) into dst
 * (dst_dt BF16 [n][d] or FP8 E4M3 codes [n][d] plus dst_scale[n]; 16-byte aligned) for
 * every g with row_gen[g] == gen, with the same arithmetic as lgs_quantize_features (the
 * same bits).
 */
lgs_status lgs_quantize_marked_rows(int32_t n, int32_t d, int32_t gen, const int32_t *row_gen, const float *src,
                                   lgs_dtype dst_dt, void *dst, float *dst_scale, hipStream_t stream);

/*
 * Number of distinct Gaussians over all pixels' Top-K slots (ids in [0, n) in
 * topk_ids[n_pix*k]); the U of the feature adjoint's memory traffic.  flags[n + 1]
 * is caller scratch (overwritten); *count (host) receives the result.
 * Synchronises `stream`.
 */
lgs_status lgs_union_count(int64_t n_pix, int32_t k, int32_t n, const int32_t *topk_ids,
                           int32_t *flags, int64_t *count, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LGS_H */
