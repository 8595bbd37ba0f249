// Projection of 3D Gaussians to screen-space splats (Sec. 3.1, the EWA splat of the
// 3DGS rasterizer the paper follows) and its adjoint.  One thread per Gaussian;
// FP32 throughout, with the depth key as an explicit fused chain.
#include <algorithm>

#include "lgs_device.hpp"
#include "lgs_host.hpp"

namespace lgs {
namespace {

struct CamDev {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int W, H;
    float limx, limy;   // guard band: 1.3x the half field of view (tan)
};

// The cameras of one batched call (views share the image size), passed by value.
constexpr int kMaxViews = 16;
struct CamSet {
    CamDev c[kMaxViews];
};

CamDev make_cam(const lgs_camera *c) {
    CamDev d;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) d.R[3 * i + j] = c->Rt[4 * i + j];
        d.t[i] = c->Rt[4 * i + 3];
    }
    d.fx = c->fx; d.fy = c->fy; d.cx = c->cx; d.cy = c->cy;
    d.W = c->width; d.H = c->height;
    d.limx = 1.3f * (0.5f * (float)c->width / c->fx);
    d.limy = 1.3f * (0.5f * (float)c->height / c->fy);
    return d;
}

// Everything the forward computes for one Gaussian, kept for the adjoint.
struct Splat {
    float t[3];          // view-space mean; t[2] is the depth key
    float s[3];          // scales
    float qn[4], qlen;   // unit quaternion and |q|
    float Rq[9];         // rotation of the unit quaternion
    float Sg[6];         // 3D covariance xx xy xz yy yz zz
    float T[6];          // J R, 2x3 row-major
    float j00, j02, j11, j12;   // the nonzero entries of the Jacobian J
    float A, B, C;       // Sigma2D
    float ca, cb, cc;    // conic
    float mx, my, o;
    bool clampx, clampy;
};

__device__ __forceinline__ bool finite3(const float *p) {
    return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
}

// The view-independent half of splat_of: the validity tests on the parameters, the
// scales, the unit quaternion and its rotation, the 3D covariance and the opacity;
// m receives the mean.  Returns false for a Gaussian culled in every view.
__device__ __forceinline__ bool splat_gauss(int g, const float *__restrict__ means,
                                            const float *__restrict__ log_scales, const float *__restrict__ quats,
                                            const float *__restrict__ opacity_logits,
                                            const float *__restrict__ rgb, Splat &s, float (&mv)[3]) {
    const float *m = means + 3 * g;
    const float *ls = log_scales + 3 * g;
    const float *q = quats + 4 * g;
    float opl = opacity_logits[g];
    if (!finite3(m) || !finite3(ls) || !finite3(rgb + 3 * g) || !isfinite(opl) ||
        !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2]) || !isfinite(q[3]))
        return false;
    if (q[0] == 0.0f && q[1] == 0.0f && q[2] == 0.0f && q[3] == 0.0f) return false;
    if (ls[0] > 10.0f || ls[1] > 10.0f || ls[2] > 10.0f) return false;
    if (opl < -5.53733427f) return false;                 // opacity < 1/255
    mv[0] = m[0]; mv[1] = m[1]; mv[2] = m[2];
    for (int i = 0; i < 3; ++i) s.s[i] = expf(ls[i]);
    // normalise the quaternion; pre-scale by its largest entry so tiny ones survive
    float qm = fmaxf(fmaxf(fabsf(q[0]), fabsf(q[1])), fmaxf(fabsf(q[2]), fabsf(q[3])));
    float qs[4] = {q[0] / qm, q[1] / qm, q[2] / qm, q[3] / qm};
    float ql = sqrtf(qs[0] * qs[0] + qs[1] * qs[1] + qs[2] * qs[2] + qs[3] * qs[3]);
    for (int i = 0; i < 4; ++i) s.qn[i] = qs[i] / ql;
    s.qlen = ql * qm;
    float w = s.qn[0], x = s.qn[1], y = s.qn[2], zq = s.qn[3];
    float *R = s.Rq;
    R[0] = 1.f - 2.f * (y * y + zq * zq); R[1] = 2.f * (x * y - w * zq);       R[2] = 2.f * (x * zq + w * y);
    R[3] = 2.f * (x * y + w * zq);       R[4] = 1.f - 2.f * (x * x + zq * zq); R[5] = 2.f * (y * zq - w * x);
    R[6] = 2.f * (x * zq - w * y);       R[7] = 2.f * (y * zq + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
    // Sigma = M M^T, M = Rq diag(s)
    float M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = R[3 * i + j] * s.s[j];
    int k6 = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
            s.Sg[k6++] = M[3 * i] * M[3 * j] + M[3 * i + 1] * M[3 * j + 1] + M[3 * i + 2] * M[3 * j + 2];
    s.o = 1.0f / (1.0f + expf(-opl));
    return true;
}

// The view-dependent half: view-space mean, the depth test, the perspective Jacobian,
// the 2D covariance, its conic and the screen-space mean.  Returns false when culled.
__device__ __forceinline__ bool splat_view(const CamDev &c, const float (&m)[3], Splat &s) {
    float mx = m[0], my = m[1], mz = m[2];
    float z = fmaf(c.R[8], mz, fmaf(c.R[7], my, fmaf(c.R[6], mx, c.t[2])));
    if (!(z > 0.2f)) return false;
    s.t[0] = fmaf(c.R[0], mx, fmaf(c.R[1], my, fmaf(c.R[2], mz, c.t[0])));
    s.t[1] = fmaf(c.R[3], mx, fmaf(c.R[4], my, fmaf(c.R[5], mz, c.t[1])));
    s.t[2] = z;
    // perspective Jacobian with the guard-band clamp
    float tx = s.t[0], ty = s.t[1];
    float rx = tx / z, ry = ty / z;
    s.clampx = rx < -c.limx || rx > c.limx;
    s.clampy = ry < -c.limy || ry > c.limy;
    float xt = fminf(fmaxf(rx, -c.limx), c.limx) * z;
    float yt = fminf(fmaxf(ry, -c.limy), c.limy) * z;
    float j00 = c.fx / z, j02 = -c.fx * xt / (z * z);
    float j11 = c.fy / z, j12 = -c.fy * yt / (z * z);
    s.j00 = j00; s.j02 = j02; s.j11 = j11; s.j12 = j12;
    for (int j = 0; j < 3; ++j) {
        s.T[j] = j00 * c.R[j] + j02 * c.R[6 + j];
        s.T[3 + j] = j11 * c.R[3 + j] + j12 * c.R[6 + j];
    }
    // Sigma2D = T Sigma T^T + 0.3 I
    const float *S = s.Sg;
    float Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    float TS0[3], TS1[3];
    for (int j = 0; j < 3; ++j) {
        TS0[j] = s.T[0] * Sf[j] + s.T[1] * Sf[3 + j] + s.T[2] * Sf[6 + j];
        TS1[j] = s.T[3] * Sf[j] + s.T[4] * Sf[3 + j] + s.T[5] * Sf[6 + j];
    }
    s.A = TS0[0] * s.T[0] + TS0[1] * s.T[1] + TS0[2] * s.T[2] + 0.3f;
    s.B = TS0[0] * s.T[3] + TS0[1] * s.T[4] + TS0[2] * s.T[5];
    s.C = TS1[0] * s.T[3] + TS1[1] * s.T[4] + TS1[2] * s.T[5] + 0.3f;
    float det = s.A * s.C - s.B * s.B;
    if (!(det > 0.0f) || !isfinite(det)) return false;
    s.ca = s.C / det;
    s.cb = -s.B / det;
    s.cc = s.A / det;
    s.mx = c.fx * tx / z + c.cx;
    s.my = c.fy * ty / z + c.cy;
    return true;
}

// The splat of Gaussian g in camera c; returns false for a culled Gaussian.
__device__ __forceinline__ bool splat_of(const CamDev &c, int g, const float *__restrict__ means,
                                         const float *__restrict__ log_scales, const float *__restrict__ quats,
                                         const float *__restrict__ opacity_logits,
                                         const float *__restrict__ rgb, Splat &s) {
    float m[3];
    return splat_gauss(g, means, log_scales, quats, opacity_logits, rgb, s, m) && splat_view(c, m, s);
}


// One thread per Gaussian: its view-independent state once, then its splat in each view
// (record v * n + g), written in view order.
__global__ __launch_bounds__(256) void project_fwd_kernel(
    CamSet cs, int views, int n, const float *__restrict__ means, const float *__restrict__ log_scales,
    const float *__restrict__ quats, const float *__restrict__ opacity_logits,
    const float *__restrict__ rgb, float2 *__restrict__ mean2d, float *__restrict__ conic,
    float *__restrict__ depth, float *__restrict__ opacity, int4 *__restrict__ tile_rect,
    int *__restrict__ tiles_touched) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    Splat base;
    float m[3];
    const bool live = splat_gauss(g, means, log_scales, quats, opacity_logits, rgb, base, m);
    for (int v = 0; v < views; ++v) {
        const CamDev &c = cs.c[v];
        const long r = (long)v * n + g;   // the record of (view, Gaussian)
        Splat s = base;
        if (!live || !splat_view(c, m, s)) {
            mean2d[r] = make_float2(0.f, 0.f);
            conic[3 * r] = conic[3 * r + 1] = conic[3 * r + 2] = 0.f;
            depth[r] = 0.f;
            opacity[r] = 0.f;
            tile_rect[r] = make_int4(0, 0, 0, 0);
            tiles_touched[r] = 0;
            continue;
        }
        mean2d[r] = make_float2(s.mx, s.my);
        conic[3 * r] = s.ca;
        conic[3 * r + 1] = s.cb;
        conic[3 * r + 2] = s.cc;
        depth[r] = s.t[2];
        opacity[r] = s.o;
        // support {alpha >= 1/255} is the ellipse d^T Sigma2D^-1 d <= 2 ln(255 o); its box
        // has half extents sqrt(2 ln(255 o) A), sqrt(2 ln(255 o) C); pad by a pixel
        float lvl = fmaxf(2.0f * logf(255.0f * s.o), 0.0f);
        float hx = sqrtf(lvl * s.A), hy = sqrtf(lvl * s.C);
        float fx0 = ceilf(s.mx - hx - 0.5f) - 1.0f, fx1 = floorf(s.mx + hx - 0.5f) + 1.0f;
        float fy0 = ceilf(s.my - hy - 0.5f) - 1.0f, fy1 = floorf(s.my + hy - 0.5f) + 1.0f;
        fx0 = fmaxf(fx0, 0.0f);
        fy0 = fmaxf(fy0, 0.0f);
        fx1 = fminf(fx1, (float)(c.W - 1));
        fy1 = fminf(fy1, (float)(c.H - 1));
        if (!(fx1 >= fx0) || !(fy1 >= fy0)) {
            tile_rect[r] = make_int4(0, 0, 0, 0);
            tiles_touched[r] = 0;
            continue;
        }
        int tx0 = (int)fx0 / kTile, tx1 = (int)fx1 / kTile + 1;
        int ty0 = (int)fy0 / kTile, ty1 = (int)fy1 / kTile + 1;
        tile_rect[r] = make_int4(tx0, ty0, tx1, ty1);
        tiles_touched[r] = (tx1 - tx0) * (ty1 - ty0);
    }
}

// Per-Gaussian share of the camera-pose gradient for a left increment exp(xi^) [R|t],
// xi = (rho, phi): the view-space mean moves by rho + phi x t and the rotation by
// [phi]x R.  rho gets dL/dt; phi gets t x dL/dt (the mean) plus, from T = J R, the
// vector (M12 - M21, M20 - M02, M01 - M10) of M = R dT^T J.
__device__ __forceinline__ void pose_share(const CamDev &c, const Splat &s, const float (&dT)[6], float dtx,
                                           float dty, float dtz, float (&out)[6]) {
    out[0] = dtx;
    out[1] = dty;
    out[2] = dtz;
    const float tx = s.t[0], ty = s.t[1], tz = s.t[2];
    out[3] = ty * dtz - tz * dty;
    out[4] = tz * dtx - tx * dtz;
    out[5] = tx * dty - ty * dtx;
    // N = dT^T J (3x3): J rows (j00, 0, j02) and (0, j11, j12)
    float N[9];
    for (int a = 0; a < 3; ++a) {
        N[3 * a + 0] = dT[a] * s.j00;
        N[3 * a + 1] = dT[3 + a] * s.j11;
        N[3 * a + 2] = dT[a] * s.j02 + dT[3 + a] * s.j12;
    }
    float M[9];   // R N
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            M[3 * i + j] = c.R[3 * i] * N[j] + c.R[3 * i + 1] * N[3 + j] + c.R[3 * i + 2] * N[6 + j];
    out[3] += M[5] - M[7];
    out[4] += M[6] - M[2];
    out[5] += M[1] - M[3];
}

// Parameter gradients of one Gaussian.
struct ParamGrad {
    float mu[3], ls[3], q[4], opl;
};

// What the views of one Gaussian contribute to its parameter gradients, summed over
// the views.  Each piece is linear in the view's screen-space gradients given the
// view-independent state (rotation, scales, opacity), so the sum over views is taken
// before the one transform to the parameters: the mean's gradient (R^T dt), the
// symmetrised covariance gradient E = dS + dS^T (xx xy xz yy yz zz) and the opacity's.
struct ViewSum {
    float mu[3], E[6], go;
};

// The adjoint of splat_view for one record (rec: its index in the screen-space gradient
// arrays): its contribution vs to the parameter gradients and, for POSE, its share of
// the camera-pose gradient.
template <bool POSE>
__device__ __forceinline__ void project_bwd_view(const CamDev &c, long rec, const Splat &s,
                                                 const float *__restrict__ d_mean2d, const float *__restrict__ d_conic,
                                                 const float *__restrict__ d_opac, const float *__restrict__ d_depth,
                                                 ViewSum &vs, float (&pose)[6]) {
    float gmx = d_mean2d[2 * rec], gmy = d_mean2d[2 * rec + 1];
    float ga = d_conic[3 * rec], gb = d_conic[3 * rec + 1], gc = d_conic[3 * rec + 2];
    vs.go = d_opac[rec];
    float gz = d_depth[rec];

    // conic -> Sigma2D: dSigma2D = -Q G Q with G = [[ga, gb/2], [gb/2, gc]]
    float a = s.ca, b = s.cb, cq = s.cc;
    float hb = 0.5f * gb;
    float q00 = a * ga + b * hb, q01 = a * hb + b * gc;
    float q10 = b * ga + cq * hb, q11 = b * hb + cq * gc;
    float G00 = -(q00 * a + q01 * b);
    float G01 = -(q00 * b + q01 * cq);
    float G11 = -(q10 * b + q11 * cq);
    // Sigma2D = T Sigma T^T: dSigma = T^T G T, dT = 2 G T Sigma
    const float *T = s.T;
    float GT0[3], GT1[3];   // rows of G T
    for (int j = 0; j < 3; ++j) {
        GT0[j] = G00 * T[j] + G01 * T[3 + j];
        GT1[j] = G01 * T[j] + G11 * T[3 + j];
    }
    float dS[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dS[3 * i + j] = T[i] * GT0[j] + T[3 + i] * GT1[j];
    int k6 = 0;
    for (int i = 0; i < 3; ++i)
        for (int k = i; k < 3; ++k) vs.E[k6++] = dS[3 * i + k] + dS[3 * k + i];
    const float *S = s.Sg;
    float Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    float dT[6];
    for (int j = 0; j < 3; ++j) {
        dT[j] = 2.f * (GT0[0] * Sf[j] + GT0[1] * Sf[3 + j] + GT0[2] * Sf[6 + j]);
        dT[3 + j] = 2.f * (GT1[0] * Sf[j] + GT1[1] * Sf[3 + j] + GT1[2] * Sf[6 + j]);
    }
    // T = J R: dJ = dT R^T; only J00, J02, J11, J12 are non-zero
    float dJ00 = dT[0] * c.R[0] + dT[1] * c.R[1] + dT[2] * c.R[2];
    float dJ02 = dT[0] * c.R[6] + dT[1] * c.R[7] + dT[2] * c.R[8];
    float dJ11 = dT[3] * c.R[3] + dT[4] * c.R[4] + dT[5] * c.R[5];
    float dJ12 = dT[3] * c.R[6] + dT[4] * c.R[7] + dT[5] * c.R[8];
    float tx = s.t[0], ty = s.t[1], z = s.t[2];
    float iz = 1.0f / z, iz2 = iz * iz;
    float dtx = 0.f, dty = 0.f, dtz = 0.f;
    dtz -= (c.fx * dJ00 + c.fy * dJ11) * iz2;
    if (!s.clampx) {
        dtx -= c.fx * iz2 * dJ02;
        dtz += 2.f * c.fx * tx * iz2 * iz * dJ02;
    } else {
        float L = tx < 0.f ? -c.limx : c.limx;
        dtz += c.fx * L * iz2 * dJ02;
    }
    if (!s.clampy) {
        dty -= c.fy * iz2 * dJ12;
        dtz += 2.f * c.fy * ty * iz2 * iz * dJ12;
    } else {
        float L = ty < 0.f ? -c.limy : c.limy;
        dtz += c.fy * L * iz2 * dJ12;
    }
    // mean2D and the rendered depth
    dtx += gmx * c.fx * iz;
    dty += gmy * c.fy * iz;
    dtz -= (gmx * c.fx * tx + gmy * c.fy * ty) * iz2;
    dtz += gz;
    if constexpr (POSE) pose_share(c, s, dT, dtx, dty, dtz, pose);
    // t = R mu + t_cam
    for (int j = 0; j < 3; ++j) vs.mu[j] = c.R[j] * dtx + c.R[3 + j] * dty + c.R[6 + j] * dtz;
}

// Adds view v's contribution to the running sum (the first view's is taken as is).
__device__ __forceinline__ void view_sum_add(ViewSum &acc, const ViewSum &vs, bool first) {
    if (first) {
        acc = vs;
        return;
    }
    for (int j = 0; j < 3; ++j) acc.mu[j] += vs.mu[j];
    for (int j = 0; j < 6; ++j) acc.E[j] += vs.E[j];
    acc.go += vs.go;
}

// The parameter gradients from the views' summed contributions (s: the Gaussian's
// view-independent state from splat_gauss).
__device__ __forceinline__ void param_grads(const Splat &s, const ViewSum &a, ParamGrad &pg) {
    for (int j = 0; j < 3; ++j) pg.mu[j] = a.mu[j];
    // Sigma = M M^T, M = Rq diag(s): dM = E M
    float M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = s.Rq[3 * i + j] * s.s[j];
    const float Ef[9] = {a.E[0], a.E[1], a.E[2], a.E[1], a.E[3], a.E[4], a.E[2], a.E[4], a.E[5]};
    float dR[9];
    for (int j = 0; j < 3; ++j) {
        float ds = 0.f;
        for (int i = 0; i < 3; ++i) {
            float dM = 0.f;
            for (int k = 0; k < 3; ++k) dM += Ef[3 * i + k] * M[3 * k + j];
            ds += dM * s.Rq[3 * i + j];
            dR[3 * i + j] = dM * s.s[j];
        }
        pg.ls[j] = ds * s.s[j];
    }
    // rotation matrix of the unit quaternion (w, x, y, z)
    float w = s.qn[0], x = s.qn[1], y = s.qn[2], zq = s.qn[3];
    float dw = 2.f * (zq * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
    float dx = 2.f * (y * (dR[1] + dR[3]) + zq * (dR[2] + dR[6]) + w * (dR[7] - dR[5]) -
                      2.f * x * (dR[4] + dR[8]));
    float dy = 2.f * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + zq * (dR[5] + dR[7]) -
                      2.f * y * (dR[0] + dR[8]));
    float dz = 2.f * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7]) -
                      2.f * zq * (dR[0] + dR[4]));
    float dot = dw * w + dx * x + dy * y + dz * zq;
    float il = 1.0f / s.qlen;
    pg.q[0] = (dw - w * dot) * il;
    pg.q[1] = (dx - x * dot) * il;
    pg.q[2] = (dy - y * dot) * il;
    pg.q[3] = (dz - zq * dot) * il;
    pg.opl = a.go * s.o * (1.0f - s.o);
}

__device__ __forceinline__ void add_param_grads(int g, const ParamGrad &pg, float *__restrict__ d_means,
                                                float *__restrict__ d_ls, float *__restrict__ d_quats,
                                                float *__restrict__ d_opl) {
    for (int j = 0; j < 3; ++j) d_means[3 * g + j] += pg.mu[j];
    for (int j = 0; j < 3; ++j) d_ls[3 * g + j] += pg.ls[j];
    for (int j = 0; j < 4; ++j) d_quats[4 * g + j] += pg.q[j];
    d_opl[g] += pg.opl;
}


// Parameter gradients summed over the views, one thread per Gaussian: the Gaussian's
// view-independent state once, each view's contribution added in view order, one
// transform to the parameters, and the result added to memory once (deterministic).
__global__ __launch_bounds__(256) void project_bwd_kernel(
    CamSet cs, int views, int n, const float *__restrict__ means, const float *__restrict__ log_scales,
    const float *__restrict__ quats, const float *__restrict__ opacity_logits,
    const float *__restrict__ rgb, const float *__restrict__ d_mean2d,
    const float *__restrict__ d_conic, const float *__restrict__ d_opac,
    const float *__restrict__ d_depth, float *__restrict__ d_means, float *__restrict__ d_ls,
    float *__restrict__ d_quats, float *__restrict__ d_opl) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    Splat base;
    float m[3];
    if (!splat_gauss(g, means, log_scales, quats, opacity_logits, rgb, base, m)) return;
    ViewSum acc = {};
    bool any = false;
    float unused[6];
    for (int v = 0; v < views; ++v) {
        Splat s = base;
        if (!splat_view(cs.c[v], m, s)) continue;
        ViewSum vs;
        project_bwd_view<false>(cs.c[v], (long)v * n + g, s, d_mean2d, d_conic, d_opac, d_depth, vs, unused);
        view_sum_add(acc, vs, !any);
        any = true;
    }
    if (!any) return;
    ParamGrad pg;
    param_grads(base, acc, pg);
    add_param_grads(g, pg, d_means, d_ls, d_quats, d_opl);
}

constexpr int kPoseGrid = 2048;   // blocks of the pose reduction: at most this many atomics per component

// The projection adjoint with the camera-pose gradient of every view (Sec. 4.1), in one
// pass: the grid strides over the Gaussians; per Gaussian the views are walked in order,
// its parameter gradients (PARAMS) formed and written once as in project_bwd_kernel
// (the same bits), and its share of each view's pose gradient added to the thread's
// registers (MAXV >= views).  Each block then sums every view's six components (wave
// sums, the four wave partials in a fixed order) and adds them with one atomic each.
template <bool PARAMS, int MAXV>
__global__ __launch_bounds__(256) void project_bwd_pose_kernel(
    CamSet cs, int views, int n, const float *__restrict__ means, const float *__restrict__ log_scales,
    const float *__restrict__ quats, const float *__restrict__ opacity_logits,
    const float *__restrict__ rgb, const float *__restrict__ d_mean2d,
    const float *__restrict__ d_conic, const float *__restrict__ d_opac,
    const float *__restrict__ d_depth, float *__restrict__ d_means, float *__restrict__ d_ls,
    float *__restrict__ d_quats, float *__restrict__ d_opl, float *__restrict__ d_pose) {
    float pose[MAXV][6];
#pragma unroll
    for (int v = 0; v < MAXV; ++v)
#pragma unroll
        for (int q = 0; q < 6; ++q) pose[v][q] = 0.f;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        Splat base;
        float m[3];
        if (!splat_gauss(g, means, log_scales, quats, opacity_logits, rgb, base, m)) continue;
        ViewSum acc = {};
        bool any = false;
#pragma unroll
        for (int v = 0; v < MAXV; ++v) {
            if (v >= views) break;
            Splat s = base;
            if (!splat_view(cs.c[v], m, s)) continue;
            ViewSum vs;
            float sh[6];
            project_bwd_view<true>(cs.c[v], (long)v * n + g, s, d_mean2d, d_conic, d_opac, d_depth, vs, sh);
#pragma unroll
            for (int q = 0; q < 6; ++q) pose[v][q] += sh[q];
            if constexpr (PARAMS) view_sum_add(acc, vs, !any);
            any = true;
        }
        if constexpr (PARAMS) {
            if (any) {
                ParamGrad pg;
                param_grads(base, acc, pg);
                add_param_grads(g, pg, d_means, d_ls, d_quats, d_opl);
            }
        }
    }
    // every lane of the block takes part in the sums
    __shared__ float part[4][MAXV][6];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
        if (v >= views) break;
        float sum[6];
        wave_sum_many<6>(pose[v], sum);
        if ((threadIdx.x & 63) == 0)
            for (int q = 0; q < 6; ++q) part[wave][v][q] = sum[q];
    }
    __syncthreads();
    if ((int)threadIdx.x < 6 * views) {
        const int v = threadIdx.x / 6, q = threadIdx.x - 6 * v;
        const float val = (part[0][v][q] + part[1][v][q]) + (part[2][v][q] + part[3][v][q]);
        if (val != 0.f) unsafeAtomicAdd(&d_pose[6 * v + q], val);
    }
}

template <bool PARAMS>
void launch_bwd_pose(const CamSet &cs, int views, int n, const float *means, const float *log_scales,
                     const float *quats, const float *opacity_logits, const float *rgb, const float *d_mean2d,
                     const float *d_conic, const float *d_opac, const float *d_depth, float *d_means, float *d_ls,
                     float *d_quats, float *d_opl, float *d_pose, hipStream_t st) {
    const unsigned grid = (unsigned)std::min<long>(((long)n + 255) / 256, kPoseGrid);
#define POSE_CALL(MV)                                                                                            \
    hipLaunchKernelGGL((project_bwd_pose_kernel<PARAMS, MV>), dim3(grid), dim3(256), 0, st, cs, views, n, means, \
                       log_scales, quats, opacity_logits, rgb, d_mean2d, d_conic, d_opac, d_depth, d_means, d_ls,  \
                       d_quats, d_opl, d_pose)
    if (views <= 2)
        POSE_CALL(2);
    else if (views <= 4)
        POSE_CALL(4);
    else if (views <= 8)
        POSE_CALL(8);
    else
        POSE_CALL(16);
#undef POSE_CALL
}

// Host-side set of cameras; all views must share the image size.
lgs_status make_camset(const lgs_camera *cams, int views, CamSet &cs) {
    LGS_REQUIRE(cams, LGS_ERR_INVALID_ARG, "camera array is NULL");
    LGS_REQUIRE(views >= 1 && views <= kMaxViews, LGS_ERR_INVALID_ARG, "views = %d outside [1, %d]", views,
                kMaxViews);
    for (int v = 0; v < views; ++v) {
        lgs_status st = check_camera(&cams[v]);
        if (st) return st;
        LGS_REQUIRE(cams[v].width == cams[0].width && cams[v].height == cams[0].height, LGS_ERR_INVALID_ARG,
                    "view %d has size %dx%d, view 0 %dx%d: batched views share the image size", v, cams[v].width,
                    cams[v].height, cams[0].width, cams[0].height);
        cs.c[v] = make_cam(&cams[v]);
    }
    return LGS_OK;
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_project_fwd_views(const lgs_camera *cams, int32_t views, int32_t n, const float *means,
                                            const float *log_scales, const float *quats,
                                            const float *opacity_logits, const float *rgb, float *mean2d,
                                            float *conic, float *depth, float *opacity, int32_t *tile_rect,
                                            int32_t *tiles_touched, hipStream_t stream) {
    CamSet cs;
    lgs_status st = make_camset(cams, views, cs);
    if (st) return st;
    LGS_REQUIRE(n >= 0, LGS_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(means && log_scales && quats && opacity_logits && rgb && mean2d && conic && depth &&
                    opacity && tile_rect && tiles_touched,
                LGS_ERR_INVALID_ARG, "lgs_project_fwd: NULL pointer");
    LGS_REQUIRE(((uintptr_t)mean2d & 7u) == 0 && aligned16(tile_rect), LGS_ERR_INVALID_ARG,
                "lgs_project_fwd: mean2d must be 8-byte and tile_rect 16-byte aligned");
    hipLaunchKernelGGL(project_fwd_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, cs, views, n, means,
                       log_scales, quats, opacity_logits, rgb, (float2 *)mean2d, conic, depth, opacity,
                       (int4 *)tile_rect, tiles_touched);
    return check_launch("project_fwd");
}

extern "C" lgs_status lgs_project_fwd(const lgs_camera *cam, int32_t n, const float *means,
                                      const float *log_scales, const float *quats,
                                      const float *opacity_logits, const float *rgb,
                                      float *mean2d, float *conic, float *depth, float *opacity,
                                      int32_t *tile_rect, int32_t *tiles_touched,
                                      hipStream_t stream) {
    return lgs_project_fwd_views(cam, 1, n, means, log_scales, quats, opacity_logits, rgb, mean2d, conic, depth,
                                 opacity, tile_rect, tiles_touched, stream);
}

extern "C" lgs_status lgs_project_bwd_views(const lgs_camera *cams, int32_t views, int32_t n, const float *means,
                                            const float *log_scales, const float *quats,
                                            const float *opacity_logits, const float *rgb,
                                            const float *dL_dmean2d, const float *dL_dconic,
                                            const float *dL_dopacity, const float *dL_ddepth_g, float *dL_dmeans,
                                            float *dL_dlog_scales, float *dL_dquats, float *dL_dopacity_logits,
                                            float *dL_dpose, hipStream_t stream) {
    CamSet cs;
    lgs_status st = make_camset(cams, views, cs);
    if (st) return st;
    LGS_REQUIRE(n >= 0, LGS_ERR_INVALID_ARG, "n must be >= 0");
    const int nparams = (dL_dmeans != nullptr) + (dL_dlog_scales != nullptr) + (dL_dquats != nullptr) +
                        (dL_dopacity_logits != nullptr);
    LGS_REQUIRE(nparams == 0 || nparams == 4, LGS_ERR_INVALID_ARG,
                "lgs_project_bwd: the four parameter gradients are given together or not at all");
    LGS_REQUIRE(nparams == 4 || dL_dpose, LGS_ERR_INVALID_ARG, "lgs_project_bwd: no output");
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(means && log_scales && quats && opacity_logits && rgb && dL_dmean2d && dL_dconic && dL_dopacity &&
                    dL_ddepth_g,
                LGS_ERR_INVALID_ARG, "lgs_project_bwd: NULL input");
    if (!dL_dpose)
        hipLaunchKernelGGL(project_bwd_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, cs, views, n, means,
                           log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic, dL_dopacity, dL_ddepth_g,
                           dL_dmeans, dL_dlog_scales, dL_dquats, dL_dopacity_logits);
    else if (nparams)
        launch_bwd_pose<true>(cs, views, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                              dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats, dL_dopacity_logits,
                              dL_dpose, stream);
    else
        launch_bwd_pose<false>(cs, views, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                               dL_dopacity, dL_ddepth_g, nullptr, nullptr, nullptr, nullptr, dL_dpose, stream);
    return check_launch("project_bwd");
}

extern "C" lgs_status lgs_project_bwd(const lgs_camera *cam, int32_t n, const float *means,
                                      const float *log_scales, const float *quats,
                                      const float *opacity_logits, const float *rgb,
                                      const float *dL_dmean2d, const float *dL_dconic,
                                      const float *dL_dopacity, const float *dL_ddepth_g,
                                      float *dL_dmeans, float *dL_dlog_scales, float *dL_dquats,
                                      float *dL_dopacity_logits, hipStream_t stream) {
    LGS_REQUIRE(n <= 0 || (dL_dmeans && dL_dlog_scales && dL_dquats && dL_dopacity_logits), LGS_ERR_INVALID_ARG,
                "lgs_project_bwd: NULL pointer");
    return lgs_project_bwd_views(cam, 1, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                                 dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats,
                                 dL_dopacity_logits, nullptr, stream);
}

extern "C" lgs_status lgs_project_bwd_pose(const lgs_camera *cam, int32_t n, const float *means,
                                           const float *log_scales, const float *quats,
                                           const float *opacity_logits, const float *rgb,
                                           const float *dL_dmean2d, const float *dL_dconic,
                                           const float *dL_dopacity, const float *dL_ddepth_g,
                                           float *dL_dmeans, float *dL_dlog_scales, float *dL_dquats,
                                           float *dL_dopacity_logits, float *dL_dpose, hipStream_t stream) {
    LGS_REQUIRE(dL_dpose, LGS_ERR_INVALID_ARG, "lgs_project_bwd_pose: dL_dpose is NULL");
    return lgs_project_bwd_views(cam, 1, n, means, log_scales, quats, opacity_logits, rgb, dL_dmean2d, dL_dconic,
                                 dL_dopacity, dL_ddepth_g, dL_dmeans, dL_dlog_scales, dL_dquats,
                                 dL_dopacity_logits, dL_dpose, stream);
}
