/*
 * FP64 CPU oracle for Top-K Gaussian-splatting rendering (LangGS-SLAM, arXiv 2602.06991).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the HIP
 * path is checked against.  Only the test suite, the smoke check and the bench's
 * CPU-baseline leg may load it.  It shares no code, header or constant table with
 * the GPU library: every formula below is written out here from the paper and
 * from the 3DGS rasterizer the paper says it follows (Sec. 3.1).
 *
 * What it computes, per view (readings of the paper where it is silent are marked R#
 * and listed in the design notes of the repository):
 *   Projection (Sec. 3.1, the 3DGS EWA splat): o = sigmoid(theta_o); s = exp(theta_s);
 *     Sigma = Rq S^2 Rq^T; t = R mu + t_cam; J the perspective Jacobian with the 1.3x
 *     guard band (R1); Sigma2D = J R Sigma R^T J^T + 0.3 I (R1); conic = Sigma2D^-1;
 *     mu2D = (fx tx/tz + cx, fy ty/tz + cy); pixel centres at (x+1/2, y+1/2) (R4).
 *   Culls, decided on the FP32 inputs so every implementation takes them alike:
 *     any non-finite parameter, an all-zero quaternion, a log-scale above 10,
 *     theta_o below -ln(254) (opacity under 1/255), depth key <= 0.2 (R1, R3, R5).
 *   Depth key (R5): the FP32 value fmaf(R22, mz, fmaf(R21, my, fmaf(R20, mx, t2))).
 *   Blend (Eq. 1): candidates in (depth key, id) order; sigma = d^T Q d / 2,
 *     alpha = min(0.99, o e^-sigma); skip alpha < 1/255; stop before a Gaussian that
 *     would take T(1-alpha) below 1e-4 (R2); w = alpha T; C += c w; D += z w.
 *   Top-K (Eq. 2): the K largest w among the blended Gaussians, ordered by
 *     (w desc, depth key asc, id asc) (R6); padding (id -1, w 0) (R7).
 *   Feature (Eq. 3-4): F = sum_k (w_k / W) f_k with W = sum_k w_k; F = 0 if W = 0.
 *   Backward: the exact derivative of all of the above with every discrete decision
 *     (order, skip, stop, clamp, Top-K set, culls) held fixed.
 *
 * Decision margins: for every pixel the oracle reports how close each of its
 * exp- or product-dependent decisions came to flipping, so a test can tell the
 * pixels where an FP32 implementation may legitimately decide otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

typedef struct {
    double R[3][3], t[3];
    float Rf[3][3], tf[3];
    double fx, fy, cx, cy;
    int W, H;
} cam_t;

static void cam_from(const float *cam, int W, int H, cam_t *c)
{
    /* cam = { Rt[12] row-major 3x4, fx, fy, cx, cy } */
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) {
            c->Rf[i][j] = cam[4 * i + j];
            c->R[i][j] = (double)cam[4 * i + j];
        }
        c->tf[i] = cam[4 * i + 3];
        c->t[i] = (double)cam[4 * i + 3];
    }
    c->fx = cam[12];
    c->fy = cam[13];
    c->cx = cam[14];
    c->cy = cam[15];
    c->W = W;
    c->H = H;
}

/* ------------------------------------------------------------------ projection */

typedef struct {
    int valid;
    double t[3];          /* view-space mean */
    float zkey;           /* FP32 depth key */
    double m2[2];         /* mean2D */
    double cov[3];        /* Sigma2D: A, B, C */
    double con[3];        /* conic a, b, c (sigma = a dx^2/2 + b dx dy + c dy^2/2) */
    double o;             /* opacity */
    int rect[4];          /* inclusive pixel box x0, y0, x1, y1 (x1 < x0: empty) */
    /* saved for the chain rule */
    double s[3], qn[4], qnorm, Rq[3][3], Sig[3][3], J[2][3], Tm[2][3];
    int clampx, clampy;
    double limx, limy;
} proj_t;

static int all_finite(const float *p, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

static void quat_to_rot(const double q[4], double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

static void project_one(const cam_t *c, const float *mu, const float *ls, const float *q,
                        float opl, const float *rgb, proj_t *p)
{
    memset(p, 0, sizeof(*p));
    p->rect[0] = 0; p->rect[2] = -1;
    p->rect[1] = 0; p->rect[3] = -1;
    if (!all_finite(mu, 3) || !all_finite(ls, 3) || !all_finite(q, 4) || !isfinite(opl) ||
        !all_finite(rgb, 3))
        return;
    if (q[0] == 0.0f && q[1] == 0.0f && q[2] == 0.0f && q[3] == 0.0f) return;
    if (ls[0] > 10.0f || ls[1] > 10.0f || ls[2] > 10.0f) return;
    if (opl < -5.53733427f) return;
    /* depth key: the FP32 fused chain, correctly rounded at every step */
    float zk = fmaf(c->Rf[2][2], mu[2], fmaf(c->Rf[2][1], mu[1], fmaf(c->Rf[2][0], mu[0], c->tf[2])));
    if (!(zk > 0.2f)) return;
    p->zkey = zk;

    for (int i = 0; i < 3; ++i)
        p->t[i] = c->R[i][0] * mu[0] + c->R[i][1] * mu[1] + c->R[i][2] * mu[2] + c->t[i];
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];

    for (int i = 0; i < 3; ++i) p->s[i] = exp((double)ls[i]);
    double qq = 0;
    for (int i = 0; i < 4; ++i) qq += (double)q[i] * (double)q[i];
    p->qnorm = sqrt(qq);
    for (int i = 0; i < 4; ++i) p->qn[i] = q[i] / p->qnorm;
    quat_to_rot(p->qn, p->Rq);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k) a += p->Rq[i][k] * p->s[k] * p->s[k] * p->Rq[j][k];
            p->Sig[i][j] = a;
        }

    p->limx = 1.3 * (c->W / (2.0 * c->fx));
    p->limy = 1.3 * (c->H / (2.0 * c->fy));
    double rx = tx / tz, ry = ty / tz;
    p->clampx = (rx < -p->limx || rx > p->limx);
    p->clampy = (ry < -p->limy || ry > p->limy);
    double xt = (rx < -p->limx ? -p->limx : (rx > p->limx ? p->limx : rx)) * tz;
    double yt = (ry < -p->limy ? -p->limy : (ry > p->limy ? p->limy : ry)) * tz;
    p->J[0][0] = c->fx / tz; p->J[0][1] = 0;           p->J[0][2] = -c->fx * xt / (tz * tz);
    p->J[1][0] = 0;          p->J[1][1] = c->fy / tz;  p->J[1][2] = -c->fy * yt / (tz * tz);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k) a += p->J[i][k] * c->R[k][j];
            p->Tm[i][j] = a;
        }
    double S2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) a += p->Tm[i][k] * p->Sig[k][l] * p->Tm[j][l];
            S2[i][j] = a;
        }
    double A = S2[0][0] + 0.3, B = S2[0][1], C = S2[1][1] + 0.3;
    double det = A * C - B * B;
    if (!(det > 0) || !isfinite(det)) return;
    p->cov[0] = A; p->cov[1] = B; p->cov[2] = C;
    p->con[0] = C / det; p->con[1] = -B / det; p->con[2] = A / det;
    p->m2[0] = c->fx * tx / tz + c->cx;
    p->m2[1] = c->fy * ty / tz + c->cy;
    p->o = 1.0 / (1.0 + exp(-(double)opl));
    p->valid = 1;

    /* support: o exp(-sigma) >= 1/255  <=>  d^T Q d <= 2 ln(255 o): an ellipse whose
       axis-aligned half extents are sqrt(2 ln(255 o) A) and sqrt(2 ln(255 o) C) */
    double lvl = 2.0 * log(255.0 * p->o);
    if (lvl < 0) lvl = 0;
    double hx = sqrt(lvl * A), hy = sqrt(lvl * C);
    double x0 = ceil(p->m2[0] - hx - 0.5) - 1, x1 = floor(p->m2[0] + hx - 0.5) + 1;
    double y0 = ceil(p->m2[1] - hy - 0.5) - 1, y1 = floor(p->m2[1] + hy - 0.5) + 1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > c->W - 1) x1 = c->W - 1;
    if (y1 > c->H - 1) y1 = c->H - 1;
    if (x1 < x0 || y1 < y0) { p->rect[0] = 0; p->rect[2] = -1; p->rect[1] = 0; p->rect[3] = -1; return; }
    p->rect[0] = (int)x0; p->rect[1] = (int)y0; p->rect[2] = (int)x1; p->rect[3] = (int)y1;
}

static proj_t *project_all(const cam_t *c, int n, const float *means, const float *ls,
                           const float *q, const float *opl, const float *rgb)
{
    proj_t *P = (proj_t *)malloc(sizeof(proj_t) * (size_t)(n > 0 ? n : 1));
    if (!P) return NULL;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < n; ++g)
        project_one(c, means + 3 * g, ls + 3 * g, q + 4 * g, opl[g], rgb + 3 * g, &P[g]);
    return P;
}

int orc_project(int n, const float *means, const float *ls, const float *q, const float *opl,
                const float *rgb, const float *cam, int W, int H,
                int *valid, double *mean2d, double *cov2d, double *conic, double *tview,
                float *zkey, double *opacity, int *rect)
{
    cam_t c;
    cam_from(cam, W, H, &c);
    proj_t *P = project_all(&c, n, means, ls, q, opl, rgb);
    if (!P) return -1;
    for (int g = 0; g < n; ++g) {
        valid[g] = P[g].valid;
        mean2d[2 * g] = P[g].m2[0]; mean2d[2 * g + 1] = P[g].m2[1];
        for (int i = 0; i < 3; ++i) {
            cov2d[3 * g + i] = P[g].cov[i];
            conic[3 * g + i] = P[g].con[i];
            tview[3 * g + i] = P[g].t[i];
        }
        zkey[g] = P[g].zkey;
        opacity[g] = P[g].o;
        for (int i = 0; i < 4; ++i) rect[4 * g + i] = P[g].rect[i];
    }
    free(P);
    return 0;
}

/* ------------------------------------------------------------- candidate lists */

typedef struct { float z; int id; } cand_t;

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->z < y->z) return -1;
    if (x->z > y->z) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    int ntx, nty;
    int *start;     /* ntx*nty + 1 */
    cand_t *list;   /* per tile, (zkey, id) ascending */
} bins_t;

/* Candidate lists: in "brute" mode every valid Gaussian is a candidate of every pixel;
   otherwise Gaussians are filed by 16x16 tile from their support box.  Either way a
   pixel keeps only Gaussians with alpha >= 1/255, so both give the same result. */
static int make_bins(const proj_t *P, int n, int W, int H, int brute, bins_t *b)
{
    b->ntx = brute ? 1 : (W + ORC_TILE - 1) / ORC_TILE;
    b->nty = brute ? 1 : (H + ORC_TILE - 1) / ORC_TILE;
    int T = b->ntx * b->nty;
    b->start = (int *)calloc((size_t)T + 1, sizeof(int));
    if (!b->start) return -1;
    /* pass 0 counts, pass 1 fills */
    int *fill = (int *)calloc((size_t)T, sizeof(int));
    if (!fill) return -1;
    b->list = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        for (int g = 0; g < n; ++g) {
            if (!P[g].valid) continue;
            int tx0 = 0, tx1 = 0, ty0 = 0, ty1 = 0;
            if (!brute) {
                if (P[g].rect[2] < P[g].rect[0] || P[g].rect[3] < P[g].rect[1]) continue;
                tx0 = P[g].rect[0] / ORC_TILE; tx1 = P[g].rect[2] / ORC_TILE;
                ty0 = P[g].rect[1] / ORC_TILE; ty1 = P[g].rect[3] / ORC_TILE;
            }
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    int t = ty * b->ntx + tx;
                    if (pass == 0) { b->start[t + 1]++; continue; }
                    b->list[fill[t]].z = P[g].zkey;
                    b->list[fill[t]++].id = g;
                }
        }
        if (pass == 0) {
            for (int t = 0; t < T; ++t) b->start[t + 1] += b->start[t];
            memcpy(fill, b->start, sizeof(int) * (size_t)T);
            b->list = (cand_t *)malloc(sizeof(cand_t) * (size_t)(b->start[T] > 0 ? b->start[T] : 1));
            if (!b->list) { free(fill); return -1; }
        }
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < T; ++t)
        qsort(b->list + b->start[t], (size_t)(b->start[t + 1] - b->start[t]), sizeof(cand_t), cand_cmp);
    return 0;
}

static void free_bins(bins_t *b) { free(b->start); free(b->list); }

/* --------------------------------------------------------------- per-pixel blend */

typedef struct {
    int id;
    double alpha, T, w, sigma, ex, dx, dy;
    int clamped;
} blend_t;

typedef struct {
    double C[3], D, T;
    int n;              /* blended count */
    double m_skip, m_clamp, m_T, m_topk;
    uint64_t sig;
} pix_t;

static uint64_t mix64(uint64_t h, uint64_t v)
{
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h * 0xBF58476D1CE4E5B9ull;
}

/* Blends the candidates of pixel (x, y); fills bl[0..n) with the blended Gaussians. */
static void blend_pixel(const proj_t *P, const float *rgb, const cand_t *cands, int nc, int x, int y,
                        int use_rect, blend_t *bl, pix_t *out)
{
    double px = x + 0.5, py = y + 0.5;
    double T = 1.0;
    out->C[0] = out->C[1] = out->C[2] = 0;
    out->D = 0;
    out->n = 0;
    out->m_skip = out->m_clamp = out->m_T = INFINITY;
    out->sig = 0x1234567ull;
    for (int j = 0; j < nc; ++j) {
        int g = cands[j].id;
        const proj_t *p = &P[g];
        if (use_rect && (x < p->rect[0] || x > p->rect[2] || y < p->rect[1] || y > p->rect[3])) continue;
        double dx = px - p->m2[0], dy = py - p->m2[1];
        double sigma = 0.5 * (p->con[0] * dx * dx + p->con[2] * dy * dy) + p->con[1] * dx * dy;
        if (sigma < 0) sigma = 0;
        double ex = exp(-sigma);
        double raw = p->o * ex;
        int clamped = raw > 0.99;
        double alpha = clamped ? 0.99 : raw;
        double ms = fabs(alpha * 255.0 - 1.0);
        if (ms < out->m_skip) out->m_skip = ms;
        double mc = fabs(raw / 0.99 - 1.0);
        if (mc < out->m_clamp) out->m_clamp = mc;
        if (alpha < 1.0 / 255.0) continue;
        double Tn = T * (1.0 - alpha);
        double mt = fabs(Tn / 1e-4 - 1.0);
        if (mt < out->m_T) out->m_T = mt;
        if (Tn < 1e-4) break;
        double w = alpha * T;
        const float *c = rgb + 3 * g;
        for (int k = 0; k < 3; ++k) out->C[k] += c[k] * w;
        out->D += p->t[2] * w;
        blend_t *b = &bl[out->n++];
        b->id = g; b->alpha = alpha; b->T = T; b->w = w; b->sigma = sigma; b->ex = ex;
        b->dx = dx; b->dy = dy; b->clamped = clamped;
        out->sig = mix64(out->sig, (uint64_t)(uint32_t)g * 2u + (uint64_t)clamped);
        T = Tn;
    }
    out->T = T;
}

/* Top-K selection (Eq. 2) over weights listed in blend order, i.e. in (depth key, id)
   order: rank r takes the largest remaining weight, the earliest listed on a tie, so
   the order is (w desc, depth key asc, id asc).  Writes the list positions of the first
   min(R, n) ranks to rank[]. */
int orc_topk_select(int n, const double *w, int R, int *rank)
{
    char *used = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!used) return -1;
    int m = R < n ? R : n;
    for (int r = 0; r < m; ++r) {
        int best = -1;
        for (int i = 0; i < n; ++i) {
            if (used[i]) continue;
            if (best < 0 || w[i] > w[best]) best = i;
        }
        used[best] = 1;
        rank[r] = best;
    }
    free(used);
    return m;
}

static void topk_of(const blend_t *bl, int n, int K, int *ids, double *ws, int *pos, double *m_topk)
{
    int rank[64];
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) w[i] = bl[i].w;
    int R = orc_topk_select(n, w, K + 1, rank);
    free(w);
    for (int k = 0; k < K; ++k) {
        if (k < n) { ids[k] = bl[rank[k]].id; ws[k] = bl[rank[k]].w; if (pos) pos[k] = rank[k]; }
        else { ids[k] = -1; ws[k] = 0.0; if (pos) pos[k] = -1; }
    }
    double m = INFINITY;
    for (int r = 0; r + 1 < R; ++r) {
        double a = bl[rank[r]].w, b = bl[rank[r + 1]].w;
        double gap = (a - b) / a;
        if (gap < m) m = gap;
    }
    *m_topk = m;
}

static int max_list_len(const bins_t *b)
{
    int T = b->ntx * b->nty, m = 0;
    for (int t = 0; t < T; ++t)
        if (b->start[t + 1] - b->start[t] > m) m = b->start[t + 1] - b->start[t];
    return m;
}

/*
 * Forward render of one view.  Outputs per pixel p = y*W + x:
 *   C[3p..], D[p], O[p] = 1 - T_final, Tfin[p], nblend[p], topk ids/w [p*K + k],
 *   margins[4p..]: alpha-skip, alpha-clamp, T-floor (relative distance of the compared
 *   quantity from its threshold) and the smallest relative gap between adjacent
 *   ranked weights among the first K+1; sig[p] a hash of the blended sequence.
 * K must be 1..63.  brute != 0 evaluates every valid Gaussian at every pixel.
 */
int orc_render(int n, const float *means, const float *ls, const float *q, const float *opl,
               const float *rgb, const float *cam, int W, int H, int K, int brute,
               double *C, double *D, double *O, double *Tfin, int *nblend, int *topk_ids,
               double *topk_w, double *margins, uint64_t *sig)
{
    if (K < 1 || K > 63) return -2;
    cam_t c;
    cam_from(cam, W, H, &c);
    proj_t *P = project_all(&c, n, means, ls, q, opl, rgb);
    if (!P) return -1;
    bins_t b;
    if (make_bins(P, n, W, H, brute, &b)) { free(P); return -1; }
    int cap = max_list_len(&b) + 1;
    int err = 0;
#pragma omp parallel
    {
        blend_t *bl = (blend_t *)malloc(sizeof(blend_t) * (size_t)cap);
        if (!bl) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 64)
        for (long pix = 0; pix < (long)W * H; ++pix) {
            if (!bl) continue;
            int x = (int)(pix % W), y = (int)(pix / W);
            int t = brute ? 0 : (y / ORC_TILE) * b.ntx + x / ORC_TILE;
            pix_t o;
            blend_pixel(P, rgb, b.list + b.start[t], b.start[t + 1] - b.start[t], x, y, !brute, bl, &o);
            for (int k = 0; k < 3; ++k) C[3 * pix + k] = o.C[k];
            D[pix] = o.D;
            O[pix] = 1.0 - o.T;
            Tfin[pix] = o.T;
            nblend[pix] = o.n;
            double mk;
            topk_of(bl, o.n, K, topk_ids + (long)K * pix, topk_w + (long)K * pix, NULL, &mk);
            margins[4 * pix + 0] = o.m_skip;
            margins[4 * pix + 1] = o.m_clamp;
            margins[4 * pix + 2] = o.m_T;
            margins[4 * pix + 3] = mk;
            sig[pix] = o.sig;
        }
        free(bl);
    }
    free_bins(&b);
    free(P);
    return err;
}

/*
 * Vanilla feature render (the alpha-blended feature field that Top-K rendering replaces,
 * Sec. 3.2 and Tab. 4): the D-channel feature blended exactly as the colour of Eq. 1,
 * over every blended Gaussian, F[p*D + ch] = sum_i w_i feat[id_i*D + ch], with the
 * weights w_i = alpha_i T_i of the same blend.  feat[n*D] holds FP64 features.
 */
int orc_vanilla_feature(int n, const float *means, const float *ls, const float *q, const float *opl,
                        const float *rgb, const float *cam, int W, int H, int D, const double *feat,
                        double *F)
{
    cam_t c;
    cam_from(cam, W, H, &c);
    proj_t *P = project_all(&c, n, means, ls, q, opl, rgb);
    if (!P) return -1;
    bins_t b;
    if (make_bins(P, n, W, H, 0, &b)) { free(P); return -1; }
    int cap = max_list_len(&b) + 1;
    int err = 0;
#pragma omp parallel
    {
        blend_t *bl = (blend_t *)malloc(sizeof(blend_t) * (size_t)cap);
        if (!bl) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 64)
        for (long pix = 0; pix < (long)W * H; ++pix) {
            if (!bl) continue;
            int x = (int)(pix % W), y = (int)(pix / W);
            int t = (y / ORC_TILE) * b.ntx + x / ORC_TILE;
            pix_t o;
            blend_pixel(P, rgb, b.list + b.start[t], b.start[t + 1] - b.start[t], x, y, 1, bl, &o);
            double *out = F + pix * D;
            for (int ch = 0; ch < D; ++ch) out[ch] = 0;
            for (int i = 0; i < o.n; ++i) {
                const double *f = feat + (long)bl[i].id * D;
                for (int ch = 0; ch < D; ++ch) out[ch] += bl[i].w * f[ch];
            }
        }
        free(bl);
    }
    free_bins(&b);
    free(P);
    return err;
}

/*
 * Pruning statistics of Sec. 3.3 for one view, accumulated into the caller's arrays:
 *   count[g] += number of pixels whose Top-K list (Eq. 2) holds g;
 *   maxw[g] = max(maxw[g], w) over every pixel where g is blended (Eq. 5's S_g: the
 *   largest blending weight alpha T the Gaussian reaches).
 * Each thread keeps its own arrays; they are merged after the pixel loop.
 */
int orc_prune_stats(int n, const float *means, const float *ls, const float *q, const float *opl,
                    const float *rgb, const float *cam, int W, int H, int K, int *count, double *maxw)
{
    if (K < 1 || K > 63) return -2;
    cam_t c;
    cam_from(cam, W, H, &c);
    proj_t *P = project_all(&c, n, means, ls, q, opl, rgb);
    if (!P) return -1;
    bins_t b;
    if (make_bins(P, n, W, H, 0, &b)) { free(P); return -1; }
    int cap = max_list_len(&b) + 1;
    int err = 0;
#pragma omp parallel
    {
        blend_t *bl = (blend_t *)malloc(sizeof(blend_t) * (size_t)cap);
        int *cnt = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
        double *mw = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        int ids[64];
        double ws[64];
        if (!bl || !cnt || !mw) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 64)
        for (long pix = 0; pix < (long)W * H; ++pix) {
            if (!bl || !cnt || !mw) continue;
            int x = (int)(pix % W), y = (int)(pix / W);
            int t = (y / ORC_TILE) * b.ntx + x / ORC_TILE;
            pix_t o;
            blend_pixel(P, rgb, b.list + b.start[t], b.start[t + 1] - b.start[t], x, y, 1, bl, &o);
            for (int i = 0; i < o.n; ++i)
                if (bl[i].w > mw[bl[i].id]) mw[bl[i].id] = bl[i].w;
            double mk;
            topk_of(bl, o.n, K, ids, ws, NULL, &mk);
            for (int k = 0; k < K; ++k)
                if (ids[k] >= 0) cnt[ids[k]] += 1;
        }
#pragma omp critical
        {
            if (cnt && mw)
                for (int g = 0; g < n; ++g) {
                    count[g] += cnt[g];
                    if (mw[g] > maxw[g]) maxw[g] = mw[g];
                }
        }
        free(bl);
        free(cnt);
        free(mw);
    }
    free_bins(&b);
    free(P);
    return err;
}

/* Eq. 3-4: F[p] = sum_k (w_k / W) f_{id_k}, W = sum_k w_k, F = 0 where W = 0. */
int orc_feature(long n_pix, int K, int D, const int *ids, const double *w, const double *feat,
                double *F)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < n_pix; ++p) {
        double Wsum = 0;
        for (int k = 0; k < K; ++k) Wsum += w[p * K + k];
        double *out = F + p * D;
        for (int c = 0; c < D; ++c) out[c] = 0;
        if (Wsum == 0) continue;
        for (int k = 0; k < K; ++k) {
            int g = ids[p * K + k];
            if (g < 0) continue;
            double wp = w[p * K + k] / Wsum;
            for (int c = 0; c < D; ++c) out[c] += wp * feat[(long)g * D + c];
        }
    }
    return 0;
}

/* Adjoint of Eq. 3-4 alone, for given Top-K ids/weights and upstream gF[P*D]:
   with W = sum_k w_k, w'_k = w_k / W, g_k = <gF, f_k>:
     d_feat[id_k] += w'_k gF  (d_feat[n*D] is overwritten first),
     d_w[p*K + k] = (g_k - sum_j w'_j g_j) / W  (0 where W = 0 or the slot is empty). */
int orc_feature_backward(long n_pix, int K, int D, int n, const int *ids, const double *w,
                         const double *feat, const double *gF, double *d_feat, double *d_w)
{
    memset(d_feat, 0, sizeof(double) * (size_t)n * D);
    for (long p = 0; p < n_pix; ++p) {
        double Wsum = 0, gk[64], mean = 0;
        for (int k = 0; k < K; ++k) Wsum += w[p * K + k];
        for (int k = 0; k < K; ++k) {
            gk[k] = 0;
            d_w[p * K + k] = 0;
        }
        if (Wsum == 0) continue;
        for (int k = 0; k < K; ++k) {
            int g = ids[p * K + k];
            if (g < 0) continue;
            double s = 0;
            for (int c = 0; c < D; ++c) s += gF[p * D + c] * feat[(long)g * D + c];
            gk[k] = s;
            double wp = w[p * K + k] / Wsum;
            mean += wp * s;
            for (int c = 0; c < D; ++c) d_feat[(long)g * D + c] += wp * gF[p * D + c];
        }
        for (int k = 0; k < K; ++k)
            if (ids[p * K + k] >= 0) d_w[p * K + k] = (gk[k] - mean) / Wsum;
    }
    return 0;
}

/* ------------------------------------------------------------------- backward */

/* Per-Gaussian screen-space gradient slots. */
enum { G_MX, G_MY, G_CA, G_CB, G_CC, G_OP, G_R, G_G, G_B, G_Z, G_NS };

/*
 * Backward of one view for the upstream gradients gC[P*3], gD[P], gO[P], gF[P*D]
 * (any may be NULL = zero).  feat holds the stored features exactly dequantized.
 * Writes (overwrites) per-Gaussian screen-space gradients
 *   d_mean2d[2n], d_conic[3n] (a, b, c of sigma = a dx^2/2 + b dx dy + c dy^2/2),
 *   d_opac[n], d_rgb[3n], d_z[n]  (all may be NULL),
 * the per-slot Top-K weight gradient d_topkw[P*K] (may be NULL),
 * the parameter gradients d_means[3n], d_ls[3n], d_q[4n], d_opl[n], d_feat[n*D],
 * With vanilla != 0 the upstream gF is that of the vanilla feature render
 * (orc_vanilla_feature) instead of the Top-K one: every blended Gaussian then receives
 * the feature term, d_feat[id_i] += w_i gF and e_i += <gF, f_i>, and d_topkw is zero.
 * Also the camera-pose gradients (both may be NULL):
 *   d_Rt[12]: partial derivatives with respect to the 12 entries of the world->camera
 *             [R|t] (row-major 3x4), each entry taken as an independent variable;
 *   d_pose[6]: the gradient with respect to a pose increment xi = (rho, phi) applied on
 *             the left, [R|t] <- exp(xi^) [R|t], i.e. R <- (I + [phi]x) R and
 *             t <- (I + [phi]x) t + rho to first order (the rendering-loss pose
 *             refinement of Sec. 4.1): rho first, then phi.
 */
int orc_backward(int n, const float *means, const float *ls, const float *q, const float *opl,
                 const float *rgb, const float *cam, int W, int H, int K, int D,
                 const double *feat, const double *gC, const double *gD, const double *gO,
                 const double *gF,
                 double *d_mean2d, double *d_conic, double *d_opac, double *d_rgb, double *d_z,
                 double *d_topkw,
                 double *d_means, double *d_ls, double *d_q, double *d_opl, double *d_feat,
                 double *d_Rt, double *d_pose, int vanilla)
{
    if (K < 1 || K > 63) return -2;
    cam_t c;
    cam_from(cam, W, H, &c);
    proj_t *P = project_all(&c, n, means, ls, q, opl, rgb);
    if (!P) return -1;
    bins_t b;
    if (make_bins(P, n, W, H, 0, &b)) { free(P); return -1; }
    int cap = max_list_len(&b) + 1;
    long NP = (long)W * H;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthr * (size_t)n * G_NS, sizeof(double));
    /* per pixel Top-K ids and normalized weights, for the feature scatter below */
    int *tk_id = (int *)malloc(sizeof(int) * (size_t)NP * K);
    double *tk_wp = (double *)malloc(sizeof(double) * (size_t)NP * K);
    /* blended count per pixel, for the vanilla feature gradient */
    int *nbl = vanilla ? (int *)malloc(sizeof(int) * (size_t)NP) : NULL;
    if (!acc || !tk_id || !tk_wp || (vanilla && !nbl)) {
        free(acc); free(tk_id); free(tk_wp); free(nbl); free_bins(&b); free(P); return -1;
    }
    int err = 0;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *my = acc + (size_t)tid * (size_t)n * G_NS;
        blend_t *bl = (blend_t *)malloc(sizeof(blend_t) * (size_t)cap);
        double *e = (double *)malloc(sizeof(double) * (size_t)cap);
        if (!bl || !e) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 64)
        for (long pix = 0; pix < NP; ++pix) {
            if (!bl || !e) continue;
            int x = (int)(pix % W), y = (int)(pix / W);
            int t = (y / ORC_TILE) * b.ntx + x / ORC_TILE;
            pix_t o;
            blend_pixel(P, rgb, b.list + b.start[t], b.start[t + 1] - b.start[t], x, y, 1, bl, &o);
            int ids[64], pos[64];
            double ws[64], mk;
            topk_of(bl, o.n, K, ids, ws, pos, &mk);
            double Wsum = 0;
            for (int k = 0; k < K; ++k) Wsum += ws[k];
            /* feature terms: g_k = <gF, f_k>; gamma_k = (g_k - sum_j w'_j g_j) / W */
            double gam[64], gk[64], mean_g = 0;
            for (int k = 0; k < K; ++k) {
                gk[k] = 0;
                gam[k] = 0;
                tk_id[pix * K + k] = -1;
                tk_wp[pix * K + k] = 0;
            }
            if (nbl) nbl[pix] = o.n;
            if (Wsum > 0 && !vanilla) {
                for (int k = 0; k < K; ++k) {
                    if (ids[k] < 0) continue;
                    double s = 0;
                    if (gF)
                        for (int ch = 0; ch < D; ++ch) s += gF[pix * D + ch] * feat[(long)ids[k] * D + ch];
                    gk[k] = s;
                    mean_g += (ws[k] / Wsum) * s;
                    tk_id[pix * K + k] = ids[k];
                    tk_wp[pix * K + k] = ws[k] / Wsum;
                }
                for (int k = 0; k < K; ++k)
                    if (ids[k] >= 0) gam[k] = (gk[k] - mean_g) / Wsum;
            }
            if (d_topkw)
                for (int k = 0; k < K; ++k) d_topkw[pix * K + k] = gam[k];
            /* direct weight gradient e_i (O = sum_i w_i, so gO enters every e_i) */
            double gc0 = gC ? gC[3 * pix] : 0, gc1 = gC ? gC[3 * pix + 1] : 0, gc2 = gC ? gC[3 * pix + 2] : 0;
            double gd = gD ? gD[pix] : 0, go = gO ? gO[pix] : 0;
            for (int i = 0; i < o.n; ++i) {
                const float *cc = rgb + 3 * bl[i].id;
                e[i] = gc0 * cc[0] + gc1 * cc[1] + gc2 * cc[2] + gd * P[bl[i].id].t[2] + go;
            }
            for (int k = 0; k < K; ++k)
                if (pos[k] >= 0) e[pos[k]] += gam[k];
            if (vanilla && gF)   /* the feature blended like the colour: e_i += <gF, f_i> */
                for (int i = 0; i < o.n; ++i) {
                    double sdot = 0;
                    for (int ch = 0; ch < D; ++ch) sdot += gF[pix * D + ch] * feat[(long)bl[i].id * D + ch];
                    e[i] += sdot;
                }
            /* back to front: dL/dalpha_i = T_i e_i - (sum_{j>i} e_j w_j) / (1 - alpha_i) */
            double A = 0;
            for (int i = o.n - 1; i >= 0; --i) {
                const blend_t *bi = &bl[i];
                double dal = bi->T * e[i] - A / (1.0 - bi->alpha);
                A += e[i] * bi->w;
                double *a = my + (size_t)bi->id * G_NS;
                a[G_R] += bi->w * gc0;
                a[G_G] += bi->w * gc1;
                a[G_B] += bi->w * gc2;
                a[G_Z] += bi->w * gd;
                if (bi->clamped) continue;
                const proj_t *p = &P[bi->id];
                double dsig = -bi->alpha * dal;          /* alpha = o e^-sigma */
                a[G_OP] += dal * bi->ex;
                /* sigma = a dx^2/2 + b dx dy + c dy^2/2 with d = pixel - mean2D */
                a[G_MX] += dsig * -(p->con[0] * bi->dx + p->con[1] * bi->dy);
                a[G_MY] += dsig * -(p->con[1] * bi->dx + p->con[2] * bi->dy);
                a[G_CA] += dsig * 0.5 * bi->dx * bi->dx;
                a[G_CB] += dsig * bi->dx * bi->dy;
                a[G_CC] += dsig * 0.5 * bi->dy * bi->dy;
            }
        }
        free(bl);
        free(e);
    }
    if (err) { free(acc); free(tk_id); free(tk_wp); free(nbl); free_bins(&b); free(P); return err; }
    /* reduce the per-thread slots */
    for (int t = 1; t < nthr; ++t) {
        double *src = acc + (size_t)t * (size_t)n * G_NS;
        for (size_t i = 0; i < (size_t)n * G_NS; ++i) acc[i] += src[i];
    }
    /* feature gradient, vanilla: dL/df_i += w_i gF over every blended (pixel, Gaussian);
       the blended lists are replayed into CSR form, then channels are split over threads */
    if (d_feat && vanilla) {
        memset(d_feat, 0, sizeof(double) * (size_t)n * D);
        long *off = (long *)malloc(sizeof(long) * (size_t)(NP + 1));
        off[0] = 0;
        for (long pix = 0; pix < NP; ++pix) off[pix + 1] = off[pix] + nbl[pix];
        int *pid = (int *)malloc(sizeof(int) * (size_t)(off[NP] > 0 ? off[NP] : 1));
        double *pw = (double *)malloc(sizeof(double) * (size_t)(off[NP] > 0 ? off[NP] : 1));
        if (gF && pid && pw) {
#pragma omp parallel
            {
                blend_t *bl = (blend_t *)malloc(sizeof(blend_t) * (size_t)cap);
#pragma omp for schedule(dynamic, 64)
                for (long pix = 0; pix < NP; ++pix) {
                    int x = (int)(pix % W), y = (int)(pix / W);
                    int t = (y / ORC_TILE) * b.ntx + x / ORC_TILE;
                    pix_t o;
                    blend_pixel(P, rgb, b.list + b.start[t], b.start[t + 1] - b.start[t], x, y, 1, bl, &o);
                    for (int i = 0; i < o.n; ++i) {
                        pid[off[pix] + i] = bl[i].id;
                        pw[off[pix] + i] = bl[i].w;
                    }
                }
                free(bl);
            }
#pragma omp parallel for schedule(dynamic, 1)
            for (int c0 = 0; c0 < D; c0 += 8) {
                int c1 = c0 + 8 < D ? c0 + 8 : D;
                for (long pix = 0; pix < NP; ++pix)
                    for (long j = off[pix]; j < off[pix + 1]; ++j) {
                        double *dst = d_feat + (long)pid[j] * D;
                        const double *src = gF + pix * D;
                        for (int ch = c0; ch < c1; ++ch) dst[ch] += pw[j] * src[ch];
                    }
            }
        }
        free(off); free(pid); free(pw);
    }
    /* feature gradient: dL/df_k += w'_k gF */
    if (d_feat && !vanilla) {
        memset(d_feat, 0, sizeof(double) * (size_t)n * D);
        if (gF)
            for (long pix = 0; pix < NP; ++pix)
                for (int k = 0; k < K; ++k) {
                    int g = tk_id[pix * K + k];
                    if (g < 0) continue;
                    double wp = tk_wp[pix * K + k];
                    double *dst = d_feat + (long)g * D;
                    const double *src = gF + pix * D;
                    for (int ch = 0; ch < D; ++ch) dst[ch] += wp * src[ch];
                }
    }
    free(tk_id);
    free(tk_wp);
    free(nbl);

    /* chain rule, per Gaussian */
    double rt[12] = {0};
#pragma omp parallel for schedule(static) reduction(+ : rt[:12])
    for (int g = 0; g < n; ++g) {
        const double *a = acc + (size_t)g * G_NS;
        const proj_t *p = &P[g];
        if (d_mean2d) { d_mean2d[2 * g] = a[G_MX]; d_mean2d[2 * g + 1] = a[G_MY]; }
        if (d_conic) { d_conic[3 * g] = a[G_CA]; d_conic[3 * g + 1] = a[G_CB]; d_conic[3 * g + 2] = a[G_CC]; }
        if (d_opac) d_opac[g] = a[G_OP];
        if (d_rgb) { d_rgb[3 * g] = a[G_R]; d_rgb[3 * g + 1] = a[G_G]; d_rgb[3 * g + 2] = a[G_B]; }
        if (d_z) d_z[g] = a[G_Z];
        double dmu[3] = {0, 0, 0}, dls[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop = 0;
        if (p->valid) {
            double tx = p->t[0], ty = p->t[1], tz = p->t[2];
            /* conic (a, b, c) -> Sigma2D.  With Q = Sigma2D^-1, dL/dSigma2D = -Q G Q where
               G is the symmetric gradient w.r.t. Q: [[ga, gb/2], [gb/2, gc]] */
            double Q[2][2] = {{p->con[0], p->con[1]}, {p->con[1], p->con[2]}};
            double G[2][2] = {{a[G_CA], 0.5 * a[G_CB]}, {0.5 * a[G_CB], a[G_CC]}};
            double QG[2][2], GS[2][2];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) QG[i][j] = Q[i][0] * G[0][j] + Q[i][1] * G[1][j];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) GS[i][j] = -(QG[i][0] * Q[0][j] + QG[i][1] * Q[1][j]);
            /* Sigma2D = Tm Sig Tm^T (+0.3 I): dSig = Tm^T GS Tm, dTm = 2 GS Tm Sig */
            double dSig[3][3], dTm[2][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 2; ++l) s += p->Tm[k][i] * GS[k][l] * p->Tm[l][j];
                    dSig[i][j] = s;
                }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 3; ++l) s += GS[i][k] * p->Tm[k][l] * p->Sig[l][j];
                    dTm[i][j] = 2 * s;
                }
            /* Tm = J Rcam: dJ = dTm Rcam^T */
            double dJ[2][3];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += dTm[i][k] * c.R[j][k];
                    dJ[i][j] = s;
                }
            /* J entries as functions of t (with the guard-band clamp) */
            double dt[3] = {0, 0, 0};
            double fx = c.fx, fy = c.fy;
            dt[2] += dJ[0][0] * (-fx / (tz * tz)) + dJ[1][1] * (-fy / (tz * tz));
            if (!p->clampx) {
                dt[0] += dJ[0][2] * (-fx / (tz * tz));
                dt[2] += dJ[0][2] * (2 * fx * tx / (tz * tz * tz));
            } else {
                double L = tx / tz < 0 ? -p->limx : p->limx;   /* J02 = -fx L / tz */
                dt[2] += dJ[0][2] * (fx * L / (tz * tz));
            }
            if (!p->clampy) {
                dt[1] += dJ[1][2] * (-fy / (tz * tz));
                dt[2] += dJ[1][2] * (2 * fy * ty / (tz * tz * tz));
            } else {
                double L = ty / tz < 0 ? -p->limy : p->limy;
                dt[2] += dJ[1][2] * (fy * L / (tz * tz));
            }
            /* mean2D = (fx tx/tz + cx, fy ty/tz + cy) */
            dt[0] += a[G_MX] * fx / tz;
            dt[1] += a[G_MY] * fy / tz;
            dt[2] += a[G_MX] * (-fx * tx / (tz * tz)) + a[G_MY] * (-fy * ty / (tz * tz));
            /* rendered depth uses z = tz */
            dt[2] += a[G_Z];
            /* t = Rcam mu + tcam */
            for (int j = 0; j < 3; ++j)
                dmu[j] = c.R[0][j] * dt[0] + c.R[1][j] * dt[1] + c.R[2][j] * dt[2];
            /* the camera's own entries: t_i = sum_j R_ij mu_j + tcam_i gives dR_ij += dt_i mu_j
               and dtcam_i += dt_i; Tm = J Rcam gives dRcam = J^T dTm, with J (2x3) as
               projected: J00 = fx/tz, J02 = -fx xc/tz, J11 = fy/tz, J12 = -fy yc/tz, where
               xc, yc are the (clamped) ratios tx/tz, ty/tz */
            double xc = p->clampx ? (tx / tz < 0 ? -p->limx : p->limx) : tx / tz;
            double yc = p->clampy ? (ty / tz < 0 ? -p->limy : p->limy) : ty / tz;
            double Jm[2][3] = {{fx / tz, 0, -fx * xc / tz}, {0, fy / tz, -fy * yc / tz}};
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j)
                    rt[4 * i + j] += dt[i] * (double)means[3 * g + j] + Jm[0][i] * dTm[0][j] + Jm[1][i] * dTm[1][j];
                rt[4 * i + 3] += dt[i];
            }
            /* Sig = M M^T with M = Rq diag(s): dM = 2 dSig M (dSig symmetric) */
            double M[3][3], dM[3][3];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) M[i][j] = p->Rq[i][j] * p->s[j];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += (dSig[i][k] + dSig[k][i]) * M[k][j];
                    dM[i][j] = s;
                }
            /* M_ij = Rq_ij s_j */
            double dRq[3][3];
            for (int j = 0; j < 3; ++j) {
                double ds = 0;
                for (int i = 0; i < 3; ++i) {
                    ds += dM[i][j] * p->Rq[i][j];
                    dRq[i][j] = dM[i][j] * p->s[j];
                }
                dls[j] = ds * p->s[j];
            }
            /* Rq(q^) for q^ = (w, x, y, z) */
            double w = p->qn[0], x = p->qn[1], y = p->qn[2], z = p->qn[3];
            double dqn[4];
            dqn[0] = 2 * (-z * dRq[0][1] + y * dRq[0][2] + z * dRq[1][0] - x * dRq[1][2] - y * dRq[2][0] + x * dRq[2][1]);
            dqn[1] = 2 * (y * dRq[0][1] + z * dRq[0][2] + y * dRq[1][0] - 2 * x * dRq[1][1] - w * dRq[1][2] +
                          z * dRq[2][0] + w * dRq[2][1] - 2 * x * dRq[2][2]);
            dqn[2] = 2 * (-2 * y * dRq[0][0] + x * dRq[0][1] + w * dRq[0][2] + x * dRq[1][0] + z * dRq[1][2] -
                          w * dRq[2][0] + z * dRq[2][1] - 2 * y * dRq[2][2]);
            dqn[3] = 2 * (-2 * z * dRq[0][0] - w * dRq[0][1] + x * dRq[0][2] + w * dRq[1][0] - 2 * z * dRq[1][1] +
                          y * dRq[1][2] + x * dRq[2][0] + y * dRq[2][1]);
            /* q^ = q / |q| */
            double dot = dqn[0] * w + dqn[1] * x + dqn[2] * y + dqn[3] * z;
            for (int i = 0; i < 4; ++i) dq[i] = (dqn[i] - p->qn[i] * dot) / p->qnorm;
            dop = a[G_OP] * p->o * (1 - p->o);
        }
        for (int i = 0; i < 3; ++i) {
            if (d_means) d_means[3 * g + i] = dmu[i];
            if (d_ls) d_ls[3 * g + i] = dls[i];
        }
        if (d_q)
            for (int i = 0; i < 4; ++i) d_q[4 * g + i] = dq[i];
        if (d_opl) d_opl[g] = dop;
    }
    if (d_Rt)
        for (int i = 0; i < 12; ++i) d_Rt[i] = rt[i];
    if (d_pose) {
        /* rho: t <- t + rho, so dL/drho = dL/dt.  phi: dR = [phi]x R and dt = phi x t, so
           dL = sum_ij GR_ij ([phi]x R)_ij + Gt . (phi x t), with GR, Gt the partials above */
        double GR[3][3], Gt[3], M[3][3];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) GR[i][j] = rt[4 * i + j];
            Gt[i] = rt[4 * i + 3];
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s = 0;
                for (int k = 0; k < 3; ++k) s += c.R[i][k] * GR[j][k];
                M[i][j] = s;   /* (R GR^T)_ij */
            }
        /* sum_ij GR_ij (S R)_ij = sum_ik S_ik M_ki for S = [phi]x = [[0, -pz, py],
           [pz, 0, -px], [-py, px, 0]]: collecting px, py, pz gives the three lines below */
        double dphi[3];
        dphi[0] = M[1][2] - M[2][1];
        dphi[1] = M[2][0] - M[0][2];
        dphi[2] = M[0][1] - M[1][0];
        /* phi . (t x Gt) */
        dphi[0] += c.t[1] * Gt[2] - c.t[2] * Gt[1];
        dphi[1] += c.t[2] * Gt[0] - c.t[0] * Gt[2];
        dphi[2] += c.t[0] * Gt[1] - c.t[1] * Gt[0];
        for (int i = 0; i < 3; ++i) {
            d_pose[i] = Gt[i];
            d_pose[3 + i] = dphi[i];
        }
    }
    free(acc);
    free_bins(&b);
    free(P);
    return 0;
}

/* ----------------------------------------------------------------- quantizers */

/* bfloat16 from FP32 by round-to-nearest-even: of the two bfloat16 values that
   bracket x (truncation and the next one away from zero), take the nearer; on a tie
   the one whose last kept bit is 0.  Non-finite inputs keep their class. */
int orc_bf16_from_f32(long n, const float *x, uint16_t *out)
{
    for (long i = 0; i < n; ++i) {
        uint32_t u;
        memcpy(&u, &x[i], 4);
        if (!isfinite(x[i])) {
            out[i] = (uint16_t)((u >> 16) | (isnan(x[i]) ? 0x40u : 0u));
            continue;
        }
        uint32_t lo = u & 0xFFFF0000u, hi = lo + 0x10000u;
        float flo, fhi;
        memcpy(&flo, &lo, 4);
        memcpy(&fhi, &hi, 4);
        double dl = fabs((double)x[i] - (double)flo);
        double dh = isfinite(fhi) ? fabs((double)fhi - (double)x[i]) : INFINITY;
        uint32_t pick;
        if (!isfinite(fhi)) {
            /* above the largest finite bfloat16: the midpoint to 2^128 decides */
            double mid = (double)flo + ldexp(1.0, 127 - 8);
            pick = fabs((double)x[i]) >= mid ? ((u & 0x80000000u) | 0x7F800000u) : lo;
        } else if (dl < dh) pick = lo;
        else if (dh < dl) pick = hi;
        else pick = ((lo >> 16) & 1u) ? hi : lo;
        out[i] = (uint16_t)(pick >> 16);
    }
    return 0;
}

double orc_bf16_value(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* OCP FP8 E4M3FN: 1 sign, 4 exponent (bias 7), 3 mantissa bits; no infinities;
   S.1111.111 is NaN; subnormals (m/8) 2^-6; largest finite 448. */
double orc_e4m3_value(uint8_t code)
{
    int s = code >> 7, e = (code >> 3) & 15, m = code & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m / 8.0, -6);
    else v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

/* Nearest E4M3FN code to v by exhaustive search over the 127 finite non-negative codes;
   ties go to the even code (last mantissa bit 0); magnitudes past 448 saturate. */
static uint8_t e4m3_nearest(double v)
{
    int neg = signbit(v) ? 1 : 0;
    double a = fabs(v);
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 126; ++c) {
        double d = fabs(orc_e4m3_value((uint8_t)c) - a);
        if (d < bd || (d == bd && (c & 1) == 0)) { bd = d; best = c; }
    }
    return (uint8_t)((neg << 7) | best);
}

/* Per-row FP8 quantization with a power-of-two scale s = 2^floor(log2(amax / 224)),
   so every x / s is exact and amax / s lies in [224, 448); amax = 0 gives s = 1. */
int orc_fp8_quantize(long n, int D, const float *x, uint8_t *codes, float *scale)
{
#pragma omp parallel for schedule(static)
    for (long r = 0; r < n; ++r) {
        double amax = 0;
        for (int c = 0; c < D; ++c) {
            double a = fabs((double)x[r * D + c]);
            if (a > amax) amax = a;
        }
        double s = 1.0;
        if (amax > 0) {
            int ex;
            frexp(amax / 224.0, &ex);       /* amax/224 = f 2^ex, f in [0.5, 1) */
            int e = ex - 1;
            if (e < -126) e = -126;
            s = ldexp(1.0, e);
        }
        scale[r] = (float)s;
        for (int c = 0; c < D; ++c) codes[r * D + c] = e4m3_nearest((double)x[r * D + c] / s);
    }
    return 0;
}

int orc_e4m3_table(double *out256)
{
    for (int c = 0; c < 256; ++c) out256[c] = orc_e4m3_value((uint8_t)c);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the OpenMP thread count of later calls; returns the count now in effect. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
