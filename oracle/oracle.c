/*
 * FP64 CPU oracle of the differentiable tile rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * called from the test suite, the smoke check and the benchmark's CPU
 * baseline.  It shares no code, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * What it computes (paper: §3.1 "Preliminary", Eq. 1 and Eq. 2):
 *   - every 3D Gaussian G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) with
 *     Sigma built from a rotation R and a scale S (Eq. 1);
 *   - is projected onto the image plane as a 2D Gaussian G' (the sentence
 *     after Eq. 1; the paper gives no formulas, the EWA linearisation of the
 *     perspective map is used);
 *   - and the pixel colour is the depth-ordered alpha blend
 *     C(x_p) = sum_i c_i o_i G'_i(x_p) prod_{j<i} (1 - o_j G'_j(x_p))   (Eq. 2).
 * The paper is silent on the rasterizer's discrete rules; the readings used
 * here are: near/far culling; quaternion (w,x,y,z) normalised inside;
 * Jacobian frustum clamp at the image extent +15%% per side; 2D low-pass
 * dilation (0.3 px^2) with optional opacity compensation (the anti-aliasing
 * of §3.5.4); pixel centres at integer + 0.5; 3-sigma extent of the largest
 * eigenvalue rounded up; integer tile rectangle of 16x16 tiles; real SH up
 * to degree 3 with +0.5 offset and clamp at 0; pairs ordered by
 * (tile, float32 depth bits, index); alpha = min(0.99, o' G'); skip
 * alpha < 1/255; stop before compositing an entry that would take the
 * transmittance below 1e-4; accumulated depth D = sum z_i alpha_i T_i for the
 * depth regulariser of §3.5.3.
 *
 * Everything is evaluated in double precision, pixel by pixel, in the
 * plainest form: no tiling tricks beyond the tile rectangles that define
 * which Gaussians a pixel sees, no reordering, no fused recurrences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16
#define ORC_ALPHA_MAX 0.99
#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_T_MIN 1e-4

typedef struct {
    double fx, fy, cx, cy;
    double R[3][3];          /* world -> camera rotation */
    double t[3];             /* world -> camera translation */
    int32_t W, H;
    double znear, zfar;
} ocam_t;

typedef struct {
    int32_t sh_degree;       /* 0..3 */
    double dilation;         /* px^2 added to the 2D covariance diagonal */
    int32_t aa;              /* 1: opacity compensation by rho */
    double bg[3];
} oopt_t;

/* per-slot projection outputs (arrays of n entries times the component count) */
typedef struct {
    int32_t *visible;        /* [n] */
    double *tcam;            /* [n][3] */
    double *cov2d;           /* [n][3] a, b, c before dilation */
    double *rho;             /* [n] */
    double *conic;           /* [n][3] A, B, C of the inverse dilated covariance */
    double *mean2d;          /* [n][2] */
    double *depth;           /* [n] */
    double *opac;            /* [n] o' = o * rho */
    double *rgb;             /* [n][3] */
    int32_t *clamped;        /* [n][3] raw colour < 0 */
    double *extent;          /* [n] 3 sqrt(lambda_max), before rounding up */
    int32_t *radius;         /* [n] */
    int32_t *rect;           /* [n][4] tile x0, y0, x1, y1 (inclusive) */
    int32_t *tiles;          /* [n] number of tiles covered, 0 if culled */
} oproj_t;

/* ------------------------------------------------------------------------ */
/* real spherical harmonics, degree <= 3, on a unit direction                */
/* ------------------------------------------------------------------------ */

/* Real SH with the Condon-Shortley phase kept: for m > 0 the basis is
 * sqrt(2) Re Y_l^m, for m < 0 it is sqrt(2) Im Y_l^|m|, ordered m = -l..l.
 * Written as polynomials in (x, y, z) that are valid on the unit sphere. */
static void sh_basis(double x, double y, double z, double Y[16]) {
    const double pi = M_PI;
    const double k0 = 0.5 * sqrt(1.0 / pi);
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2 = 0.5 * sqrt(15.0 / pi);
    const double k6 = 0.25 * sqrt(5.0 / pi);
    const double k8 = 0.25 * sqrt(15.0 / pi);
    const double k9 = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double k10 = 0.5 * sqrt(105.0 / pi);
    const double k11 = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double k12 = 0.25 * sqrt(7.0 / pi);
    const double k14 = 0.25 * sqrt(105.0 / pi);
    Y[0] = k0;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2 * x * y;
    Y[5] = -k2 * y * z;
    Y[6] = k6 * (2.0 * z * z - x * x - y * y);
    Y[7] = -k2 * x * z;
    Y[8] = k8 * (x * x - y * y);
    Y[9] = -k9 * y * (3.0 * x * x - y * y);
    Y[10] = k10 * x * y * z;
    Y[11] = -k11 * y * (4.0 * z * z - x * x - y * y);
    Y[12] = k12 * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -k11 * x * (4.0 * z * z - x * x - y * y);
    Y[14] = k14 * z * (x * x - y * y);
    Y[15] = -k9 * x * (x * x - 3.0 * y * y);
}

/* gradient of each basis polynomial with respect to (x, y, z) */
static void sh_basis_grad(double x, double y, double z, double dY[16][3]) {
    const double pi = M_PI;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2 = 0.5 * sqrt(15.0 / pi);
    const double k6 = 0.25 * sqrt(5.0 / pi);
    const double k8 = 0.25 * sqrt(15.0 / pi);
    const double k9 = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double k10 = 0.5 * sqrt(105.0 / pi);
    const double k11 = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double k12 = 0.25 * sqrt(7.0 / pi);
    const double k14 = 0.25 * sqrt(105.0 / pi);
    memset(dY, 0, sizeof(double) * 48);
    dY[1][1] = -k1;
    dY[2][2] = k1;
    dY[3][0] = -k1;
    dY[4][0] = k2 * y;           dY[4][1] = k2 * x;
    dY[5][1] = -k2 * z;          dY[5][2] = -k2 * y;
    dY[6][0] = -2.0 * k6 * x;    dY[6][1] = -2.0 * k6 * y;   dY[6][2] = 4.0 * k6 * z;
    dY[7][0] = -k2 * z;          dY[7][2] = -k2 * x;
    dY[8][0] = 2.0 * k8 * x;     dY[8][1] = -2.0 * k8 * y;
    dY[9][0] = -6.0 * k9 * x * y;
    dY[9][1] = -k9 * (3.0 * x * x - 3.0 * y * y);
    dY[10][0] = k10 * y * z;     dY[10][1] = k10 * x * z;    dY[10][2] = k10 * x * y;
    dY[11][0] = 2.0 * k11 * x * y;
    dY[11][1] = -k11 * (4.0 * z * z - x * x - 3.0 * y * y);
    dY[11][2] = -8.0 * k11 * y * z;
    dY[12][0] = -6.0 * k12 * x * z;
    dY[12][1] = -6.0 * k12 * y * z;
    dY[12][2] = k12 * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    dY[13][0] = -k11 * (4.0 * z * z - 3.0 * x * x - y * y);
    dY[13][1] = 2.0 * k11 * x * y;
    dY[13][2] = -8.0 * k11 * x * z;
    dY[14][0] = 2.0 * k14 * x * z;
    dY[14][1] = -2.0 * k14 * y * z;
    dY[14][2] = k14 * (x * x - y * y);
    dY[15][0] = -k9 * (3.0 * x * x - 3.0 * y * y);
    dY[15][1] = 6.0 * k9 * x * y;
}

void orc_sh_basis(int64_t n, const double *dirs /* [n][3] */, double *out /* [n][16] */) {
    for (int64_t i = 0; i < n; i++) sh_basis(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], out + 16 * i);
}

/* ------------------------------------------------------------------------ */
/* rotation from a unit quaternion (w, x, y, z)                              */
/* ------------------------------------------------------------------------ */

static void quat_to_rot(const double q[4], double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Sigma = R S S^T R^T of Eq. 1 for one Gaussian, exposed for the pins. */
void orc_cov3d(const double q[4], const double s[3], double out[9]) {
    double qn[4], nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]), R[3][3];
    for (int i = 0; i < 4; i++) qn[i] = q[i] / nq;
    quat_to_rot(qn, R);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += R[i][k] * s[k] * s[k] * R[j][k];
            out[3 * i + j] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian (EWA linearisation of the perspective map)     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int visible;
    double t[3];
    double qn[4], qnorm;
    double Rq[3][3];
    double Sigma[3][3];
    double u, v, uc, vc;
    int u_clamped, v_clamped;
    double J[2][3];
    double Tm[2][3];         /* J * R_cw */
    double a, b, c;          /* 2D covariance before dilation */
    double ad, cd;           /* diagonal after dilation */
    double det2, detd;
    double rho;
    double conic[3];
    double mean2d[2];
    double opac;
    double dir[3], dnorm, dhat[3];
    double Y[16];
    double raw[3];
    double rgb[3];
    int clamped[3];
    double extent;
    int radius;
    int rect[4];
    int tiles;
} proj1_t;

/* cbase: the constant of the colour polynomial per channel (NULL: 0.5, the
 * plain 3DGS offset; with appearance offsets it is their colour part) */
static void project_one(const ocam_t *cam, const oopt_t *opt, const double mu[3], const double s[3],
                        const double q[4], double o, const double *sh, int64_t sh_stride, const double *cbase,
                        proj1_t *P) {
    memset(P, 0, sizeof(*P));
    /* camera-space mean */
    for (int i = 0; i < 3; i++)
        P->t[i] = cam->R[i][0] * mu[0] + cam->R[i][1] * mu[1] + cam->R[i][2] * mu[2] + cam->t[i];
    double tz = P->t[2];
    if (!(tz >= cam->znear && tz <= cam->zfar)) return;

    /* Sigma = R S S^T R^T (Eq. 1) */
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(P->qnorm > 0.0)) return;
    for (int i = 0; i < 4; i++) P->qn[i] = q[i] / P->qnorm;
    quat_to_rot(P->qn, P->Rq);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += P->Rq[i][k] * s[k] * s[k] * P->Rq[j][k];
            P->Sigma[i][j] = acc;
        }

    /* Jacobian of (fx x/z + cx, fy y/z + cy), ratios clamped to the image
     * extent plus 15% of the width (height) on each side */
    P->u = P->t[0] / tz;
    P->v = P->t[1] / tz;
    double ulo = -(cam->cx + 0.15 * cam->W) / cam->fx, uhi = (cam->W - cam->cx + 0.15 * cam->W) / cam->fx;
    double vlo = -(cam->cy + 0.15 * cam->H) / cam->fy, vhi = (cam->H - cam->cy + 0.15 * cam->H) / cam->fy;
    P->uc = P->u;
    P->vc = P->v;
    if (P->uc < ulo) { P->uc = ulo; P->u_clamped = 1; }
    if (P->uc > uhi) { P->uc = uhi; P->u_clamped = 1; }
    if (P->vc < vlo) { P->vc = vlo; P->v_clamped = 1; }
    if (P->vc > vhi) { P->vc = vhi; P->v_clamped = 1; }
    P->J[0][0] = cam->fx / tz; P->J[0][1] = 0.0; P->J[0][2] = -cam->fx * P->uc / tz;
    P->J[1][0] = 0.0; P->J[1][1] = cam->fy / tz; P->J[1][2] = -cam->fy * P->vc / tz;

    /* Sigma_2D = J W Sigma W^T J^T with W the camera rotation */
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++) acc += P->J[i][k] * cam->R[k][j];
            P->Tm[i][j] = acc;
        }
    double S2[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            double acc = 0.0;
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) acc += P->Tm[i][k] * P->Sigma[k][l] * P->Tm[j][l];
            S2[i][j] = acc;
        }
    P->a = S2[0][0];
    P->b = 0.5 * (S2[0][1] + S2[1][0]);
    P->c = S2[1][1];

    /* low-pass dilation and opacity compensation */
    P->ad = P->a + opt->dilation;
    P->cd = P->c + opt->dilation;
    P->det2 = P->a * P->c - P->b * P->b;
    P->detd = P->ad * P->cd - P->b * P->b;
    if (!(P->detd > 0.0)) return;
    P->rho = 1.0;
    if (opt->aa) {
        double ratio = P->det2 / P->detd;
        P->rho = ratio > 0.0 ? sqrt(ratio) : 0.0;
    }
    P->conic[0] = P->cd / P->detd;
    P->conic[1] = -P->b / P->detd;
    P->conic[2] = P->ad / P->detd;
    P->mean2d[0] = cam->fx * P->u + cam->cx;
    P->mean2d[1] = cam->fy * P->v + cam->cy;
    P->opac = o * P->rho;

    /* 3-sigma extent of the largest eigenvalue and the tile rectangle */
    double lmax = 0.5 * (P->ad + P->cd) + sqrt(0.25 * (P->ad - P->cd) * (P->ad - P->cd) + P->b * P->b);
    P->extent = 3.0 * sqrt(lmax);
    if (!isfinite(P->extent) || !isfinite(P->mean2d[0]) || !isfinite(P->mean2d[1])) return;
    double r = ceil(P->extent);
    int TW = (cam->W + ORC_TILE - 1) / ORC_TILE, TH = (cam->H + ORC_TILE - 1) / ORC_TILE;
    double fx0 = floor((floor(P->mean2d[0]) - r) / ORC_TILE), fx1 = floor((floor(P->mean2d[0]) + r) / ORC_TILE);
    double fy0 = floor((floor(P->mean2d[1]) - r) / ORC_TILE), fy1 = floor((floor(P->mean2d[1]) + r) / ORC_TILE);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > TW - 1) fx1 = TW - 1;
    if (fy1 > TH - 1) fy1 = TH - 1;
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    P->radius = (int)(r < 2e9 ? r : 2e9);
    P->rect[0] = (int)fx0; P->rect[1] = (int)fy0; P->rect[2] = (int)fx1; P->rect[3] = (int)fy1;
    P->tiles = (P->rect[2] - P->rect[0] + 1) * (P->rect[3] - P->rect[1] + 1);

    /* view-dependent colour from the world-space viewing direction */
    double campos[3];
    for (int i = 0; i < 3; i++)
        campos[i] = -(cam->R[0][i] * cam->t[0] + cam->R[1][i] * cam->t[1] + cam->R[2][i] * cam->t[2]);
    for (int i = 0; i < 3; i++) P->dir[i] = mu[i] - campos[i];
    P->dnorm = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
    for (int i = 0; i < 3; i++) P->dhat[i] = P->dir[i] / P->dnorm;
    sh_basis(P->dhat[0], P->dhat[1], P->dhat[2], P->Y);
    int nb = (opt->sh_degree + 1) * (opt->sh_degree + 1);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int k = 0; k < nb; k++) acc += sh[(k * 3 + ch) * sh_stride] * P->Y[k];
        P->raw[ch] = acc + (cbase ? cbase[ch] : 0.5);
        P->clamped[ch] = P->raw[ch] < 0.0;
        P->rgb[ch] = P->clamped[ch] ? 0.0 : P->raw[ch];
    }
    P->visible = 1;
}

static void load_params(int64_t n, int64_t i, const double *means, const double *scales, const double *quats,
                        double mu[3], double s[3], double q[4]) {
    for (int k = 0; k < 3; k++) { mu[k] = means[k * n + i]; s[k] = scales[k * n + i]; }
    for (int k = 0; k < 4; k++) q[k] = quats[k * n + i];
}

int orc_project(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                const double *sh, const double *cbase /* [n][3] or NULL */, const ocam_t *cam, const oopt_t *opt,
                oproj_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double mu[3], s[3], q[4];
        load_params(n, i, means, scales, quats, mu, s, q);
        proj1_t P;
        project_one(cam, opt, mu, s, q, opac[i], sh + i, n, cbase ? cbase + 3 * i : NULL, &P);
        out->visible[i] = P.visible;
        for (int k = 0; k < 3; k++) out->tcam[3 * i + k] = P.t[k];
        out->cov2d[3 * i] = P.a; out->cov2d[3 * i + 1] = P.b; out->cov2d[3 * i + 2] = P.c;
        out->rho[i] = P.rho;
        for (int k = 0; k < 3; k++) out->conic[3 * i + k] = P.conic[k];
        out->mean2d[2 * i] = P.mean2d[0]; out->mean2d[2 * i + 1] = P.mean2d[1];
        out->depth[i] = P.t[2];
        out->opac[i] = P.opac;
        for (int k = 0; k < 3; k++) { out->rgb[3 * i + k] = P.rgb[k]; out->clamped[3 * i + k] = P.clamped[k]; }
        out->extent[i] = P.extent;
        out->radius[i] = P.radius;
        for (int k = 0; k < 4; k++) out->rect[4 * i + k] = P.visible ? P.rect[k] : 0;
        out->tiles[i] = P.visible ? P.tiles : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* binning: (tile, depth key, slot) pairs, sorted, and per-tile ranges       */
/* ------------------------------------------------------------------------ */

typedef struct { uint32_t tile, key, slot; } opair_t;

static int pair_cmp(const void *pa, const void *pb) {
    const opair_t *a = (const opair_t *)pa, *b = (const opair_t *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->slot != b->slot) return a->slot < b->slot ? -1 : 1;
    return 0;
}

/* The exponent of G' at pixel centre (px, py) for a Gaussian with 2D mean m
 * and conic (A, B, C), i.e. -1/2 d^T Sigma'^-1 d with d = p - m; also the
 * offsets.  Compositing and tile culling both evaluate this one expression. */
static double entry_power(const double *m, const double *cn, double px, double py, double *dx_out, double *dy_out) {
    double dx = px - m[0], dy = py - m[1];
    *dx_out = dx;
    *dy_out = dy;
    return -0.5 * (cn[0] * dx * dx + cn[2] * dy * dy) - cn[1] * dx * dy;
}

/* Tile-based culling (§3.4.2: a Gaussian whose contribution to a tile is
 * negligible is skipped there).  The reading: an entry contributes nothing
 * to a tile when the skip rule of the blend (alpha = min(0.99, o' G') below
 * 1/255, or a positive exponent) holds at every pixel centre of the tile
 * inside the image.  This tests every such pixel centre with the
 * compositing's own expressions, so culling never changes an image.
 * An exponent more than 1e-9 below ln(1/(255 o')) fails the skip test
 * without evaluating exp (a margin far above the rounding of log and exp). */
static int tile_reached(const double *m, const double *cn, double opac, int tx, int ty, int W, int H) {
    if (!(opac >= ORC_ALPHA_MIN)) return 0;   /* o' G' <= o' since G' <= 1 */
    double lim = log(ORC_ALPHA_MIN / opac) - 1e-9;
    for (int y = ty * ORC_TILE; y < (ty + 1) * ORC_TILE && y < H; y++)
        for (int x = tx * ORC_TILE; x < (tx + 1) * ORC_TILE && x < W; x++) {
            double dx, dy;
            double power = entry_power(m, cn, x + 0.5, y + 0.5, &dx, &dy);
            if (power > 0.0 || power < lim) continue;
            double raw = opac * exp(power);
            double alpha = raw < ORC_ALPHA_MAX ? raw : ORC_ALPHA_MAX;
            if (alpha >= ORC_ALPHA_MIN) return 1;
        }
    return 0;
}

/* Whether tile (tx, ty) of slot s's rectangle is enumerated: its bit in a
 * given covered-tile mask (mask[s] == 0: every tile), and, with 2D records
 * given, tile culling by tile_reached. */
static int tile_kept(int64_t s, int tx, int ty, const int32_t *rect, const uint64_t *mask, const double *mean2d,
                     const double *conic, const double *opac, int W, int H) {
    uint64_t mk = mask ? mask[s] : 0;
    int w = rect[4 * s + 2] - rect[4 * s] + 1;
    if (mk && !((mk >> ((ty - rect[4 * s + 1]) * w + (tx - rect[4 * s]))) & 1)) return 0;
    if (mean2d && !tile_reached(mean2d + 2 * s, conic + 3 * s, opac[s], tx, ty, W, H)) return 0;
    return 1;
}

/* Enumerates one pair per (slot, kept tile of the slot's rectangle; see
 * tile_kept: mask[s] selects tiles of a rectangle computed elsewhere, the
 * nullable 2D records mean2d [n][2], conic [n][3], opac [n] turn on tile
 * culling), sorts the pairs by (global tile id, depth key, slot) --
 * "processed in depth order" of §3.1, ties by input index -- and writes
 * [start, end) per global tile.  slot_view[s] selects the view of a slot;
 * its tiles are numbered view_tile_off[v] + ty * view_tiles_x[v] + tx and
 * its image is view_W[v] x view_H[v].  slot_tiles (nullable) receives the
 * number of pairs of each slot.  Returns P, or -P when P > capacity. */
int64_t orc_bin(int64_t n_slots, const int32_t *rect, const int32_t *tiles, const uint64_t *mask,
                const double *mean2d, const double *conic, const double *opac, const uint32_t *depth_key,
                const int32_t *slot_view, const int32_t *view_tiles_x, const int32_t *view_W, const int32_t *view_H,
                const int32_t *view_tile_off, int64_t n_tiles_total, int64_t capacity, uint32_t *pair_tile,
                uint32_t *pair_slot, uint32_t *ranges /* [n_tiles_total][2] */, int32_t *slot_tiles) {
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_slots + 1));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t s = 0; s < n_slots; s++) {
        int64_t c = 0;
        if (tiles[s] > 0) {
            int v = slot_view[s];
            for (int ty = rect[4 * s + 1]; ty <= rect[4 * s + 3]; ty++)
                for (int tx = rect[4 * s]; tx <= rect[4 * s + 2]; tx++)
                    c += tile_kept(s, tx, ty, rect, mask, mean2d, conic, opac, view_W[v], view_H[v]);
        }
        cnt[s] = c;
    }
    int64_t P = 0;
    for (int64_t s = 0; s < n_slots; s++) {
        int64_t c = cnt[s];
        if (slot_tiles) slot_tiles[s] = (int32_t)c;
        cnt[s] = P;
        P += c;
    }
    if (P > capacity) { free(cnt); return -P; }
    opair_t *pairs = (opair_t *)malloc(sizeof(opair_t) * (size_t)(P > 0 ? P : 1));
    if (!pairs) { free(cnt); return -1; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t s = 0; s < n_slots; s++) {
        if (tiles[s] <= 0) continue;
        int v = slot_view[s];
        int64_t k = cnt[s];
        for (int ty = rect[4 * s + 1]; ty <= rect[4 * s + 3]; ty++)
            for (int tx = rect[4 * s]; tx <= rect[4 * s + 2]; tx++) {
                if (!tile_kept(s, tx, ty, rect, mask, mean2d, conic, opac, view_W[v], view_H[v])) continue;
                pairs[k].tile = (uint32_t)(view_tile_off[v] + ty * view_tiles_x[v] + tx);
                pairs[k].key = depth_key[s];
                pairs[k].slot = (uint32_t)s;
                k++;
            }
    }
    free(cnt);
    qsort(pairs, (size_t)P, sizeof(opair_t), pair_cmp);
    for (int64_t t = 0; t < n_tiles_total; t++) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t i = 0; i < P; i++) {
        pair_tile[i] = pairs[i].tile;
        pair_slot[i] = pairs[i].slot;
        if (i == 0 || pairs[i].tile != pairs[i - 1].tile) ranges[2 * pairs[i].tile] = (uint32_t)i;
        if (i == P - 1 || pairs[i].tile != pairs[i + 1].tile) ranges[2 * pairs[i].tile + 1] = (uint32_t)(i + 1);
    }
    free(pairs);
    return P;
}

/* ------------------------------------------------------------------------ */
/* compositing (Eq. 2) per pixel, front to back                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *mean2d, *conic, *opac, *rgb, *depth;   /* per slot */
} o2d_t;

/* guard-band flags per pixel */
#define ORC_GUARD_SKIP 1     /* an evaluated alpha lies near 1/255 */
#define ORC_GUARD_STOP 2     /* an evaluated T(1-alpha) lies near 1e-4 */
#define ORC_GUARD_CLAMP 4    /* an evaluated o'G' lies near 0.99 */

typedef struct {
    int pos;                 /* 0-based position in the tile list */
    int slot;
    double dx, dy, G, alpha, T;
    int clamped;
} oentry_t;

/* Composites one pixel; returns the number of composited entries and fills
 * `ent` (if non-NULL, capacity `cap`) with them in front-to-back order. */
/* Guard band.  guard_eps (nullable) = {e_0, e_T, e_clamp, e_mean, e_quad}
 * bounds how far a compared float32 evaluation of the blend can stray from
 * this FP64 one (each float32 operation rounds within its unit roundoff u):
 *   - alpha = o' exp(power) carries relative error at most
 *       e_0 + e_quad (|A dx^2 / 2| + |B dx dy| + |C dy^2 / 2|)
 *           + e_mean (|d power / d dx| (2 |dx| + 17) + |d power / d dy| (2 |dy| + 17)):
 *     e_0 for exp, o' and its product and the float32 threshold constants;
 *     e_quad for the float32 conic coefficients and the products and sums of
 *     the three-term exponent (relative to the terms' magnitudes, which
 *     exceed |power| when the terms cancel); e_mean for a mean held relative
 *     to its 16x16 tile's origin (at most |dx| + 16 from it) and the
 *     difference dx, each rounded at its own magnitude;
 *   - the factor 1 - alpha carries the relative error of alpha times
 *     alpha / (1 - alpha), or e_clamp when alpha is the (float32) clamp
 *     0.99; each step adds e_T for rounding 1 - alpha and the product, and
 *     the stop test allows one more e_T for the float32 value of 1e-4.
 * A pixel is flagged when a skip (alpha vs 1/255), clamp (o' G' vs 0.99)
 * or stop (T (1 - alpha) vs 1e-4) decision lies within that error. */
/* The flagged decisions of one pixel (list position and kind), and the
 * ones a caller asks to be taken the other way: a decision within the guard
 * band can go either way in a float32 evaluation, so each way gives a valid
 * result (orc_render_alternatives). */
typedef struct { int pos, kind; } oflag_t;

typedef struct {
    const oflag_t *flip;
    int n_flip;
    oflag_t *seen;           /* flagged decisions met, in list order */
    int cap_seen, n_seen;
} odecide_t;

static int decision_flipped(const odecide_t *d, int pos, int kind) {
    if (!d) return 0;
    for (int i = 0; i < d->n_flip; i++)
        if (d->flip[i].pos == pos && d->flip[i].kind == kind) return 1;
    return 0;
}

static void decision_seen(odecide_t *d, int pos, int kind) {
    if (!d) return;
    if (d->n_seen < d->cap_seen) { d->seen[d->n_seen].pos = pos; d->seen[d->n_seen].kind = kind; }
    d->n_seen++;
}

static int composite_pixel(const o2d_t *g, const uint32_t *pair_slot, uint32_t start, uint32_t end,
                           double px, double py, const double *guard_eps, double out[7],
                           int *last_out, int *guard_out, oentry_t *ent, int cap, odecide_t *dec) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, D = 0.0;
    double errT = 0.0;     /* relative error bound of T so far */
    int last = 0, guard = 0, n = 0;
    for (uint32_t k = start; k < end; k++) {
        int s = (int)pair_slot[k], pos = (int)(k - start);
        const double *m = g->mean2d + 2 * s, *cn = g->conic + 3 * s;
        double dx, dy;
        double power = entry_power(m, cn, px, py, &dx, &dy);
        if (power > 0.0 && !guard_eps) continue;     /* skipped, nothing to flag */
        double G = exp(power);
        double raw = g->opac[s] * G;
        int clamp = raw >= ORC_ALPHA_MAX;
        double ea = 0.0;   /* relative error bound of alpha */
        if (guard_eps) {
            double quad = fabs(0.5 * cn[0] * dx * dx) + fabs(cn[1] * dx * dy) + fabs(0.5 * cn[2] * dy * dy);
            double gx = fabs(cn[0] * dx + cn[1] * dy), gy = fabs(cn[1] * dx + cn[2] * dy);
            ea = guard_eps[0] + guard_eps[4] * quad +
                 (gx * (2.0 * fabs(dx) + 17.0) + gy * (2.0 * fabs(dy) + 17.0)) * guard_eps[3];
            if (fabs(raw - ORC_ALPHA_MAX) <= ea * ORC_ALPHA_MAX) {
                guard |= ORC_GUARD_CLAMP;
                decision_seen(dec, pos, ORC_GUARD_CLAMP);
                if (decision_flipped(dec, pos, ORC_GUARD_CLAMP)) clamp = !clamp;
            }
        }
        double alpha = clamp ? ORC_ALPHA_MAX : raw;
        /* skipped: a positive exponent, or alpha below 1/255 */
        int skip = power > 0.0 || alpha < ORC_ALPHA_MIN;
        if (guard_eps && (power >= -ea || fabs(alpha - ORC_ALPHA_MIN) <= ea * ORC_ALPHA_MIN)) {
            guard |= ORC_GUARD_SKIP;
            decision_seen(dec, pos, ORC_GUARD_SKIP);
            if (decision_flipped(dec, pos, ORC_GUARD_SKIP)) skip = !skip;
        }
        if (skip) continue;
        double Tn = T * (1.0 - alpha);
        int stop = Tn < ORC_T_MIN;
        if (guard_eps) {
            double e1 = clamp ? guard_eps[2] : ea * alpha / (1.0 - alpha);
            double eTn = errT + e1 + guard_eps[1];
            if (fabs(Tn - ORC_T_MIN) <= (eTn + guard_eps[1]) * ORC_T_MIN) {
                guard |= ORC_GUARD_STOP;
                decision_seen(dec, pos, ORC_GUARD_STOP);
                if (decision_flipped(dec, pos, ORC_GUARD_STOP)) stop = !stop;
            }
            errT = eTn;
        }
        if (stop) break;
        if (ent && n < cap) {
            ent[n].pos = pos;
            ent[n].slot = s;
            ent[n].dx = dx; ent[n].dy = dy; ent[n].G = G; ent[n].alpha = alpha; ent[n].T = T;
            ent[n].clamped = clamp;
        }
        n++;
        for (int ch = 0; ch < 3; ch++) C[ch] += g->rgb[3 * s + ch] * alpha * T;
        D += g->depth[s] * alpha * T;
        T = Tn;
        last = pos + 1;
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = D; out[4] = 1.0 - T; out[5] = T;
    *last_out = last;
    *guard_out = guard;
    return n;
}

/* Renders one view.  Pixels are addressed [y][x]; tiles of this view are
 * numbered tile_off + ty * TW + tx in `ranges`.  tile_mask (nullable) limits
 * the work to the tiles whose mask byte is non-zero. */
int orc_render(const ocam_t *cam, const oopt_t *opt, int64_t tile_off, const double *mean2d,
               const double *conic, const double *opac, const double *rgb, const double *depth,
               const uint32_t *pair_slot, const uint32_t *ranges, const uint8_t *tile_mask,
               const double *guard_eps, double *out_rgb, double *out_depth, double *out_alpha,
               double *out_T, int32_t *out_last, uint8_t *out_guard) {
    o2d_t g = {mean2d, conic, opac, rgb, depth};
    int TW = (cam->W + ORC_TILE - 1) / ORC_TILE, TH = (cam->H + ORC_TILE - 1) / ORC_TILE;
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < TW * TH; t++) {
        if (tile_mask && !tile_mask[t]) continue;
        int tx = t % TW, ty = t / TW;
        uint32_t start = ranges[2 * (tile_off + t)], end = ranges[2 * (tile_off + t) + 1];
        for (int y = ty * ORC_TILE; y < (ty + 1) * ORC_TILE && y < cam->H; y++)
            for (int x = tx * ORC_TILE; x < (tx + 1) * ORC_TILE && x < cam->W; x++) {
                double o[7];
                int last, guard;
                composite_pixel(&g, pair_slot, start, end, x + 0.5, y + 0.5, guard_eps, o, &last, &guard, NULL, 0,
                                NULL);
                int64_t p = (int64_t)y * cam->W + x;
                for (int ch = 0; ch < 3; ch++) out_rgb[3 * p + ch] = o[ch] + o[5] * opt->bg[ch];
                out_depth[p] = o[3];
                out_alpha[p] = o[4];
                out_T[p] = o[5];
                out_last[p] = last;
                if (out_guard) out_guard[p] = (uint8_t)guard;
            }
    }
    return 0;
}

static int flag_in(const oflag_t *f, int n, oflag_t x) {
    for (int i = 0; i < n; i++)
        if (f[i].pos == x.pos && f[i].kind == x.kind) return 1;
    return 0;
}

/* For each listed pixel (index y * W + x) of one view: the outputs
 * (rgb + T bg, depth, alpha) of the blend under every combination of its
 * flagged decisions taken either way.  The set of decisions is closed: a
 * combination that meets a further flagged decision adds it, and the
 * enumeration restarts.  n_alt[i] = 2^m for m <= max_flags flagged
 * decisions (out[i] holds that many alternatives of 5 values, the first
 * one with no decision flipped), or -m when there are more. */
int orc_render_alternatives(const ocam_t *cam, const oopt_t *opt, int64_t tile_off, const double *mean2d,
                            const double *conic, const double *opac, const double *rgb, const double *depth,
                            const uint32_t *pair_slot, const uint32_t *ranges, const double *guard_eps,
                            int64_t n_px, const int64_t *pix, int max_flags, double *out, int32_t *n_alt) {
    o2d_t g = {mean2d, conic, opac, rgb, depth};
    int TW = (cam->W + ORC_TILE - 1) / ORC_TILE;
    int n_max = 1 << max_flags;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_px; i++) {
        int x = (int)(pix[i] % cam->W), y = (int)(pix[i] / cam->W);
        int t = (y / ORC_TILE) * TW + x / ORC_TILE;
        uint32_t start = ranges[2 * (tile_off + t)], end = ranges[2 * (tile_off + t) + 1];
        oflag_t F[32], seen[64], flip[32];
        int m = 0, closed = 0;
        /* the decisions flagged on the plain path */
        {
            odecide_t d = {NULL, 0, seen, 64, 0};
            double o[7];
            int last, guard;
            composite_pixel(&g, pair_slot, start, end, x + 0.5, y + 0.5, guard_eps, o, &last, &guard, NULL, 0, &d);
            for (int k = 0; k < d.n_seen && k < 64 && m < 32; k++)
                if (!flag_in(F, m, seen[k])) F[m++] = seen[k];
            if (d.n_seen > 64) m = 32;
        }
        while (!closed && m <= max_flags) {
            closed = 1;
            for (int mask = 0; mask < (1 << m) && closed; mask++) {
                int nf = 0;
                for (int b = 0; b < m; b++)
                    if (mask >> b & 1) flip[nf++] = F[b];
                odecide_t d = {flip, nf, seen, 64, 0};
                double o[7];
                int last, guard;
                composite_pixel(&g, pair_slot, start, end, x + 0.5, y + 0.5, guard_eps, o, &last, &guard, NULL, 0, &d);
                if (d.n_seen > 64) { m = 32; closed = 0; break; }
                for (int k = 0; k < d.n_seen; k++)
                    if (!flag_in(F, m, seen[k])) {
                        if (m < 32) F[m] = seen[k];
                        m++;
                        closed = 0;
                    }
                if (closed) {
                    double *r = out + ((int64_t)i * n_max + mask) * 5;
                    for (int ch = 0; ch < 3; ch++) r[ch] = o[ch] + o[5] * opt->bg[ch];
                    r[3] = o[3];
                    r[4] = o[4];
                }
            }
        }
        n_alt[i] = m <= max_flags ? (1 << m) : -m;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* backward of the compositing: per-slot gradients of the 2D quantities      */
/* ------------------------------------------------------------------------ */

/* d2 layout per slot (10 doubles): d mean2d (x, y), d conic (A, B, C),
 * d o', d rgb (3), d depth.  absg per slot (2): sum over pixels of
 * |d mean2d x| and |d mean2d y| (the homodirectional accumulation of AbsGS). */
static void atomic_add(double *p, double v) {
#pragma omp atomic
    *p += v;
}

int orc_render_bwd(const ocam_t *cam, const oopt_t *opt, int64_t tile_off, const double *mean2d,
                   const double *conic, const double *opac, const double *rgb, const double *depth,
                   const uint32_t *pair_slot, const uint32_t *ranges, const uint8_t *tile_mask,
                   const double *g_rgb, const double *g_depth, const double *g_alpha, double *d2,
                   double *absg) {
    o2d_t g = {mean2d, conic, opac, rgb, depth};
    int TW = (cam->W + ORC_TILE - 1) / ORC_TILE, TH = (cam->H + ORC_TILE - 1) / ORC_TILE;
#pragma omp parallel
    {
        int cap = 4096;
        oentry_t *ent = (oentry_t *)malloc(sizeof(oentry_t) * cap);
        double *suf = (double *)malloc(sizeof(double) * 4 * (cap + 1));
#pragma omp for schedule(dynamic, 4)
        for (int t = 0; t < TW * TH; t++) {
            if (tile_mask && !tile_mask[t]) continue;
            int tx = t % TW, ty = t / TW;
            uint32_t start = ranges[2 * (tile_off + t)], end = ranges[2 * (tile_off + t) + 1];
            if (end - start > (uint32_t)cap) {
                cap = (int)(end - start);
                ent = (oentry_t *)realloc(ent, sizeof(oentry_t) * cap);
                suf = (double *)realloc(suf, sizeof(double) * 4 * (cap + 1));
            }
            for (int y = ty * ORC_TILE; y < (ty + 1) * ORC_TILE && y < cam->H; y++)
                for (int x = tx * ORC_TILE; x < (tx + 1) * ORC_TILE && x < cam->W; x++) {
                    double o[7];
                    int last, guard;
                    int n = composite_pixel(&g, pair_slot, start, end, x + 0.5, y + 0.5, NULL, o, &last, &guard,
                                            ent, cap, NULL);
                    double Tf = o[5];
                    int64_t p = (int64_t)y * cam->W + x;
                    const double *gc = g_rgb + 3 * p;
                    double gd = g_depth[p], ga = g_alpha[p];
                    /* suffix sums S_i = sum_{j > i} c_j alpha_j T_j (and z) */
                    for (int q = 0; q < 4; q++) suf[4 * n + q] = 0.0;
                    for (int i = n - 1; i >= 0; i--) {
                        int s = ent[i].slot;
                        double w = ent[i].alpha * ent[i].T;
                        for (int ch = 0; ch < 3; ch++) suf[4 * i + ch] = suf[4 * (i + 1) + ch] + rgb[3 * s + ch] * w;
                        suf[4 * i + 3] = suf[4 * (i + 1) + 3] + depth[s] * w;
                    }
                    for (int i = 0; i < n; i++) {
                        int s = ent[i].slot;
                        double al = ent[i].alpha, Ti = ent[i].T, w = al * Ti;
                        double one_m = 1.0 - al;
                        /* dC/dalpha_i = c_i T_i - (sum_{j>i} c_j w_j + T_final bg) / (1 - alpha_i) */
                        double dal = 0.0;
                        for (int ch = 0; ch < 3; ch++)
                            dal += gc[ch] * (rgb[3 * s + ch] * Ti - (suf[4 * (i + 1) + ch] + Tf * opt->bg[ch]) / one_m);
                        dal += gd * (depth[s] * Ti - suf[4 * (i + 1) + 3] / one_m);
                        dal += ga * (Tf / one_m);
                        double *out = d2 + 10 * s;
                        for (int ch = 0; ch < 3; ch++) atomic_add(&out[6 + ch], gc[ch] * w);
                        atomic_add(&out[9], gd * w);
                        if (ent[i].clamped) continue;
                        /* alpha = o' G, G = exp(power) */
                        double G = ent[i].G;
                        atomic_add(&out[5], dal * G);
                        double dpow = dal * opac[s] * G;
                        const double *cn = conic + 3 * s;
                        double dx = ent[i].dx, dy = ent[i].dy;
                        double dmx = dpow * (cn[0] * dx + cn[1] * dy);
                        double dmy = dpow * (cn[1] * dx + cn[2] * dy);
                        atomic_add(&out[0], dmx);
                        atomic_add(&out[1], dmy);
                        atomic_add(&out[2], -0.5 * dx * dx * dpow);
                        atomic_add(&out[3], -dx * dy * dpow);
                        atomic_add(&out[4], -0.5 * dy * dy * dpow);
                        if (absg) {
                            atomic_add(&absg[2 * s], fabs(dmx));
                            atomic_add(&absg[2 * s + 1], fabs(dmy));
                        }
                    }
                }
        }
        free(ent);
        free(suf);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* backward of the projection and colour: chain to the 3D parameters         */
/* ------------------------------------------------------------------------ */

/* Adds this view's parameter gradients to d_means[3][n], d_scales[3][n],
 * d_quats[4][n], d_opac[n], d_sh[16][3][n] and, when given, d_cbase[n][3]
 * (the colour constant); writes |d mean2d| per slot. */
int orc_project_bwd(int64_t n, const double *means, const double *scales, const double *quats, const double *opac,
                    const double *sh, const double *cbase, const ocam_t *cam, const oopt_t *opt, const double *d2,
                    double *d_means, double *d_scales, double *d_quats, double *d_opac, double *d_sh,
                    double *d_cbase, double *mean2d_norm) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double mu[3], s[3], q[4];
        load_params(n, i, means, scales, quats, mu, s, q);
        proj1_t P;
        project_one(cam, opt, mu, s, q, opac[i], sh + i, n, cbase ? cbase + 3 * i : NULL, &P);
        const double *g = d2 + 10 * i;
        mean2d_norm[i] = sqrt(g[0] * g[0] + g[1] * g[1]);
        if (!P.visible) continue;
        double dmu[3] = {0.0, 0.0, 0.0}, dt[3] = {0.0, 0.0, 0.0};

        /* colour: raw = sum_k sh_k Y_k(dhat) + cbase, clamped at 0 */
        int nb = (opt->sh_degree + 1) * (opt->sh_degree + 1);
        double graw[3];
        for (int ch = 0; ch < 3; ch++) graw[ch] = P.clamped[ch] ? 0.0 : g[6 + ch];
        if (d_cbase)
            for (int ch = 0; ch < 3; ch++) d_cbase[3 * i + ch] += graw[ch];
        for (int k = 0; k < nb; k++)
            for (int ch = 0; ch < 3; ch++) d_sh[(k * 3 + ch) * n + i] += graw[ch] * P.Y[k];
        double dY[16][3];
        sh_basis_grad(P.dhat[0], P.dhat[1], P.dhat[2], dY);
        double ddhat[3] = {0.0, 0.0, 0.0};
        for (int k = 1; k < nb; k++) {
            double gk = 0.0;
            for (int ch = 0; ch < 3; ch++) gk += graw[ch] * sh[(k * 3 + ch) * n + i];
            for (int a = 0; a < 3; a++) ddhat[a] += gk * dY[k][a];
        }
        double dd = ddhat[0] * P.dhat[0] + ddhat[1] * P.dhat[1] + ddhat[2] * P.dhat[2];
        for (int a = 0; a < 3; a++) dmu[a] += (ddhat[a] - P.dhat[a] * dd) / P.dnorm;

        /* mean2d = (fx tx/tz + cx, fy ty/tz + cy); depth = tz */
        double tz = P.t[2];
        dt[0] += g[0] * cam->fx / tz;
        dt[2] += -g[0] * cam->fx * P.t[0] / (tz * tz);
        dt[1] += g[1] * cam->fy / tz;
        dt[2] += -g[1] * cam->fy * P.t[1] / (tz * tz);
        dt[2] += g[9];

        /* conic = inverse of the dilated covariance [[ad, b], [b, cd]] */
        double A = P.conic[0], B = P.conic[1], C = P.conic[2];
        double dA = g[2], dB = g[3], dC = g[4];
        double ga = dA * (-A * A) + dB * (-A * B) + dC * (-B * B);
        double gb = dA * (-2.0 * A * B) + dB * (-(A * C + B * B)) + dC * (-2.0 * B * C);
        double gcc = dA * (-B * B) + dB * (-B * C) + dC * (-C * C);

        /* o' = o rho, rho = sqrt(det2 / detd) */
        d_opac[i] += g[5] * P.rho;
        if (opt->aa && P.rho > 0.0) {
            double drho = g[5] * opac[i];
            double dd2 = P.detd * P.detd;
            double r_a = (P.c * P.detd - P.det2 * P.cd) / dd2;
            double r_c = (P.a * P.detd - P.det2 * P.ad) / dd2;
            double r_b = (-2.0 * P.b * P.detd + 2.0 * P.b * P.det2) / dd2;
            double k = drho / (2.0 * P.rho);
            ga += k * r_a;
            gb += k * r_b;
            gcc += k * r_c;
        }

        /* Sigma_2D = Tm Sigma Tm^T, Tm = J W */
        double G2[2][2] = {{ga, 0.5 * gb}, {0.5 * gb, gcc}};
        double dSigma[3][3], dTm[2][3];
        for (int a = 0; a < 3; a++)
            for (int b2 = 0; b2 < 3; b2++) {
                double acc = 0.0;
                for (int k = 0; k < 2; k++)
                    for (int l = 0; l < 2; l++) acc += P.Tm[k][a] * G2[k][l] * P.Tm[l][b2];
                dSigma[a][b2] = acc;
            }
        for (int a = 0; a < 2; a++)
            for (int b2 = 0; b2 < 3; b2++) {
                double acc = 0.0;
                for (int k = 0; k < 2; k++)
                    for (int l = 0; l < 3; l++) acc += G2[a][k] * P.Tm[k][l] * P.Sigma[l][b2];
                dTm[a][b2] = 2.0 * acc;
            }
        double dJ[2][3];
        for (int a = 0; a < 2; a++)
            for (int b2 = 0; b2 < 3; b2++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++) acc += dTm[a][k] * cam->R[b2][k];
                dJ[a][b2] = acc;
            }
        /* J = [[fx/tz, 0, -fx uc/tz], [0, fy/tz, -fy vc/tz]], uc = tx/tz unless clamped */
        dt[2] += dJ[0][0] * (-cam->fx / (tz * tz));
        dt[2] += dJ[1][1] * (-cam->fy / (tz * tz));
        if (!P.u_clamped) {
            dt[0] += dJ[0][2] * (-cam->fx / (tz * tz));
            dt[2] += dJ[0][2] * (2.0 * cam->fx * P.t[0] / (tz * tz * tz));
        } else {
            dt[2] += dJ[0][2] * (cam->fx * P.uc / (tz * tz));
        }
        if (!P.v_clamped) {
            dt[1] += dJ[1][2] * (-cam->fy / (tz * tz));
            dt[2] += dJ[1][2] * (2.0 * cam->fy * P.t[1] / (tz * tz * tz));
        } else {
            dt[2] += dJ[1][2] * (cam->fy * P.vc / (tz * tz));
        }
        /* t = W mu + t_w */
        for (int a = 0; a < 3; a++) dmu[a] += cam->R[0][a] * dt[0] + cam->R[1][a] * dt[1] + cam->R[2][a] * dt[2];
        for (int a = 0; a < 3; a++) d_means[a * n + i] += dmu[a];

        /* Sigma = M M^T, M = Rq diag(s) */
        double M[3][3], dM[3][3];
        for (int a = 0; a < 3; a++)
            for (int b2 = 0; b2 < 3; b2++) M[a][b2] = P.Rq[a][b2] * s[b2];
        for (int a = 0; a < 3; a++)
            for (int b2 = 0; b2 < 3; b2++) {
                double acc = 0.0;
                for (int k = 0; k < 3; k++) acc += (dSigma[a][k] + dSigma[k][a]) * M[k][b2];
                dM[a][b2] = acc;
            }
        double dR[3][3];
        for (int b2 = 0; b2 < 3; b2++) {
            double acc = 0.0;
            for (int a = 0; a < 3; a++) { acc += dM[a][b2] * P.Rq[a][b2]; dR[a][b2] = dM[a][b2] * s[b2]; }
            d_scales[b2 * n + i] += acc;
        }
        /* rotation of the unit quaternion (w, x, y, z): partial derivatives */
        double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
        double dqn[4];
        dqn[0] = 2.0 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
        dqn[1] = 2.0 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0 * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                        w * dR[2][1] - 2.0 * x * dR[2][2]);
        dqn[2] = 2.0 * (-2.0 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                        z * dR[2][1] - 2.0 * y * dR[2][2]);
        dqn[3] = 2.0 * (-2.0 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0 * z * dR[1][1] +
                        y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
        /* q_hat = q / |q| */
        double dot = dqn[0] * P.qn[0] + dqn[1] * P.qn[1] + dqn[2] * P.qn[2] + dqn[3] * P.qn[3];
        for (int a = 0; a < 4; a++) d_quats[a * n + i] += (dqn[a] - P.qn[a] * dot) / P.qnorm;
    }
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
