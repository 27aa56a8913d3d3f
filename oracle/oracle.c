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
    int32_t tile_cull;       /* 1: tile rectangle narrowed to the alpha box; 2: and, for rectangles
                                of at most 64 tiles, only tiles the alpha ellipse reaches (project_one) */
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
    uint64_t *mask;          /* [n] covered tiles of the rectangle, bit (ty - y0) w + (tx - x0);
                                0 = every tile of the rectangle (nullable) */
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
    uint64_t mask;
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
    if (opt->tile_cull) {
        /* Tile-based culling (adopted in §3.4.2 to skip Gaussians of negligible
         * contribution in a tile).  A pixel centre can pass the skip rule only
         * where o' G' >= 1/255, i.e. inside the ellipse d^T Sigma'^-1 d <= 2 tau,
         * tau = ln(255 o'), whose bounding box has half-widths
         * sqrt(2 tau Sigma'_xx) and sqrt(2 tau Sigma'_yy).  The box is widened
         * by margins for the float32 arithmetic of the compositing kernels
         * (1e-5 on tau, relative 1e-6 and 1e-3 px on the half-widths) and the
         * rectangle keeps only tiles holding pixel centres inside it, so no
         * image changes.  With o' below 1/255 (compared in float32) nothing
         * passes anywhere and the Gaussian is culled. */
        if (!((float)P->opac >= 1.0f / 255.0f)) return;
        double tau = log(255.0 * P->opac) + 1e-5;
        double hx = sqrt(2.0 * tau * P->ad) * (1.0 + 1e-6) + 1e-3;
        double hy = sqrt(2.0 * tau * P->cd) * (1.0 + 1e-6) + 1e-3;
        /* pixels p with |p + 0.5 - m| <= h, then their tiles */
        double bx0 = floor(ceil(P->mean2d[0] - hx - 0.5) / ORC_TILE), bx1 = floor(floor(P->mean2d[0] + hx - 0.5) / ORC_TILE);
        double by0 = floor(ceil(P->mean2d[1] - hy - 0.5) / ORC_TILE), by1 = floor(floor(P->mean2d[1] + hy - 0.5) / ORC_TILE);
        if (bx0 > fx0) fx0 = bx0;
        if (by0 > fy0) fy0 = by0;
        if (bx1 < fx1) fx1 = bx1;
        if (by1 < fy1) fy1 = by1;
    }
    if (!(fx0 <= fx1 && fy0 <= fy1)) return;
    P->radius = (int)(r < 2e9 ? r : 2e9);
    P->rect[0] = (int)fx0; P->rect[1] = (int)fy0; P->rect[2] = (int)fx1; P->rect[3] = (int)fy1;
    P->tiles = (P->rect[2] - P->rect[0] + 1) * (P->rect[3] - P->rect[1] + 1);
    P->mask = 0;
    if (opt->tile_cull >= 2 && P->tiles <= 64) {
        /* Exact tile culling: keep a tile only if the alpha ellipse
         * q(d) = d^T Sigma'^-1 d <= L, L = 2 tau (1 + 4e-6) (tau as for the
         * box), reaches the rectangle of its pixel centres (widened by
         * 1e-3 px).  Row by row: the ellipse within a row's strip
         * [ylo, yhi] is convex, so it meets a tile of the row iff its
         * x-extent over the strip meets the tile's column range.  For fixed
         * y the ellipse spans x = (-B y -+ sqrt(A L - det y^2)) / A; the upper
         * end is concave in y with its maximum at the ellipse's rightmost
         * point (X, -B X / C), X = sqrt(L C / det), and the lower end convex
         * with its minimum at (-X, B X / C): over the strip (clipped to the
         * ellipse's y-extent +-sqrt(L A / det)) both are taken at those y
         * clamped into the strip. */
        double tau = log(255.0 * P->opac) + 1e-5;
        double L = 2.0 * tau * (1.0 + 4e-6);
        double A = P->conic[0], B = P->conic[1], C = P->conic[2];
        double det = A * C - B * B;
        double X = sqrt(L * C / det), Y = sqrt(L * A / det), yr = -B / C * X;
        int w = P->rect[2] - P->rect[0] + 1, cnt = 0;
        for (int ty = P->rect[1]; ty <= P->rect[3]; ty++) {
            int py1 = ty * ORC_TILE + ORC_TILE - 1;
            if (py1 > cam->H - 1) py1 = cam->H - 1;
            double ylo = ty * ORC_TILE + 0.5 - 1e-3 - P->mean2d[1], yhi = py1 + 0.5 + 1e-3 - P->mean2d[1];
            double a = ylo > -Y ? ylo : -Y, b = yhi < Y ? yhi : Y;
            if (a > b) continue;
            double y1 = yr < a ? a : (yr > b ? b : yr);
            double y2 = -yr < a ? a : (-yr > b ? b : -yr);
            double r1 = A * L - det * y1 * y1, r2 = A * L - det * y2 * y2;
            double xhi_e = (-B * y1 + sqrt(r1 > 0.0 ? r1 : 0.0)) / A;
            double xlo_e = (-B * y2 - sqrt(r2 > 0.0 ? r2 : 0.0)) / A;
            for (int tx = P->rect[0]; tx <= P->rect[2]; tx++) {
                int px1 = tx * ORC_TILE + ORC_TILE - 1;
                if (px1 > cam->W - 1) px1 = cam->W - 1;
                double xlo = tx * ORC_TILE + 0.5 - 1e-3 - P->mean2d[0], xhi = px1 + 0.5 + 1e-3 - P->mean2d[0];
                if (xlo <= xhi_e && xhi >= xlo_e) {
                    P->mask |= 1ull << ((ty - P->rect[1]) * w + (tx - P->rect[0]));
                    cnt++;
                }
            }
        }
        if (cnt == 0) return;
        P->tiles = cnt;
    }

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
        if (out->mask) out->mask[i] = P.visible ? P.mask : 0;
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

/* Enumerates one pair per (slot, covered tile: a tile of the slot's
 * rectangle whose bit is set in mask[s], every tile when mask is NULL or
 * mask[s] is 0), sorts the
 * pairs by (global tile id, depth key, slot) -- "processed in depth order"
 * of §3.1, ties by input index -- and writes [start, end) per global tile.
 * slot_view[s] selects the view of a slot; its tiles are numbered
 * view_tile_off[v] + ty * view_tiles_x[v] + tx. */
int64_t orc_bin(int64_t n_slots, const int32_t *rect, const int32_t *tiles, const uint64_t *mask,
                const uint32_t *depth_key, const int32_t *slot_view, const int32_t *view_tiles_x,
                const int32_t *view_tile_off, int64_t n_tiles_total, int64_t capacity, uint32_t *pair_tile,
                uint32_t *pair_slot, uint32_t *ranges /* [n_tiles_total][2] */) {
    int64_t P = 0;
    for (int64_t s = 0; s < n_slots; s++) P += tiles[s];
    if (P > capacity) return -P;
    opair_t *pairs = (opair_t *)malloc(sizeof(opair_t) * (size_t)(P > 0 ? P : 1));
    if (!pairs) return -1;
    int64_t k = 0;
    for (int64_t s = 0; s < n_slots; s++) {
        if (tiles[s] <= 0) continue;
        int v = slot_view[s];
        uint64_t m = mask ? mask[s] : 0;
        int w = rect[4 * s + 2] - rect[4 * s] + 1;
        for (int ty = rect[4 * s + 1]; ty <= rect[4 * s + 3]; ty++)
            for (int tx = rect[4 * s]; tx <= rect[4 * s + 2]; tx++) {
                if (m && !((m >> ((ty - rect[4 * s + 1]) * w + (tx - rect[4 * s]))) & 1)) continue;
                pairs[k].tile = (uint32_t)(view_tile_off[v] + ty * view_tiles_x[v] + tx);
                pairs[k].key = depth_key[s];
                pairs[k].slot = (uint32_t)s;
                k++;
            }
    }
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
/* Guard band.  guard_eps (nullable) = {e_alpha, e_T, e_clamp, e_mean}: a
 * compared implementation evaluates alpha with relative error at most
 * e_alpha + |d power / d mean| * (|dx| + 17) * e_mean (e_mean models a mean
 * held relative to its 16x16 tile's origin with that relative rounding; the
 * tile-relative mean is at most |dx| + 16 from the origin), and T with the
 * accumulated relative error of the alphas before it plus e_T.  A pixel is
 * flagged when a skip (alpha vs 1/255), stop (T(1 - alpha) vs 1e-4) or clamp
 * (o' G' vs 0.99) decision lies inside that error. */
static int composite_pixel(const o2d_t *g, const uint32_t *pair_slot, uint32_t start, uint32_t end,
                           double px, double py, const double *guard_eps, double out[7],
                           int *last_out, int *guard_out, oentry_t *ent, int cap) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0}, D = 0.0;
    double errT = 0.0;     /* relative error bound of T so far */
    int last = 0, guard = 0, n = 0;
    for (uint32_t k = start; k < end; k++) {
        int s = (int)pair_slot[k];
        const double *m = g->mean2d + 2 * s, *cn = g->conic + 3 * s;
        double dx = px - m[0], dy = py - m[1];
        double power = -0.5 * (cn[0] * dx * dx + cn[2] * dy * dy) - cn[1] * dx * dy;
        if (power > 0.0) continue;
        double G = exp(power);
        double raw = g->opac[s] * G;
        double alpha = raw < ORC_ALPHA_MAX ? raw : ORC_ALPHA_MAX;
        double ea = 0.0;   /* relative error bound of alpha */
        if (guard_eps) {
            double gx = fabs(cn[0] * dx + cn[1] * dy), gy = fabs(cn[1] * dx + cn[2] * dy);
            ea = guard_eps[0] + (gx * (fabs(dx) + 17.0) + gy * (fabs(dy) + 17.0)) * guard_eps[3];
            if (fabs(alpha - ORC_ALPHA_MIN) <= ea * ORC_ALPHA_MIN) guard |= ORC_GUARD_SKIP;
            if (fabs(raw - ORC_ALPHA_MAX) <= (ea + guard_eps[2]) * ORC_ALPHA_MAX) guard |= ORC_GUARD_CLAMP;
        }
        if (alpha < ORC_ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        if (guard_eps) {
            double eTn = errT + ea * alpha / (1.0 - alpha) + guard_eps[1];
            if (fabs(Tn - ORC_T_MIN) <= eTn * ORC_T_MIN) guard |= ORC_GUARD_STOP;
            errT = eTn;
        }
        if (Tn < ORC_T_MIN) break;
        if (ent && n < cap) {
            ent[n].pos = (int)(k - start);
            ent[n].slot = s;
            ent[n].dx = dx; ent[n].dy = dy; ent[n].G = G; ent[n].alpha = alpha; ent[n].T = T;
            ent[n].clamped = raw >= ORC_ALPHA_MAX;
        }
        n++;
        for (int ch = 0; ch < 3; ch++) C[ch] += g->rgb[3 * s + ch] * alpha * T;
        D += g->depth[s] * alpha * T;
        T = Tn;
        last = (int)(k - start) + 1;
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
                composite_pixel(&g, pair_slot, start, end, x + 0.5, y + 0.5, guard_eps, o, &last, &guard, NULL, 0);
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
                                            ent, cap);
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
