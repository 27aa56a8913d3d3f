// Backward of projection and colour -- gfx950.
//
// A workgroup owns a span of 1024 consecutive Gaussians.  It first finds
// which of them some view sees (tiles > 0), writes the per-view statistics
// and the zero colour-coefficient rows of the others with coalesced stores,
// and packs the seen ones into an LDS list; then one thread per listed
// Gaussian reads its parameters once, recomputes the projection in FP64 for
// each view that sees it, chains that view's 2D gradients (mean2d, conic,
// opacity', colour, depth) back to the parameters, and writes the sums once:
// the coefficient rows directly, the one-float-per-Gaussian rows (means,
// scales, quats, opacity, appearance) into LDS rows of the span that start
// at zero and are streamed out whole at the end, so every cache line of
// those arrays is written once and completely instead of in two partial
// halves (zeros, then the seen Gaussians' values).  When the outputs were
// zeroed beforehand (k_zero_floats on a second stream beside the
// compositing backward), the chain writes the seen Gaussians' entries
// directly and the unseen ones are left alone.  Only a small fraction of a
// large scene is in view, so the compaction keeps the FP64 chain on full
// waves and the parameter reads on the Gaussians that need them; 2D
// gradients of unseen slots are never read.  With
// Sigma_2D = V V^T and V = (J W) M, M = R(q) diag(s), the covariance
// gradient flows as dV = 2 G V, d(JW) = dV M^T, dM += (JW)^T dV; dM is
// accumulated over views and pushed through R(q) and s once at the end.
// HBM-bound; geometry in FP64 for the same reason as the forward.
//
// Paper: backward of Eq. 1 and of the projection of §3.1; the per-view
// |dL/d mean2d| is the image-space statistic that densification thresholds
// (§3.1, §3.3 Eq. 4), and the absolute accumulation is the AbsGS statistic
// of §3.5.4.
#include "gs_internal.h"

namespace gs {

namespace {

// gradient of each basis polynomial of sh_eval_basis with respect to (x, y, z)
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int k, float& gx, float& gy,
                                              float& gz) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float k1 = (float)ShK::k1, k2 = (float)ShK::k2, k6 = (float)ShK::k6, k8 = (float)ShK::k8,
                k9 = (float)ShK::k9, k10 = (float)ShK::k10, k11 = (float)ShK::k11, k12 = (float)ShK::k12,
                k14 = (float)ShK::k14;
    gx = gy = gz = 0.0f;
    switch (k) {
        case 1: gy = -k1; break;
        case 2: gz = k1; break;
        case 3: gx = -k1; break;
        case 4: gx = k2 * y; gy = k2 * x; break;
        case 5: gy = -k2 * z; gz = -k2 * y; break;
        case 6: gx = -2.0f * k6 * x; gy = -2.0f * k6 * y; gz = 4.0f * k6 * z; break;
        case 7: gx = -k2 * z; gz = -k2 * x; break;
        case 8: gx = 2.0f * k8 * x; gy = -2.0f * k8 * y; break;
        case 9: gx = -6.0f * k9 * x * y; gy = -3.0f * k9 * (xx - yy); break;
        case 10: gx = k10 * y * z; gy = k10 * x * z; gz = k10 * x * y; break;
        case 11: gx = 2.0f * k11 * x * y; gy = -k11 * (4.0f * zz - xx - 3.0f * yy); gz = -8.0f * k11 * y * z; break;
        case 12: gx = -6.0f * k12 * x * z; gy = -6.0f * k12 * y * z; gz = k12 * (6.0f * zz - 3.0f * xx - 3.0f * yy); break;
        case 13: gx = -k11 * (4.0f * zz - 3.0f * xx - yy); gy = 2.0f * k11 * x * y; gz = -8.0f * k11 * x * z; break;
        case 14: gx = 2.0f * k14 * x * z; gy = -2.0f * k14 * y * z; gz = k14 * (xx - yy); break;
        case 15: gx = -3.0f * k9 * (xx - yy); gy = 6.0f * k9 * x * y; break;
        default: break;
    }
}

typedef float F4 __attribute__((ext_vector_type(4)));

constexpr int kG2 = GS_GRAD2D_FLOATS;
constexpr int kPB = 256;                  // threads per workgroup
constexpr int kSpanPer = 4;               // Gaussians per thread in the scan
constexpr int kSpan = kPB * kSpanPer;     // Gaussians per workgroup

// gradient rows staged in LDS per workgroup span: means (3), scales (3),
// quats (4), opacity (1), appearance offsets (4)
constexpr int kStageRows = 15;
constexpr int kStageApp = 11;

// Destinations of a seen Gaussian's one-float gradients, by row c (means
// 0-2, scales 3-5, quats 6-9, opacity 10, appearance offsets 11-14): the
// span's LDS rows, or the output arrays themselves
struct StageRows {
    float* s;
    int loc;
    __device__ void put(int c, float v) const { s[c * kSpan + loc] = v; }
};
struct OutRows {
    const GradPtrs& out;
    int64_t n, g;
    __device__ void put(int c, float v) const {
        float* p = c < 3 ? out.means + c * n + g : c < 6 ? out.scales + (c - 3) * n + g
                 : c < 10 ? out.quats + (c - 6) * n + g : c == 10 ? out.opac + g : out.app + 4 * g + (c - kStageApp);
        __builtin_nontemporal_store(v, p);
    }
};

// full chain for one seen Gaussian g; vis = mask of the views that see it.
// Writes its SH coefficient gradients to out.sh and the other gradients to
// `rows`.
template <class Rows>
__device__ __forceinline__ void project_bwd_one(const GaussPtrs& gp, int64_t n, const ViewTable& vt,
                                                const OptK& opt, const float* __restrict__ grad2d,
                                                const GradPtrs& out, int64_t g, uint32_t vis, const Rows& rows) {
    const int nb = (opt.sh_degree + 1) * (opt.sh_degree + 1);
    const int nq = (3 * nb + 3) >> 2;    // float4s of a coefficient row in use
    const float4* shq = reinterpret_cast<const float4*>(gp.sh) + 12 * g;
    float4* dshq = reinterpret_cast<float4*>(out.sh) + 12 * g;
    const double mu0 = gp.means[g], mu1 = gp.means[n + g], mu2 = gp.means[2 * n + g];
    const double s0 = gp.scales[g], s1 = gp.scales[n + g], s2 = gp.scales[2 * n + g];
    const double q0 = gp.quats[g], q1 = gp.quats[n + g], q2 = gp.quats[2 * n + g], q3 = gp.quats[3 * n + g];
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    double M[9];   // R(q) diag(s)
    M[0] = (1.0 - 2.0 * (y * y + z * z)) * s0; M[1] = 2.0 * (x * y - w * z) * s1; M[2] = 2.0 * (x * z + w * y) * s2;
    M[3] = 2.0 * (x * y + w * z) * s0; M[4] = (1.0 - 2.0 * (x * x + z * z)) * s1; M[5] = 2.0 * (y * z - w * x) * s2;
    M[6] = 2.0 * (x * z - w * y) * s0; M[7] = 2.0 * (y * z + w * x) * s1; M[8] = (1.0 - 2.0 * (x * x + y * y)) * s2;
    // appearance offsets: colour constant dc (else 1/2), opacity o (1 - do)
    const float4 app = gp.app ? reinterpret_cast<const float4*>(gp.app)[g] : make_float4(0.5f, 0.5f, 0.5f, 0.0f);
    const double o_raw = gp.opac[g];
    const double o = o_raw * (gp.app ? 1.0 - (double)app.w : 1.0);
    float dcb0 = 0.0f, dcb1 = 0.0f, dcb2 = 0.0f;

    double dmu[3] = {0.0, 0.0, 0.0};
    double dM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double dop = 0.0;
    bool first = true;    // the first visible view writes d_sh, later ones add to it

    for (int v = 0; v < vt.n_views; ++v) {
        if (!(vis & (1u << v))) continue;
        const ViewK& V = vt.v[v];
        const int64_t slot = (int64_t)v * n + g;
        const float* g2 = grad2d + slot * kG2;
        const double gmx = g2[0], gmy = g2[1], gA = g2[2], gB = g2[3], gC = g2[4], gop = g2[5];
        const double gz = g2[9];
        float W[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) W[i] = V.R[i];
        const double tx = W[0] * mu0 + W[1] * mu1 + W[2] * mu2 + (double)V.t[0];
        const double ty = W[3] * mu0 + W[4] * mu1 + W[5] * mu2 + (double)V.t[1];
        const double tz = W[6] * mu0 + W[7] * mu1 + W[8] * mu2 + (double)V.t[2];
        const double fx = V.fx, fy = V.fy;

        // ---- colour: raw = sum_k sh_k Y_k(dhat) + dc, clamped at 0 (SH in FP32)
        {
            const double e0d = mu0 - V.campos[0], e1d = mu1 - V.campos[1], e2d = mu2 - V.campos[2];
            const double dn = sqrt(e0d * e0d + e1d * e1d + e2d * e2d);
            const double inv = 1.0 / dn;
            const float d0 = (float)(e0d * inv), d1 = (float)(e1d * inv), d2 = (float)(e2d * inv);
            float Y[16];
            sh_eval_basis<float>(d0, d1, d2, opt.sh_degree, Y);
            // one pass over the coefficient row gives the colour and, per
            // channel c, S_c = sum_k sh_kc grad Y_k, so that the direction
            // gradient is sum_c gr_c S_c and the row is not held in registers
            // (coefficient e of the row is channel e % 3 of basis e / 3)
            float raw[3] = {app.x, app.y, app.z};
            float S[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                if (q < nq) {
                    const float4 t = shq[q];
                    const float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = (4 * q + j) / 3, c = (4 * q + j) % 3;
                        if (k < nb) {
                            raw[c] = fmaf(tv[j], Y[k], raw[c]);
                            if (k > 0) {
                                float bx, by, bz;
                                sh_basis_grad(d0, d1, d2, k, bx, by, bz);
                                S[c][0] = fmaf(tv[j], bx, S[c][0]);
                                S[c][1] = fmaf(tv[j], by, S[c][1]);
                                S[c][2] = fmaf(tv[j], bz, S[c][2]);
                            }
                        }
                    }
                }
            }
            const float gr[3] = {raw[0] < 0.0f ? 0.0f : g2[6], raw[1] < 0.0f ? 0.0f : g2[7],
                                 raw[2] < 0.0f ? 0.0f : g2[8]};
            dcb0 += gr[0]; dcb1 += gr[1]; dcb2 += gr[2];
            const float e0 = gr[0] * S[0][0] + gr[1] * S[1][0] + gr[2] * S[2][0];
            const float e1 = gr[0] * S[0][1] + gr[1] * S[1][1] + gr[2] * S[2][1];
            const float e2 = gr[0] * S[0][2] + gr[1] * S[1][2] + gr[2] * S[2][2];
            // d sh_kc = gr_c Y_k, added to the earlier views' sums
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                float d[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = (4 * q + j) / 3, c = (4 * q + j) % 3;
                    d[j] = k < nb ? gr[c] * Y[k] : 0.0f;
                }
                float4 t = make_float4(d[0], d[1], d[2], d[3]);
                if (!first && q < nq) {
                    const float4 p = dshq[q];
                    t.x += p.x; t.y += p.y; t.z += p.z; t.w += p.w;
                }
                if (first || q < nq) dshq[q] = t;
            }
            first = false;
            const double dd = (double)e0 * d0 + (double)e1 * d1 + (double)e2 * d2;
            dmu[0] += ((double)e0 - d0 * dd) * inv;
            dmu[1] += ((double)e1 - d1 * dd) * inv;
            dmu[2] += ((double)e2 - d2 * dd) * inv;
        }

        // ---- geometry, recomputed as in the forward
        const double u = tx / tz, vv = ty / tz;
        const bool ucl = u < V.ulo || u > V.uhi, vcl = vv < V.vlo || vv > V.vhi;
        const double uc = fmin(fmax(u, V.ulo), V.uhi), vc = fmin(fmax(vv, V.vlo), V.vhi);
        const double j00 = fx / tz, j02 = -fx * uc / tz, j11 = fy / tz, j12 = -fy * vc / tz;
        double Tm[6];
        Tm[0] = j00 * W[0] + j02 * W[6]; Tm[1] = j00 * W[1] + j02 * W[7]; Tm[2] = j00 * W[2] + j02 * W[8];
        Tm[3] = j11 * W[3] + j12 * W[6]; Tm[4] = j11 * W[4] + j12 * W[7]; Tm[5] = j11 * W[5] + j12 * W[8];
        double Vm[6];   // Tm M; Sigma_2D = Vm Vm^T
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                Vm[3 * r + c] = Tm[3 * r] * M[c] + Tm[3 * r + 1] * M[3 + c] + Tm[3 * r + 2] * M[6 + c];
        const double ca = Vm[0] * Vm[0] + Vm[1] * Vm[1] + Vm[2] * Vm[2];
        const double cb = Vm[0] * Vm[3] + Vm[1] * Vm[4] + Vm[2] * Vm[5];
        const double cc = Vm[3] * Vm[3] + Vm[4] * Vm[4] + Vm[5] * Vm[5];
        const double x0 = Vm[1] * Vm[5] - Vm[2] * Vm[4], x1 = Vm[2] * Vm[3] - Vm[0] * Vm[5],
                     x2 = Vm[0] * Vm[4] - Vm[1] * Vm[3];
        const double det2 = x0 * x0 + x1 * x1 + x2 * x2;
        const double dil = (double)opt.dilation;
        const double ad = ca + dil, cd = cc + dil;
        const double detd = det2 + dil * (ca + cc) + dil * dil;
        const double invd = 1.0 / detd;
        const double A = cd * invd, B = -cb * invd, C = ad * invd;
        const double rho = opt.aa ? (det2 > 0.0 ? sqrt(det2 * invd) : 0.0) : 1.0;

        double dt0 = 0.0, dt1 = 0.0, dt2 = 0.0;
        // mean2d = (fx tx/tz + cx, fy ty/tz + cy), depth = tz
        dt0 += gmx * fx / tz;
        dt2 -= gmx * fx * tx / (tz * tz);
        dt1 += gmy * fy / tz;
        dt2 -= gmy * fy * ty / (tz * tz);
        dt2 += gz;
        // conic = inverse of [[ad, cb], [cb, cd]]
        double ga = gA * (-A * A) + gB * (-A * B) + gC * (-B * B);
        double gb = gA * (-2.0 * A * B) + gB * (-(A * C + B * B)) + gC * (-2.0 * B * C);
        double gc = gA * (-B * B) + gB * (-B * C) + gC * (-C * C);
        // opacity' = o rho, rho = sqrt(det2 / detd)
        dop += gop * rho;
        if (opt.aa && rho > 0.0) {
            const double k = gop * o / (2.0 * rho) * invd * invd;
            ga += k * (cc * detd - det2 * cd);
            gc += k * (ca * detd - det2 * ad);
            gb += k * (-2.0 * cb * detd + 2.0 * cb * det2);
        }
        // Sigma_2D = Vm Vm^T with the symmetric gradient G = [[ga, gb/2], [gb/2, gc]]
        const double G01 = 0.5 * gb;
        double dVm[6];
        for (int c = 0; c < 3; ++c) {
            dVm[c] = 2.0 * (ga * Vm[c] + G01 * Vm[3 + c]);
            dVm[3 + c] = 2.0 * (G01 * Vm[c] + gc * Vm[3 + c]);
        }
        // Vm = Tm M: dM += Tm^T dVm, dTm = dVm M^T
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) dM[3 * r + c] += Tm[r] * dVm[c] + Tm[3 + r] * dVm[3 + c];
        double dTm[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                dTm[3 * r + c] = dVm[3 * r] * M[3 * c] + dVm[3 * r + 1] * M[3 * c + 1] + dVm[3 * r + 2] * M[3 * c + 2];
        // dJ = dTm W^T; J has entries (0,0), (0,2), (1,1), (1,2)
        const double dJ00 = dTm[0] * W[0] + dTm[1] * W[1] + dTm[2] * W[2];
        const double dJ02 = dTm[0] * W[6] + dTm[1] * W[7] + dTm[2] * W[8];
        const double dJ11 = dTm[3] * W[3] + dTm[4] * W[4] + dTm[5] * W[5];
        const double dJ12 = dTm[3] * W[6] + dTm[4] * W[7] + dTm[5] * W[8];
        const double tz2 = tz * tz;
        dt2 += dJ00 * (-fx / tz2) + dJ11 * (-fy / tz2);
        if (!ucl) {
            dt0 += dJ02 * (-fx / tz2);
            dt2 += dJ02 * (2.0 * fx * tx / (tz2 * tz));
        } else {
            dt2 += dJ02 * (fx * uc / tz2);
        }
        if (!vcl) {
            dt1 += dJ12 * (-fy / tz2);
            dt2 += dJ12 * (2.0 * fy * ty / (tz2 * tz));
        } else {
            dt2 += dJ12 * (fy * vc / tz2);
        }
        // t = W mu + t_w
        dmu[0] += W[0] * dt0 + W[3] * dt1 + W[6] * dt2;
        dmu[1] += W[1] * dt0 + W[4] * dt1 + W[7] * dt2;
        dmu[2] += W[2] * dt0 + W[5] * dt1 + W[8] * dt2;
    }

    // M = R(q) diag(s): ds_c = sum_r dM[r][c] R[r][c], dR[r][c] = dM[r][c] s_c
    const double sc[3] = {s0, s1, s2};
    double dR[9], ds[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ds[c] += dM[3 * r + c] * M[3 * r + c] / sc[c];
            dR[3 * r + c] = dM[3 * r + c] * sc[c];
        }
    // rotation of the unit quaternion (w, x, y, z)
    double dq[4];
    dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.0 * x * dR[8]);
    dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
    dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
    // normalisation q / |q|
    const double dot = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    const double qh[4] = {w, x, y, z};
    for (int c = 0; c < 3; ++c) rows.put(c, (float)dmu[c]);
    for (int c = 0; c < 3; ++c) rows.put(3 + c, (float)ds[c]);
    for (int c = 0; c < 4; ++c) rows.put(6 + c, (float)((dq[c] - qh[c] * dot) / qn));
    // dop is the gradient with respect to o (1 - do)
    rows.put(10, (float)(gp.app ? dop * (1.0 - (double)app.w) : dop));
    if (out.app) {
        rows.put(kStageApp + 0, dcb0);
        rows.put(kStageApp + 1, dcb1);
        rows.put(kStageApp + 2, dcb2);
        rows.put(kStageApp + 3, (float)(-dop * o_raw));
    }
}


// kZeroed: the gradient outputs already hold zeros (gs_grads_zero, run
// beside the compositing backward), so only the entries of Gaussians some
// view sees are written, straight from the chain (scattered either way):
// no LDS rows, so more workgroups fit on a compute unit
template <bool kZeroed>
__global__ __launch_bounds__(kPB) void k_project_bwd(GaussPtrs gp, int64_t n, ViewTable vt, OptK opt,
                                                     Projected proj, const float* __restrict__ grad2d, GradPtrs out,
                                                     float* __restrict__ mean2d_norm, float* __restrict__ absgrad) {
    __shared__ uint32_t s_list[kSpan];     // local index | view mask << 16
    __shared__ uint32_t s_group[kSpan];    // the list grouped by view mask (several views)
    __shared__ uint32_t s_hist[256];
    __shared__ uint8_t s_seen[kSpan];
    __shared__ uint32_t s_count;
    // the span's gradient rows: zeros, then the chain's values, then one
    // coalesced write of every row (each cache line written once, whole)
    __shared__ float s_grad[kZeroed ? 1 : kStageRows * kSpan];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t g0 = (int64_t)blockIdx.x * kSpan;
    if (tid == 0) s_count = 0;
    __syncthreads();

    // pass 1: statistics, visibility, zeroed LDS rows, compaction
    for (int i = 0; i < kSpanPer; ++i) {
        const int loc = i * kPB + tid;
        const int64_t g = g0 + loc;
        uint32_t vis = 0;
        if (g < n) {
            for (int v = 0; v < vt.n_views; ++v) {
                const int64_t slot = (int64_t)v * n + g;
                const bool seen = proj.tiles[slot] != 0;
                float nrm = 0.0f, ax = 0.0f, ay = 0.0f;
                if (seen) {
                    const float* g2 = grad2d + slot * kG2;
                    const float dmx = g2[0], dmy = g2[1];
                    nrm = sqrtf(dmx * dmx + dmy * dmy);
                    ax = g2[10];
                    ay = g2[11];
                    vis |= 1u << v;
                }
                __builtin_nontemporal_store(nrm, mean2d_norm + slot);
                if (absgrad) {
                    __builtin_nontemporal_store(ax, absgrad + 2 * slot);
                    __builtin_nontemporal_store(ay, absgrad + 2 * slot + 1);
                }
            }
        }
        if (!kZeroed) {
#pragma unroll
            for (int c = 0; c < kStageRows; ++c) s_grad[c * kSpan + loc] = 0.0f;
        }
        s_seen[loc] = vis ? 1 : 0;
        const uint64_t m = __ballot(vis != 0);
        if (m) {
            const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_count, (uint32_t)__popcll(m));
            base = __shfl(base, 0);
            if (vis) s_list[base + below] = (uint32_t)loc | (vis << 16);
        }
    }
    __syncthreads();

    // zero coefficient rows of unseen Gaussians: coalesced 16-byte stores
    const int64_t rows = n - g0 < kSpan ? n - g0 : kSpan;
    F4* dsh = reinterpret_cast<F4*>(out.sh) + 12 * g0;
    if (!kZeroed)
        for (int q = tid; q < 12 * rows; q += kPB)
            if (!s_seen[q / 12]) __builtin_nontemporal_store(F4{0.0f, 0.0f, 0.0f, 0.0f}, dsh + q);

    // pass 2: the chain, one thread per seen Gaussian (with several views,
    // Gaussians seen by the same views side by side)
    const uint32_t cnt = s_count;
    const uint32_t* lst = s_list;
    if (vt.n_views > 1) {
        group_by_views(s_list, cnt, s_group, s_hist);
        lst = s_group;
    }
    for (uint32_t j = tid; j < cnt; j += kPB) {
        const uint32_t e = lst[j];
        const int64_t g = g0 + (e & 0xFFFFu);
        if (kZeroed)
            project_bwd_one(gp, n, vt, opt, grad2d, out, g, e >> 16, OutRows{out, n, g});
        else
            project_bwd_one(gp, n, vt, opt, grad2d, out, g, e >> 16, StageRows{s_grad, (int)(e & 0xFFFFu)});
    }
    if (kZeroed) return;
    __syncthreads();

    // pass 3: the span's rows, streamed out (not read again here)
    for (int c = 0; c < 11; ++c) {
        float* row = c < 3 ? out.means + c * n : c < 6 ? out.scales + (c - 3) * n
                   : c < 10 ? out.quats + (c - 6) * n : out.opac;
        for (int loc = tid; loc < rows; loc += kPB) __builtin_nontemporal_store(s_grad[c * kSpan + loc], row + g0 + loc);
    }
    if (out.app)
        for (int loc = tid; loc < rows; loc += kPB)
            __builtin_nontemporal_store(F4{s_grad[(kStageApp + 0) * kSpan + loc], s_grad[(kStageApp + 1) * kSpan + loc],
                                           s_grad[(kStageApp + 2) * kSpan + loc], s_grad[(kStageApp + 3) * kSpan + loc]},
                                        reinterpret_cast<F4*>(out.app) + g0 + loc);
}

}  // namespace

hipError_t launch_project_bwd(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                              const Projected& proj, const float* grad2d, const GradPtrs& out, float* mean2d_norm,
                              float* absgrad, hipStream_t s, bool grads_zeroed) {
    const unsigned blocks = (unsigned)((n + kSpan - 1) / kSpan);
    const hipEvent_t timed_ = timer_begin(GS_KERNEL_PROJECT_BWD, s);
    if (grads_zeroed)
        hipLaunchKernelGGL(k_project_bwd<true>, dim3(blocks), dim3(kPB), 0, s, g, n, vt, opt, proj, grad2d, out,
                           mean2d_norm, absgrad);
    else
        hipLaunchKernelGGL(k_project_bwd<false>, dim3(blocks), dim3(kPB), 0, s, g, n, vt, opt, proj, grad2d, out,
                           mean2d_norm, absgrad);
    timer_end(timed_, s);
    return hipGetLastError();
}

namespace {

// Zeroes n floats with 16-byte streaming stores from a grid of at most
// kZeroGrid workgroups (grid-stride).  Beside the issue-bound compositing
// backward, one workgroup on a quarter of the compute units writes over
// 2 TB/s and takes a seventh of those units' wave slots; a grid over every
// unit slows the backward by more than the fill saves.
constexpr unsigned kZeroGrid = 64;
__global__ __launch_bounds__(256) void k_zero_floats(float* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t head = (int64_t)(((16 - ((uintptr_t)p & 15)) & 15) / 4);     // floats before the first 16-byte boundary
    const int64_t h = head < n ? head : n;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i0 < h) p[i0] = 0.0f;
    F4* q = reinterpret_cast<F4*>(p + h);
    const int64_t n4 = (n - h) / 4;
    for (int64_t i = i0; i < n4; i += stride) __builtin_nontemporal_store(F4{0.0f, 0.0f, 0.0f, 0.0f}, q + i);
    const int64_t t = h + 4 * n4 + i0;
    if (t < n) p[t] = 0.0f;
}

}  // namespace

hipError_t launch_zero_grads(const GradPtrs& out, int64_t n, hipStream_t s) {
    const struct {
        float* p;
        int64_t count;
    } parts[] = {{out.means, 3 * n}, {out.scales, 3 * n}, {out.quats, 4 * n}, {out.opac, n}, {out.sh, 48 * n},
                 {out.app, out.app ? 4 * n : 0}};
    for (const auto& a : parts) {
        if (!a.p || a.count <= 0) continue;
        const int64_t need = (a.count / 4 + 255) / 256 + 1;
        const unsigned grid = (unsigned)(need < (int64_t)kZeroGrid ? need : (int64_t)kZeroGrid);
        hipLaunchKernelGGL(k_zero_floats, dim3(grid), dim3(256), 0, s, a.p, a.count);
    }
    return hipGetLastError();
}

}  // namespace gs
