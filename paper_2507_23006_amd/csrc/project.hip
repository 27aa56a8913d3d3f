// Projection of 3D Gaussians to 2D (EWA) with SH colour -- gfx950.
//
// Two launch shapes share the per-view arithmetic: one thread per Gaussian
// walking every view of the launch (training: all views see the same
// Gaussians, whose parameters are then read from HBM once), or one thread
// per slot of a segment table (served views, each with its own selection of
// level-of-detail segments).  Geometry reads are structure-of-arrays;
// records are written as four float4s so the compositing kernels gather a
// record with 16-byte loads.  Arithmetic is FP64: the kernel is bound by HBM and
// CDNA4 executes FP64 FMAs at the non-packed FP32 rate, so the geometry that
// decides tile rectangles and depth keys carries no FP32 rounding.
//
// Paper: §3.1 (Eq. 1 for Sigma = R S S^T R^T; the projection to 2D Gaussians
// G' in the text after it), §3.5.4 (anti-aliasing dilation and opacity
// compensation), colour c of §3.1 as degree-3 SH.
#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ void quat_rotation(double w, double x, double y, double z, double R[9]) {
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// camera-space position t = R mu + t_w of a mean in view V
__device__ __forceinline__ void view_point(const ViewK& V, double mu0, double mu1, double mu2, double& tx, double& ty,
                                           double& tz) {
    tx = (double)V.R[0] * mu0 + (double)V.R[1] * mu1 + (double)V.R[2] * mu2 + (double)V.t[0];
    ty = (double)V.R[3] * mu0 + (double)V.R[4] * mu1 + (double)V.R[5] * mu2 + (double)V.t[1];
    tz = (double)V.R[6] * mu0 + (double)V.R[7] * mu1 + (double)V.R[8] * mu2 + (double)V.t[2];
}

// M = R(q) diag(s) of Gaussian g with scales s0..s2, and its opacity op
// (times 1 - do under appearance offsets); false for a zero quaternion
__device__ __forceinline__ bool load_shape(const GaussPtrs& gp, int64_t n, int64_t g, double s0, double s1, double s2,
                                           double op, double M[9], double& opac) {
    double qw = gp.quats[g], qx = gp.quats[n + g], qy = gp.quats[2 * n + g], qz = gp.quats[3 * n + g];
    const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qn > 0.0)) return false;
    const double inv = 1.0 / qn;
    double Rq[9];
    quat_rotation(qw * inv, qx * inv, qy * inv, qz * inv, Rq);
    M[0] = Rq[0] * s0; M[1] = Rq[1] * s1; M[2] = Rq[2] * s2;
    M[3] = Rq[3] * s0; M[4] = Rq[4] * s1; M[5] = Rq[5] * s2;
    M[6] = Rq[6] * s0; M[7] = Rq[7] * s1; M[8] = Rq[8] * s2;
    opac = op;
    if (gp.app) opac *= 1.0 - (double)gp.app[4 * g + 3];
    return true;
}

// Exact tile culling of a rectangle of w x h <= 64 tiles at (ix0, iy0): bit
// (ty - iy0) w + (tx - ix0) is set when the alpha ellipse
// q(d) = A dx^2 + 2 B dx dy + C dy^2 <= L, L = 2 tau (1 + 4e-6), reaches the
// tile's pixel-centre rectangle widened by 1e-3 px.  Row by row: the ellipse
// within a row's strip is convex, so it meets a tile iff its x-extent over the
// strip meets the tile's columns.  For fixed y the ellipse spans
// x = (-B y -+ sqrt(A L - det y^2)) / A; the upper end is concave in y and
// peaks at the rightmost point (X, -B X / C), X = sqrt(L C / det), the lower
// end is convex with its minimum at (-X, B X / C), so over a strip (clipped
// to the ellipse's y-extent +-sqrt(L A / det)) both come from those y clamped
// into it.  O(rows) square roots per Gaussian instead of work per tile, so a
// wave is not held by its widest lane.  Plain IEEE operations in a fixed
// order (no contraction).
__device__ uint64_t covered_tiles(const ViewK& V, double mx, double my, double A, double B, double C, double tau,
                                  int ix0, int iy0, int w, int h) {
#pragma clang fp contract(off)
    const double L = 2.0 * tau * (1.0 + 4e-6);
    const double det = A * C - B * B;
    const double X = sqrt(L * C / det), Y = sqrt(L * A / det), yr = -B / C * X;
    uint64_t m = 0;
    for (int j = 0; j < h; ++j) {
        const int ty = iy0 + j;
        int py1 = ty * kTile + kTile - 1;
        if (py1 > V.H - 1) py1 = V.H - 1;
        const double ylo = (double)(ty * kTile) + 0.5 - 1e-3 - my, yhi = (double)py1 + 0.5 + 1e-3 - my;
        const double a = ylo > -Y ? ylo : -Y, b = yhi < Y ? yhi : Y;
        if (a > b) continue;
        const double y1 = yr < a ? a : (yr > b ? b : yr);
        const double y2 = -yr < a ? a : (-yr > b ? b : -yr);
        const double r1 = A * L - det * y1 * y1, r2 = A * L - det * y2 * y2;
        const double xhi_e = (-B * y1 + sqrt(r1 > 0.0 ? r1 : 0.0)) / A;
        const double xlo_e = (-B * y2 - sqrt(r2 > 0.0 ? r2 : 0.0)) / A;
        for (int i = 0; i < w; ++i) {
            const int tx = ix0 + i;
            int px1 = tx * kTile + kTile - 1;
            if (px1 > V.W - 1) px1 = V.W - 1;
            const double xlo = (double)(tx * kTile) + 0.5 - 1e-3 - mx, xhi = (double)px1 + 0.5 + 1e-3 - mx;
            if (xlo <= xhi_e && xhi >= xlo_e) m |= 1ull << (j * w + i);
        }
    }
    return m;
}

// 2D Gaussian of (t, M, opac) in view V: writes the record's geometry words
// (float4s 0, 1 and 3; the .w of float4 2 is returned in yfrac for the
// colour's write) and the rectangle of `slot`; returns the number of tiles
// covered, 0 when culled
__device__ __forceinline__ uint32_t project_view(const ViewK& V, const OptK& opt, double tx, double ty, double tz,
                                                 const double M[9], double opac, const Projected& out,
                                                 int64_t slot, float& yfrac) {
    const double W0 = V.R[0], W1 = V.R[1], W2 = V.R[2], W3 = V.R[3], W4 = V.R[4], W5 = V.R[5], W6 = V.R[6],
                 W7 = V.R[7], W8 = V.R[8];
    const double fx = V.fx, fy = V.fy;
    const double u = tx / tz, vv = ty / tz;
    const double uc = fmin(fmax(u, V.ulo), V.uhi);
    const double vc = fmin(fmax(vv, V.vlo), V.vhi);
    const double j00 = fx / tz, j02 = -fx * uc / tz, j11 = fy / tz, j12 = -fy * vc / tz;
    // Tm = J W (2x3), Vm = Tm M (2x3): Sigma_2D = Vm Vm^T
    const double T0 = j00 * W0 + j02 * W6, T1 = j00 * W1 + j02 * W7, T2 = j00 * W2 + j02 * W8;
    const double T3 = j11 * W3 + j12 * W6, T4 = j11 * W4 + j12 * W7, T5 = j11 * W5 + j12 * W8;
    const double a0 = T0 * M[0] + T1 * M[3] + T2 * M[6];
    const double a1 = T0 * M[1] + T1 * M[4] + T2 * M[7];
    const double a2 = T0 * M[2] + T1 * M[5] + T2 * M[8];
    const double b0 = T3 * M[0] + T4 * M[3] + T5 * M[6];
    const double b1 = T3 * M[1] + T4 * M[4] + T5 * M[7];
    const double b2 = T3 * M[2] + T4 * M[5] + T5 * M[8];
    const double ca = a0 * a0 + a1 * a1 + a2 * a2;
    const double cb = a0 * b0 + a1 * b1 + a2 * b2;
    const double cc = b0 * b0 + b1 * b1 + b2 * b2;
    // det(Sigma_2D) = |a x b|^2 (Lagrange identity, no cancellation)
    const double x0 = a1 * b2 - a2 * b1, x1 = a2 * b0 - a0 * b2, x2 = a0 * b1 - a1 * b0;
    const double det2 = x0 * x0 + x1 * x1 + x2 * x2;
    const double dil = (double)opt.dilation;
    const double ad = ca + dil, cd = cc + dil;
    const double detd = det2 + dil * (ca + cc) + dil * dil;
    const double mx = fx * u + (double)V.cx, my = fy * vv + (double)V.cy;
    const double lmax = 0.5 * (ad + cd) + sqrt(0.25 * (ad - cd) * (ad - cd) + cb * cb);
    const double ext = 3.0 * sqrt(lmax);
    if (!(detd > 0.0 && isfinite(ext) && isfinite(mx) && isfinite(my))) return 0;
    const double r = ceil(ext);
    const int TW = V.tiles_x, TH = V.tiles_y;
    double x0t = floor((floor(mx) - r) * (1.0 / kTile)), x1t = floor((floor(mx) + r) * (1.0 / kTile));
    double y0t = floor((floor(my) - r) * (1.0 / kTile)), y1t = floor((floor(my) + r) * (1.0 / kTile));
    x0t = fmax(x0t, 0.0);
    y0t = fmax(y0t, 0.0);
    x1t = fmin(x1t, (double)(TW - 1));
    y1t = fmin(y1t, (double)(TH - 1));
    // Tile-based culling: alpha = o' G' reaches 1/255 only inside the ellipse
    // x^T Sigma'^-1 x <= 2 tau, tau = ln(255 o'), whose bounding box has
    // half-widths sqrt(2 tau Sigma'_xx), sqrt(2 tau Sigma'_yy).  Widened by
    // margins for the float32 compositing arithmetic (1e-5 on tau, relative
    // 1e-6 and 1e-3 px), the box keeps the tiles whose pixel centres it
    // reaches; the rectangle drops the others, which no entry could change.
    // The box also travels in the record for the per-quadrant culling.
    const double rho = opt.aa ? (det2 > 0.0 ? sqrt(det2 / detd) : 0.0) : 1.0;
    const double o2 = opac * rho;
    if (!((float)o2 >= kAlphaMin)) return 0;     // below the skip threshold everywhere
    const double tau = log(255.0 * o2) + 1e-5;
    const double hxd = sqrt(2.0 * tau * ad) * (1.0 + 1e-6) + 1e-3;
    const double hyd = sqrt(2.0 * tau * cd) * (1.0 + 1e-6) + 1e-3;
    x0t = fmax(x0t, floor(ceil(mx - hxd - 0.5) * (1.0 / kTile)));
    x1t = fmin(x1t, floor(floor(mx + hxd - 0.5) * (1.0 / kTile)));
    y0t = fmax(y0t, floor(ceil(my - hyd - 0.5) * (1.0 / kTile)));
    y1t = fmin(y1t, floor(floor(my + hyd - 0.5) * (1.0 / kTile)));
    if (!(x0t <= x1t && y0t <= y1t)) return 0;
    const int ix0 = (int)x0t, iy0 = (int)y0t, ix1 = (int)x1t, iy1 = (int)y1t;
    const int w = ix1 - ix0 + 1, h = iy1 - iy0 + 1;
    uint32_t covered = (uint32_t)(w * h);
    if (out.tile_mask) {
        uint64_t m = 0;
        if (w * h <= 64) {
            m = covered_tiles(V, mx, my, cd / detd, -cb / detd, ad / detd, tau, ix0, iy0, w, h);
            if (!m) return 0;     // the ellipse reaches no pixel centre of the image
            covered = (uint32_t)__popcll(m);
        }
        out.tile_mask[slot] = m;
    }
    const double invd = 1.0 / detd;
    const double A = cd * invd, B = -cb * invd, C = ad * invd;
    // mean = integer part (exact in float32) + fraction, so that the
    // compositing kernels can form a tile-relative mean without the
    // rounding of a large absolute pixel coordinate
    const double fmx = floor(mx), fmy = floor(my);
    out.rec[4 * slot + 0] = make_float4((float)fmx, (float)fmy, (float)(-0.5 * kLog2e * A), (float)(-kLog2e * B));
    out.rec[4 * slot + 1] = make_float4((float)(-0.5 * kLog2e * C), (float)(opac * rho), (float)tz, (float)(mx - fmx));
    yfrac = (float)(my - fmy);
    out.rec[4 * slot + 3] = make_float4((float)hxd, (float)hyd, 0.0f, 0.0f);
    out.rect[slot] = make_uint2((uint32_t)(V.tile_off + iy0 * TW + ix0), (uint32_t)w | ((uint32_t)TW << 16));
    return covered;
}

// view-dependent colour of a mean seen by V into the record's .xyz of
// float4 2 (written whole, with yfrac as its .w); the coefficient row is
// read as 16-byte vectors; cb is the constant of the polynomial (1/2, or
// the appearance colour offset)
__device__ __forceinline__ void colour_view(const ViewK& V, const OptK& opt, double mu0, double mu1, double mu2,
                                            const float4* __restrict__ shq, float4 cb, const Projected& out,
                                            int64_t slot, float yfrac) {
    const int nb = (opt.sh_degree + 1) * (opt.sh_degree + 1);
    const int nq = (3 * nb + 3) >> 2;    // float4s that hold the used coefficients
    // direction in FP64 (mu and the camera centre are large numbers), the
    // SH polynomial in FP32
    const double e0 = mu0 - V.campos[0], e1 = mu1 - V.campos[1], e2 = mu2 - V.campos[2];
    const double inv = 1.0 / sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    float Y[16];
    sh_eval_basis<float>((float)(e0 * inv), (float)(e1 * inv), (float)(e2 * inv), opt.sh_degree, Y);
    float shv[48];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const float4 t = q < nq ? shq[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        shv[4 * q + 0] = t.x; shv[4 * q + 1] = t.y; shv[4 * q + 2] = t.z; shv[4 * q + 3] = t.w;
    }
    float c[3] = {cb.x, cb.y, cb.z};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < nb) {
            c[0] = fmaf(shv[3 * k + 0], Y[k], c[0]);
            c[1] = fmaf(shv[3 * k + 1], Y[k], c[1]);
            c[2] = fmaf(shv[3 * k + 2], Y[k], c[2]);
        }
    }
    out.rec[4 * slot + 2] = make_float4(fmaxf(c[0], 0.0f), fmaxf(c[1], 0.0f), fmaxf(c[2], 0.0f), yfrac);
}

// Conservative pre-test of project_view: false only when the Gaussian
// certainly covers no tile.  With M = R(q) diag(s), R orthonormal,
// lambda_max(Sigma_2D) = |J W M|^2 <= |J|_F^2 s_max^2, so the 3-sigma radius
// is at most 3 sqrt(|J|_F^2 s_max^2 + dilation); if even that rectangle
// misses the image, or the opacity is below the skip threshold (o' = o rho
// <= o), the exact test culls too.
__device__ __forceinline__ bool may_cover(const ViewK& V, const OptK& opt, double tx, double ty, double tz,
                                          double smax, float opac) {
    if (!(opac >= kAlphaMin)) return false;
    const double u = tx / tz, vv = ty / tz;
    const double uc = fmin(fmax(u, V.ulo), V.uhi), vc = fmin(fmax(vv, V.vlo), V.vhi);
    const double fx = V.fx, fy = V.fy;
    const double jf2 = (fx * fx * (1.0 + uc * uc) + fy * fy * (1.0 + vc * vc)) / (tz * tz);
    const double rb = ceil(3.0 * sqrt(jf2 * smax * smax + (double)opt.dilation) * (1.0 + 1e-6)) + 1.0;
    const double mx = fx * u + (double)V.cx, my = fy * vv + (double)V.cy;
    if (!(isfinite(rb) && isfinite(mx) && isfinite(my))) return true;    // the exact path decides
    const double fmx = floor(mx), fmy = floor(my);
    return fmx + rb >= 0.0 && fmx - rb <= (double)(V.tiles_x * kTile - 1) && fmy + rb >= 0.0 &&
           fmy - rb <= (double)(V.tiles_y * kTile - 1);
}

// exact projection and colour of Gaussian g (mean mu, scales s, opacity
// op, as stored) into the views of `cand`; slot of view v = slot_base +
// v * slot_stride
__device__ __forceinline__ void project_candidate(const GaussPtrs& gp, int64_t n, const ViewTable& vt,
                                                  const OptK& opt, const Projected& out, int64_t g, uint32_t cand,
                                                  int64_t slot_base, int64_t slot_stride, const float mu[3],
                                                  const float sc[3], float op) {
    const double mu0 = mu[0], mu1 = mu[1], mu2 = mu[2];
    double M[9], opac = 0.0;
    const bool shape_ok = load_shape(gp, n, g, sc[0], sc[1], sc[2], op, M, opac);
    const float4* shq = reinterpret_cast<const float4*>(gp.sh) + 12 * g;
    const float4 cb = gp.app ? reinterpret_cast<const float4*>(gp.app)[g] : make_float4(0.5f, 0.5f, 0.5f, 0.0f);
    for (int v = 0; v < vt.n_views; ++v) {
        if (!(cand & (1u << v))) continue;
        const ViewK& V = vt.v[v];
        const int64_t slot = slot_base + v * slot_stride;
        double tx, ty, tz;
        view_point(V, mu0, mu1, mu2, tx, ty, tz);
        float yfrac = 0.0f;
        const uint32_t ntiles = shape_ok ? project_view(V, opt, tx, ty, tz, M, opac, out, slot, yfrac) : 0u;
        if (ntiles) colour_view(V, opt, mu0, mu1, mu2, shq, cb, out, slot, yfrac);
        out.tiles[slot] = ntiles;
        out.dkey[slot] = ntiles ? __float_as_uint((float)tz) : 0xFFFFFFFFu;
    }
}

constexpr int kPF = 256;                 // threads per workgroup
constexpr int kPFPer = 4;                // items per thread in the pre-test
constexpr int kPFSpan = kPF * kPFPer;    // items per workgroup

// appends the lanes with cand != 0 to the workgroup's LDS list as
// (local index | cand << 16)
__device__ __forceinline__ void list_append(uint32_t cand, int loc, int lane, uint32_t* s_list, uint32_t* s_count) {
    const uint64_t m = __ballot(cand != 0);
    if (!m) return;
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(s_count, (uint32_t)__popcll(m));
    base = __shfl(base, 0);
    if (cand) s_list[base + below] = (uint32_t)loc | (cand << 16);
}

// Every view of the launch sees the same n Gaussians: slot = view * n + g.
// A workgroup owns 1024 Gaussians.  Pass 1 reads each mean (and, for
// Gaussians in front of some camera, its scales and opacity), runs the
// conservative pre-test per view, writes the culled slots' count and key
// with coalesced stores and lists the rest in LDS with the values it read;
// pass 2 runs the FP64 EWA and the colour on full waves of listed Gaussians
// only (a large scene leaves most lanes culled, which would otherwise idle
// through the FP64 chain of their wave's few visible neighbours), reading
// from HBM only their quaternions and coefficient rows.
__global__ __launch_bounds__(kPF, 4) void k_project_fwd(GaussPtrs gp, int64_t n, ViewTable vt, OptK opt,
                                                     Projected out) {
    __shared__ uint32_t s_list[kPFSpan];
    __shared__ uint32_t s_group[kPFSpan];   // the list grouped by view mask (several views)
    __shared__ uint32_t s_hist[256];
    __shared__ float s_par[7][kPFSpan];     // listed Gaussians' mean, scales, opacity
    __shared__ uint32_t s_count;
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t g0 = (int64_t)blockIdx.x * kPFSpan;
    if (tid == 0) s_count = 0;
    __syncthreads();
    // the thread's kPFPer Gaussians move through each phase together, so
    // their independent loads are in flight at once: means; depths and the
    // views each lies in; scales and opacity of those in front of a view;
    // the conservative test
    float mu[kPFPer][3];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        const int64_t g = g0 + i * kPF + tid;
        const bool ok = g < n;
        mu[i][0] = ok ? gp.means[g] : 0.0f;
        mu[i][1] = ok ? gp.means[n + g] : 0.0f;
        mu[i][2] = ok ? gp.means[2 * n + g] : 0.0f;
    }
    uint32_t front[kPFPer];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        front[i] = 0;
        if (g0 + i * kPF + tid >= n) continue;
        for (int v = 0; v < vt.n_views; ++v) {
            const ViewK& V = vt.v[v];
            double tx, ty, tz;
            view_point(V, mu[i][0], mu[i][1], mu[i][2], tx, ty, tz);
            if (tz >= (double)V.znear && tz <= (double)V.zfar) front[i] |= 1u << v;
        }
    }
    float sc[kPFPer][3], op[kPFPer];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        const int64_t g = g0 + i * kPF + tid;
        sc[i][0] = sc[i][1] = sc[i][2] = op[i] = 0.0f;
        if (front[i]) {
            sc[i][0] = gp.scales[g];
            sc[i][1] = gp.scales[n + g];
            sc[i][2] = gp.scales[2 * n + g];
            op[i] = gp.opac[g];
        }
    }
    for (int i = 0; i < kPFPer; ++i) {
        const int loc = i * kPF + tid;
        const int64_t g = g0 + loc;
        uint32_t cand = 0;
        if (g < n) {
            for (int v = 0; v < vt.n_views; ++v) {
                const ViewK& V = vt.v[v];
                if (front[i] & (1u << v)) {
                    double tx, ty, tz;
                    view_point(V, mu[i][0], mu[i][1], mu[i][2], tx, ty, tz);
                    const float sm = fmaxf(fabsf(sc[i][0]), fmaxf(fabsf(sc[i][1]), fabsf(sc[i][2])));
                    if (may_cover(V, opt, tx, ty, tz, (double)sm, op[i])) cand |= 1u << v;
                }
                if (!(cand & (1u << v))) {
                    const int64_t slot = (int64_t)v * n + g;
                    __builtin_nontemporal_store(0u, out.tiles + slot);
                    __builtin_nontemporal_store(0xFFFFFFFFu, out.dkey + slot);
                }
            }
            if (cand) {
                s_par[0][loc] = mu[i][0]; s_par[1][loc] = mu[i][1]; s_par[2][loc] = mu[i][2];
                s_par[3][loc] = sc[i][0]; s_par[4][loc] = sc[i][1]; s_par[5][loc] = sc[i][2];
                s_par[6][loc] = op[i];
            }
        }
        list_append(cand, loc, lane, s_list, &s_count);
    }
    __syncthreads();
    const uint32_t cnt = s_count;
    const uint32_t* lst = s_list;
    if (vt.n_views > 1) {      // Gaussians that are candidates in the same views side by side
        group_by_views(s_list, cnt, s_group, s_hist);
        lst = s_group;
    }
    for (uint32_t j = tid; j < cnt; j += kPF) {
        const uint32_t e = lst[j];
        const int loc = (int)(e & 0xFFFFu);
        const float mu[3] = {s_par[0][loc], s_par[1][loc], s_par[2][loc]};
        const float sc[3] = {s_par[3][loc], s_par[4][loc], s_par[5][loc]};
        project_candidate(gp, n, vt, opt, out, g0 + loc, e >> 16, g0 + loc, n, mu, sc, s_par[6][loc]);
    }
}

// slot s of a segment table: the last segment with slot_start <= s
__device__ __forceinline__ int segment_of(const SlotSeg* __restrict__ segs, int32_t n_seg, uint32_t s) {
    int lo = 0, hi = n_seg;      // invariant: segs[lo].slot_start <= s, answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].slot_start <= s) lo = mid; else hi = mid;
    }
    return lo;
}

// Views with their own selections of Gaussians (served requests): slot s
// maps to Gaussian gstart + (s - slot_start) of its segment, seen by the
// segment's view.  Same two passes as k_project_fwd, over 1024 slots, with
// the values pass 1 read kept in LDS for pass 2; the segments that the
// workgroup's slots fall in are staged in LDS when there are at most
// kSlotSegCache of them (else each slot searches them in global memory).
constexpr int kSlotSegCache = 128;
__global__ __launch_bounds__(kPF, 4) void k_project_slots(GaussPtrs gp, int64_t n, ViewTable vt, OptK opt,
                                                          const SlotSeg* __restrict__ segs, int32_t n_seg,
                                                          uint32_t n_slots, Projected out) {
    __shared__ uint32_t s_list[kPFSpan];
    __shared__ float s_par[7][kPFSpan];     // listed slots' mean, scales, opacity
    __shared__ uint32_t s_gid[kPFSpan];     // listed slots' Gaussian (n < 2^32, checked at launch)
    __shared__ SlotSeg s_seg[kSlotSegCache];
    __shared__ int32_t s_seg_lo, s_seg_n;
    __shared__ uint32_t s_count;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t s0 = blockIdx.x * kPFSpan;
    // the segments of this workgroup's slots, staged in LDS when few
    if (tid == 0) {
        s_count = 0;
        const int32_t lo = segment_of(segs, n_seg, s0);
        const int32_t hi = segment_of(segs, n_seg, min(s0 + (uint32_t)kPFSpan, n_slots) - 1u);
        s_seg_lo = lo;
        s_seg_n = hi - lo + 1;
    }
    __syncthreads();
    const int32_t seg_lo = s_seg_lo, seg_n = s_seg_n;
    const bool staged = seg_n <= kSlotSegCache;
    if (staged)
        for (int k = tid; k < seg_n; k += kPF) s_seg[k] = segs[seg_lo + k];
    __syncthreads();
    // the thread's kPFSpan / kPF slots move through each phase together, so
    // that their independent loads are in flight at once
    constexpr uint32_t kNone = 0xFFFFFFFFu;      // no slot (n < 2^32, so no Gaussian has this index)
    uint32_t g[kPFPer], view[kPFPer];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        const uint32_t s = s0 + i * kPF + tid;
        g[i] = kNone;
        view[i] = 0;
        if (s < n_slots) {
            SlotSeg sg;
            if (staged) {
                int lo = 0, hi = seg_n;      // invariant: s_seg[lo].slot_start <= s, answer in [lo, hi)
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_seg[mid].slot_start <= s) lo = mid; else hi = mid;
                }
                sg = s_seg[lo];
            } else {
                sg = segs[seg_lo + segment_of(segs + seg_lo, seg_n, s)];
            }
            g[i] = (uint32_t)(sg.gstart + (int64_t)(s - sg.slot_start));
            view[i] = sg.view;
        }
    }
    float mu[kPFPer][3];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        const bool ok = g[i] != kNone;
        mu[i][0] = ok ? gp.means[g[i]] : 0.0f;
        mu[i][1] = ok ? gp.means[n + g[i]] : 0.0f;
        mu[i][2] = ok ? gp.means[2 * n + g[i]] : 0.0f;
    }
    bool front[kPFPer];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        front[i] = false;
        if (g[i] == kNone) continue;
        const ViewK& V = vt.v[view[i]];
        double tx, ty, tz;
        view_point(V, mu[i][0], mu[i][1], mu[i][2], tx, ty, tz);
        front[i] = tz >= (double)V.znear && tz <= (double)V.zfar;
    }
    float sc[kPFPer][3], op[kPFPer];
#pragma unroll
    for (int i = 0; i < kPFPer; ++i) {
        sc[i][0] = sc[i][1] = sc[i][2] = op[i] = 0.0f;
        if (front[i]) {
            sc[i][0] = gp.scales[g[i]];
            sc[i][1] = gp.scales[n + g[i]];
            sc[i][2] = gp.scales[2 * n + g[i]];
            op[i] = gp.opac[g[i]];
        }
    }
    for (int i = 0; i < kPFPer; ++i) {
        const int loc = i * kPF + tid;
        const uint32_t s = s0 + (uint32_t)loc;
        uint32_t cand = 0;
        if (g[i] != kNone) {
            if (front[i]) {
                const ViewK& V = vt.v[view[i]];
                double tx, ty, tz;
                view_point(V, mu[i][0], mu[i][1], mu[i][2], tx, ty, tz);
                const double smax = fmax(fabs((double)sc[i][0]), fmax(fabs((double)sc[i][1]), fabs((double)sc[i][2])));
                if (may_cover(V, opt, tx, ty, tz, smax, op[i])) cand = 1u << view[i];
            }
            if (!cand) {
                out.tiles[s] = 0u;
                out.dkey[s] = 0xFFFFFFFFu;
            } else {
                s_par[0][loc] = mu[i][0]; s_par[1][loc] = mu[i][1]; s_par[2][loc] = mu[i][2];
                s_par[3][loc] = sc[i][0]; s_par[4][loc] = sc[i][1]; s_par[5][loc] = sc[i][2];
                s_par[6][loc] = op[i];
                s_gid[loc] = g[i];
            }
        }
        list_append(cand, loc, lane, s_list, &s_count);
    }
    __syncthreads();
    const uint32_t cnt = s_count;
    for (uint32_t j = tid; j < cnt; j += kPF) {
        const uint32_t e = s_list[j];
        const int loc = (int)(e & 0xFFFFu);
        const uint32_t s = s0 + (uint32_t)loc;
        // one view bit: the slot is s itself (stride 0)
        const float mu1[3] = {s_par[0][loc], s_par[1][loc], s_par[2][loc]};
        const float sc1[3] = {s_par[3][loc], s_par[4][loc], s_par[5][loc]};
        project_candidate(gp, n, vt, opt, out, (int64_t)s_gid[loc], e >> 16, (int64_t)s, 0, mu1, sc1, s_par[6][loc]);
    }
}

}  // namespace

hipError_t launch_project_fwd(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                              const Projected& out, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + kPFSpan - 1) / kPFSpan);
    const hipEvent_t timed_ = timer_begin(GS_KERNEL_PROJECT_FWD, s);
    hipLaunchKernelGGL(k_project_fwd, dim3(blocks), dim3(kPF), 0, s, g, n, vt, opt, out);
    timer_end(timed_, s);
    return hipGetLastError();
}

hipError_t launch_project_slots(const GaussPtrs& g, int64_t n, const ViewTable& vt, const OptK& opt,
                                const SlotSeg* segs, int32_t n_seg, uint32_t n_slots, const Projected& out,
                                hipStream_t s) {
    if (!n_slots) return hipSuccess;
    if (n > 0xFFFFFFFFLL) return hipErrorInvalidValue;     // listed Gaussians are kept as 32-bit indices
    hipLaunchKernelGGL(k_project_slots, dim3((n_slots + kPFSpan - 1) / kPFSpan), dim3(kPF), 0, s, g, n, vt, opt, segs,
                       n_seg, n_slots, out);
    return hipGetLastError();
}

}  // namespace gs
