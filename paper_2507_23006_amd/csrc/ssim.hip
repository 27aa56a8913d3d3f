// D-SSIM term of the training loss (Eq. 3) and its gradient -- gfx950.
//
// SSIM per pixel and channel with an 11x11 Gaussian window (sigma 1.5,
// weights normalised to 1), zero outside the image, C1 = 0.01^2,
// C2 = 0.03^2:  s = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sx^2 +
// sy^2 + C2)) with mx = G*x, sx^2 = G*(x^2) - mx^2, sxy = G*(xy) - mx my.
// The term is weight * (1 - mean s) over 3 W H values.
//
// Forward: one workgroup per 16x16 tile stages the 26x26 halo of x and y
// (all three channels, one fetch of the interleaved pixels) in LDS, blurs x,
// y, x^2, y^2, xy horizontally (26 x 16) and then vertically (16 x 16), one
// channel after another, and writes s's partial derivatives with respect to
// a = G*x, b = G*(x^2), c = G*(xy) for the backward, plus the tile's sum
// of s.  Backward: the blur is self-adjoint (symmetric window, zero
// padding), so dL/dx = -weight / (3 W H) (G*Pa + 2 x G*Pb + y G*Pc), three
// more separable blurs over the same halo scheme.  Both kernels are bound by
// LDS and VALU at a few hundred flops per pixel.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kR = 5;                     // window radius
constexpr int kWin = 2 * kR + 1;          // 11 taps
constexpr int kTileS = 16;
constexpr int kHalo = kTileS + 2 * kR;    // 26
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct SsimWin {
    float w[kWin];
};

// normalised Gaussian taps exp(-k^2 / (2 sigma^2)), sigma = 1.5 (host side)
SsimWin ssim_window() {
    SsimWin t;
    double s = 0.0, v[kWin];
    for (int k = 0; k < kWin; ++k) {
        const double d = k - kR;
        v[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
        s += v[k];
    }
    for (int k = 0; k < kWin; ++k) t.w[k] = (float)(v[k] / s);
    return t;
}

// the three channels of image pixel (px, py) of an interleaved [H][W][3] image, 0 outside
__device__ __forceinline__ void pix3(const float* __restrict__ img, int W, int H, int px, int py, float v[3]) {
    if (px >= 0 && px < W && py >= 0 && py < H) {
        const float* p = img + 3 * ((int64_t)py * W + px);
        v[0] = p[0]; v[1] = p[1]; v[2] = p[2];
    } else {
        v[0] = v[1] = v[2] = 0.0f;
    }
}

// One workgroup per 16x16 tile and all three channels: the interleaved halo
// is fetched once; the channels are blurred one after another through the
// same LDS rows.
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int W, int H,
                                                  SsimWin win, float* __restrict__ Pa, float* __restrict__ Pb,
                                                  float* __restrict__ Pc, double* __restrict__ partial) {
    __shared__ float sx[3][kHalo][kHalo], sy[3][kHalo][kHalo];
    __shared__ float h[5][kHalo][kTileS];
    __shared__ double s_sum[4];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kTileS - kR, y0 = blockIdx.y * kTileS - kR;
    for (int i = tid; i < kHalo * kHalo; i += 256) {
        const int r = i / kHalo, c = i - r * kHalo;
        float a[3], b[3];
        pix3(x, W, H, x0 + c, y0 + r, a);
        pix3(y, W, H, x0 + c, y0 + r, b);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            sx[ch][r][c] = a[ch];
            sy[ch][r][c] = b[ch];
        }
    }
    const int r = tid / kTileS, c = tid - r * kTileS;
    const int px = blockIdx.x * kTileS + c, py = blockIdx.y * kTileS + r;
    const bool inside = px < W && py < H;
    double s_px = 0.0;
    float pa[3], pb[3], pc[3];
    for (int ch = 0; ch < 3; ++ch) {
        __syncthreads();     // halo loaded / previous channel's rows consumed
        for (int i = tid; i < kHalo * kTileS; i += 256) {
            const int hr = i / kTileS, hc = i - hr * kTileS;
            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f, a4 = 0.0f;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const float xv = sx[ch][hr][hc + k], yv = sy[ch][hr][hc + k], w = win.w[k];
                a0 = fmaf(w, xv, a0);
                a1 = fmaf(w, yv, a1);
                a2 = fmaf(w, xv * xv, a2);
                a3 = fmaf(w, yv * yv, a3);
                a4 = fmaf(w, xv * yv, a4);
            }
            h[0][hr][hc] = a0; h[1][hr][hc] = a1; h[2][hr][hc] = a2; h[3][hr][hc] = a3; h[4][hr][hc] = a4;
        }
        __syncthreads();
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float w = win.w[k];
#pragma unroll
            for (int q = 0; q < 5; ++q) m[q] = fmaf(w, h[q][r + k][c], m[q]);
        }
        const float mx = m[0], my = m[1];
        const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * cxy + kC2;
        const float B1 = mx * mx + my * my + kC1, B2 = vx + vy + kC2;
        const float inv = 1.0f / (B1 * B2);
        const float sv = A1 * A2 * inv;
        pa[ch] = (2.0f * my * (A2 - A1) - sv * 2.0f * mx * (B2 - B1)) * inv;   // ds/d(G*x)
        pb[ch] = -sv / B2;                                                      // ds/d(G*x^2)
        pc[ch] = 2.0f * A1 * inv;                                               // ds/d(G*xy)
        if (inside) s_px += sv;
    }
    if (inside) {
        const int64_t o = 3 * ((int64_t)py * W + px);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            Pa[o + ch] = pa[ch];
            Pb[o + ch] = pb[ch];
            Pc[o + ch] = pc[ch];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s_px += __shfl_xor(s_px, off, 64);
    if ((tid & 63) == 0) s_sum[tid >> 6] = s_px;
    __syncthreads();
    if (tid == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
}

__global__ __launch_bounds__(1024) void k_ssim_total(const double* __restrict__ partial, int n, double scale,
                                                     float weight, float* __restrict__ loss) {
    __shared__ double s_sum[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += partial[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < 16; ++w) b += s_sum[w];
        loss[0] = (float)((double)weight * (1.0 - b * scale));
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int W, int H,
                                                  SsimWin win, const float* __restrict__ Pa,
                                                  const float* __restrict__ Pb, const float* __restrict__ Pc,
                                                  float gscale, float* __restrict__ dx) {
    __shared__ float sp[3][3][kHalo][kHalo];     // [quantity][channel]
    __shared__ float h[3][kHalo][kTileS];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * kTileS - kR, y0 = blockIdx.y * kTileS - kR;
    for (int i = tid; i < kHalo * kHalo; i += 256) {
        const int r = i / kHalo, c = i - r * kHalo;
        float a[3], b[3], d[3];
        pix3(Pa, W, H, x0 + c, y0 + r, a);
        pix3(Pb, W, H, x0 + c, y0 + r, b);
        pix3(Pc, W, H, x0 + c, y0 + r, d);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            sp[0][ch][r][c] = a[ch];
            sp[1][ch][r][c] = b[ch];
            sp[2][ch][r][c] = d[ch];
        }
    }
    const int r = tid / kTileS, c = tid - r * kTileS;
    const int px = blockIdx.x * kTileS + c, py = blockIdx.y * kTileS + r;
    float g[3][3];
    for (int ch = 0; ch < 3; ++ch) {
        __syncthreads();
        for (int i = tid; i < kHalo * kTileS; i += 256) {
            const int hr = i / kTileS, hc = i - hr * kTileS;
            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const float w = win.w[k];
                a0 = fmaf(w, sp[0][ch][hr][hc + k], a0);
                a1 = fmaf(w, sp[1][ch][hr][hc + k], a1);
                a2 = fmaf(w, sp[2][ch][hr][hc + k], a2);
            }
            h[0][hr][hc] = a0; h[1][hr][hc] = a1; h[2][hr][hc] = a2;
        }
        __syncthreads();
        float ga = 0.0f, gb = 0.0f, gc = 0.0f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) {
            const float w = win.w[k];
            ga = fmaf(w, h[0][r + k][c], ga);
            gb = fmaf(w, h[1][r + k][c], gb);
            gc = fmaf(w, h[2][r + k][c], gc);
        }
        g[ch][0] = ga; g[ch][1] = gb; g[ch][2] = gc;
    }
    if (px >= W || py >= H) return;
    const int64_t o = 3 * ((int64_t)py * W + px);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
        dx[o + ch] = gscale * (g[ch][0] + 2.0f * x[o + ch] * g[ch][1] + y[o + ch] * g[ch][2]);
}

}  // namespace

size_t ssim_partials(int W, int H) { return (size_t)((W + kTileS - 1) / kTileS) * ((H + kTileS - 1) / kTileS); }

hipError_t launch_dssim(const float* x, const float* y, int W, int H, float weight, float* loss, float* dx, float* Pa,
                        float* Pb, float* Pc, double* partial, hipStream_t s) {
    const SsimWin win = ssim_window();
    const dim3 grid((W + kTileS - 1) / kTileS, (H + kTileS - 1) / kTileS, 1);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x, y, W, H, win, Pa, Pb, Pc, partial);
    const double n = 3.0 * (double)W * (double)H;
    hipLaunchKernelGGL(k_ssim_total, dim3(1), dim3(1024), 0, s, partial, (int)ssim_partials(W, H), 1.0 / n, weight,
                       loss);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, W, H, win, Pa, Pb, Pc, (float)(-(double)weight / n),
                       dx);
    return hipGetLastError();
}

}  // namespace gs
