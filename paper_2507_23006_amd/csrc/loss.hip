// Training loss and its gradient in one pass -- gfx950.
//
// L = mean over 3 P of |rgb - target| (the L1 term of Eq. 3)
//   + lambda * mean over P of |D / max(alpha, 1e-10) - target_depth|
// (the depth regulariser of §3.5.3 on the expected depth, lambda_d of §3.6),
// with P pixels.  Each thread handles pixels, writes dL/drgb, dL/dD and
// dL/dalpha (the subgradient of |x| is sign(x), 0 at 0; the clamp passes no
// gradient below 1e-10), and the workgroup writes its partial sum; one
// workgroup then adds the partials in a fixed order, so the loss is
// deterministic.  HBM-bound: 36 bytes read and 20 written per pixel.
#include <mutex>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kLossThreads = 256;
constexpr int kLossPerThread = 8;
constexpr int kLossSpan = kLossThreads * kLossPerThread;
// partials of the allocation-free entry point: 32768 doubles (256 KiB) per
// GPU, enough for 2^26 pixels (eight 3840x2160 views)
constexpr int kLossScratchPartials = 32768;
constexpr int kMaxDevices = 64;

__device__ __forceinline__ float sgn(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

__global__ __launch_bounds__(kLossThreads) void k_loss_partial(const float* __restrict__ rgb,
                                                               const float* __restrict__ depth,
                                                               const float* __restrict__ alpha,
                                                               const float* __restrict__ t_rgb,
                                                               const float* __restrict__ t_depth, int64_t n_pix,
                                                               float lambda, float* __restrict__ d_rgb,
                                                               float* __restrict__ d_depth,
                                                               float* __restrict__ d_alpha,
                                                               double* __restrict__ partial) {
    __shared__ double s_sum[kLossThreads / 64];
    const double inv3 = 1.0 / (3.0 * (double)n_pix), inv1 = 1.0 / (double)n_pix;
    const float g_rgb = (float)inv3, g_d = (float)(lambda * inv1);
    double acc = 0.0;
    const int64_t p0 = (int64_t)blockIdx.x * kLossSpan;
#pragma unroll
    for (int i = 0; i < kLossPerThread; ++i) {
        const int64_t p = p0 + i * kLossThreads + threadIdx.x;
        if (p >= n_pix) continue;     // predicated: the items' loads are independent
        float l_rgb = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = rgb[3 * p + c] - t_rgb[3 * p + c];
            l_rgb += fabsf(e);
            d_rgb[3 * p + c] = g_rgb * sgn(e);
        }
        acc += (double)l_rgb * inv3;
        if (t_depth) {
            const float D = depth[p], a = alpha[p];
            const bool clamped = !(a >= 1e-10f);
            const float am = clamped ? 1e-10f : a;
            const float e = D / am - t_depth[p];
            acc += (double)lambda * (double)fabsf(e) * inv1;
            const float s = g_d * sgn(e);
            d_depth[p] = s / am;
            d_alpha[p] = clamped ? 0.0f : -s * D / (am * am);
        } else {
            d_depth[p] = 0.0f;
            d_alpha[p] = 0.0f;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < kLossThreads / 64; ++w) b += s_sum[w];
        partial[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(1024) void k_loss_final(const double* __restrict__ partial, int n, float* __restrict__ loss) {
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
        loss[0] = (float)b;
    }
}

}  // namespace

// Scratch of the allocation-free entry point: the workgroup partials live
// in this file-scope array (one copy per GPU, kept until the process ends)
// instead of a caller workspace.  Host code never passes the array's name
// to a kernel -- on the host it only stands in for the symbol -- but the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kLossScratchPartials];

size_t loss_partials(int64_t n_pix) { return (size_t)((n_pix + kLossSpan - 1) / kLossSpan); }

int64_t loss_scratch_max_pixels() { return (int64_t)kLossScratchPartials * kLossSpan; }

hipError_t loss_scratch_ptr(double** out) {
    static std::mutex mu;
    static double* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double*>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_loss(const float* rgb, const float* depth, const float* alpha, const float* t_rgb,
                       const float* t_depth, int64_t n_pix, float lambda, float* loss, float* d_rgb, float* d_depth,
                       float* d_alpha, double* partial, hipStream_t s) {
    const unsigned blocks = (unsigned)loss_partials(n_pix);
    hipLaunchKernelGGL(k_loss_partial, dim3(blocks), dim3(kLossThreads), 0, s, rgb, depth, alpha, t_rgb, t_depth,
                       n_pix, lambda, d_rgb, d_depth, d_alpha, partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, s, partial, (int)blocks, loss);
    return hipGetLastError();
}

}  // namespace gs
