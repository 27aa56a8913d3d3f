// Appearance transform module (§3.5.1) -- gfx950, FP32 matrix cores.
//
// Per Gaussian i: x = (g_i / |g_i|, e / |e|) (16 + 32 values; norms floored
// at 1e-12), h = ReLU(W1 x + b1) (32), y = sigmoid(W2 h + b2) (4) = colour
// offsets (dc_r, dc_g, dc_b) and opacity offset do.  The image half of W1 x
// is the same for every Gaussian, so each workgroup folds it into the bias
// u = b1 + W1[:, 16:] e_hat once.
//
// The per-Gaussian layers are dense contractions and run on
// v_mfma_f32_16x16x4_f32 (A: lane l holds A[l % 16][l / 16]; B: B[l / 16][l % 16];
// D: lane l, register r holds D[4 (l / 16) + r][l % 16]).  A wave takes 64
// Gaussians as four groups of 16; lane (q = l / 16, j = l % 16) of group ni
// holds Gaussian 16 ni + j and reads its embedding words 4q .. 4q + 3 as one
// float4 (64 lanes = 16 rows of 64 bytes, contiguous).  The hidden layer is
// computed transposed, H^T = W1g x^T: the K index of step kk on lane group q
// is embedding word 4q + kk, so the B operand is the lane's own float4 and the
// result leaves lane (q, j) with hidden units 16 mi + 4q + r of Gaussian j.
// Sums over the hidden units take those values directly as B operands (the
// order of a contraction's K index is free), so the output layer, the
// backward of the output layer and the embedding gradient need no
// transposes.  Only the weight gradient dW1g = dA^T x_g, whose K index is the
// Gaussian, goes through LDS.
//
// The forward writes the offsets (16 B per Gaussian) and per-workgroup sums
// of do; the backward reads the embedding, the saved offsets and their
// gradients, writes the embedding gradient and keeps the weight gradients in
// registers over a grid-stride loop, then adds workgroup partials in a fixed
// order (deterministic).  Bound by HBM (80 B / 144 B per Gaussian) and the
// FP32 matrix rate (64 / 104 MFMA per 64 Gaussians).
#include <atomic>

#include "gs_internal.h"

namespace gs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kGE = GS_APP_GAUSS_DIM;     // 16
constexpr int kIE = GS_APP_IMAGE_DIM;     // 32
constexpr int kHid = GS_APP_HIDDEN;       // 32
constexpr int kOut = GS_APP_OUT;          // 4
constexpr int kIn = kGE + kIE;            // 48
constexpr int kAT = 256;                  // threads per workgroup, 4 waves
constexpr int kMaxBlocks = 2048;          // cap of the resident grids
constexpr float kNormEps = 1e-12f;
// per-workgroup partial of the backward: dW1g [32][16], db1 [32], dW2 [4][32], db2 [4]
constexpr int kPW1 = 0, kPB1 = kHid * kGE, kPW2 = kPB1 + kHid, kPB2 = kPW2 + kOut * kHid, kPart = kPB2 + kOut;

static_assert(kGE == 16 && kIE == 32 && kHid == 32 && kOut == 4, "tile mapping assumes 16/32/32/4");

__device__ __forceinline__ f4v mfma(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// fast exp and divide: a few ulp, far inside the offsets' float32 bar
__device__ __forceinline__ float sigmoid(float z) { return __fdividef(1.0f, 1.0f + __expf(-z)); }

// normalised image embedding (s_eh) and u = b1 + W1[:, 16:] e_hat (s_u);
// wave 0 computes, the workgroup waits
__device__ __forceinline__ void image_bias(const float* __restrict__ iemb, const AppMlp& w, float* s_eh,
                                           float* s_u) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        const float v = tid < kIE ? iemb[tid] : 0.0f;
        float ss = v * v;
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);   // within each half
        if (tid < kIE) s_eh[tid] = v / fmaxf(sqrtf(ss), kNormEps);
    }
    __syncthreads();
    if (tid < kHid) {
        float u = w.b1[tid];
        for (int k = 0; k < kIE; ++k) u = fmaf(w.w1[tid * kIn + kGE + k], s_eh[k], u);
        s_u[tid] = u;
    }
    __syncthreads();
}

// embedding float4 of lane (q, j) for Gaussian gi, normalised over the
// Gaussian's 4 lanes; returns 1 / max(|g|, eps) and whether |g| > eps
__device__ __forceinline__ float load_unit(const float* __restrict__ gemb, int64_t gi, int64_t n, int q,
                                           float eh[4], bool& above) {
    float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (gi < n) e = reinterpret_cast<const float4*>(gemb)[gi * 4 + q];
    float ss = e.x * e.x + e.y * e.y + e.z * e.z + e.w * e.w;
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    above = ss > kNormEps * kNormEps;
    const float inv = rsqrtf(fmaxf(ss, kNormEps * kNormEps));    // 1 / max(|g|, eps)
    eh[0] = e.x * inv; eh[1] = e.y * inv; eh[2] = e.z * inv; eh[3] = e.w * inv;
    return inv;
}

__device__ __forceinline__ float block_sum(float v, float* s_red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    return s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ __launch_bounds__(kAT) void k_app_fwd(const float* __restrict__ gemb, int64_t n,
                                                 const float* __restrict__ iemb, AppMlp w, float4* __restrict__ out,
                                                 float* __restrict__ part_do) {
    __shared__ float s_eh[kIE], s_u[kHid], s_red[4];
    image_bias(iemb, w, s_eh, s_u);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, q = lane >> 4;
    float aw1[2][4], aw2[2][4], ub[2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            aw1[mi][r] = w.w1[(16 * mi + j) * kIn + 4 * q + r];                    // W1g[16mi + j][4q + r]
            // output o goes to row 4 o of the product, i.e. register 0 of lane group o
            aw2[mi][r] = (j & 3) == 0 ? w.w2[(j >> 2) * kHid + 16 * mi + 4 * q + r] : 0.0f;
            ub[mi][r] = s_u[16 * mi + 4 * q + r];
        }
    const float b2q = w.b2[q];
    float sum_do = 0.0f;
    const int64_t n_chunks = (n + 63) / 64;
    for (int64_t c = (int64_t)blockIdx.x * 4 + wv; c < n_chunks; c += (int64_t)gridDim.x * 4) {
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int64_t gi = c * 64 + 16 * ni + j;
            float eh[4];
            bool above;
            load_unit(gemb, gi, n, q, eh, above);
            f4v h0 = {0.0f, 0.0f, 0.0f, 0.0f}, h1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                h0 = mfma(aw1[0][kk], eh[kk], h0);
                h1 = mfma(aw1[1][kk], eh[kk], h1);
            }
            // two independent accumulation chains over the hidden units
            f4v z0 = {0.0f, 0.0f, 0.0f, 0.0f}, z1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                z0 = mfma(aw2[0][r], fmaxf(h0[r] + ub[0][r], 0.0f), z0);
                z1 = mfma(aw2[1][r], fmaxf(h1[r] + ub[1][r], 0.0f), z1);
            }
            // output q of Gaussian j sits in register 0 of lane (q, j): one
            // sigmoid per lane, and the wave stores 16 rows of 16 bytes
            if (gi < n) {
                const float y = sigmoid(z0[0] + z1[0] + b2q);
                reinterpret_cast<float*>(out)[gi * 4 + q] = y;
                if (q == 3) sum_do += y;
            }
        }
    }
    const float tot = block_sum(sum_do, s_red);
    if (threadIdx.x == 0 && part_do) part_do[blockIdx.x] = tot;
}

// reg_value = reg_weight * (sum of the partials) / n, in a fixed order
__global__ __launch_bounds__(256) void k_app_reg_total(const float* __restrict__ part_do, int blocks, int64_t n,
                                                       float reg_weight, float* __restrict__ reg_value) {
    __shared__ double s[256];
    double a = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) a += (double)part_do[b];
    s[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 256; ++i) t += s[i];
        reg_value[0] = n > 0 ? (float)((double)reg_weight * t / (double)n) : 0.0f;
    }
}

__global__ __launch_bounds__(kAT) void k_app_bwd(const float* __restrict__ gemb, int64_t n,
                                                 const float* __restrict__ iemb, AppMlp w,
                                                 const float* __restrict__ y_in, const float* __restrict__ dy_in,
                                                 const float* __restrict__ d_reg, float reg_weight,
                                                 float4* __restrict__ d_gemb, float* __restrict__ partial) {
    __shared__ float s_eh[kIE], s_u[kHid];
    __shared__ float s_da[4][64][kHid + 1];   // per wave: dA [Gaussian][hidden]
    __shared__ float s_x[4][64][kGE + 1];     // per wave: x_g [Gaussian][word]
    image_bias(iemb, w, s_eh, s_u);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, q = lane >> 4;
    float aw1[2][4], ub[2][4], adh[2], ade[2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        adh[mi] = w.w2[q * kHid + 16 * mi + j];                                     // W2^T[16mi + j][q]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            aw1[mi][r] = w.w1[(16 * mi + j) * kIn + 4 * q + r];                     // W1g[16mi + j][4q + r]
            ade[mi][r] = w.w1[(16 * mi + 4 * q + r) * kIn + j];                     // W1g^T[j][16mi + 4q + r]
            ub[mi][r] = s_u[16 * mi + 4 * q + r];
        }
    }
    // gradient of reg_weight * mean(do) added to every d(do)
    const float reg_add = (d_reg && n > 0) ? d_reg[0] * reg_weight / (float)n : 0.0f;

    f4v acc_w1[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    float acc_b1[2][4] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
    float acc_w2[4][2][4];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc_w2[o][mi][r] = 0.0f;
    float acc_b2 = 0.0f;

    const int64_t n_chunks = (n + 63) / 64;
    for (int64_t c = (int64_t)blockIdx.x * 4 + wv; c < n_chunks; c += (int64_t)gridDim.x * 4) {
#pragma unroll 1
        for (int ni = 0; ni < 4; ++ni) {
            const int64_t gi = c * 64 + 16 * ni + j;
            const bool valid = gi < n;
            float eh[4];
            bool above;
            const float inv = load_unit(gemb, gi, n, q, eh, above);
#pragma unroll
            for (int r = 0; r < 4; ++r) s_x[wv][16 * ni + j][4 * q + r] = eh[r];
            f4v a0 = {0.0f, 0.0f, 0.0f, 0.0f}, a1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                a0 = mfma(aw1[0][kk], eh[kk], a0);
                a1 = mfma(aw1[1][kk], eh[kk], a1);
            }
            // output q of Gaussian j: dz = dy y (1 - y)
            // (the regulariser's share, ~1/n, is kept out of the sum with dy,
            // where float32 would drop it)
            float dz = 0.0f;
            if (valid) {
                const float yv = y_in[gi * 4 + q];
                const float sg = yv * (1.0f - yv);
                dz = fmaf(q == 3 ? reg_add : 0.0f, sg, dy_in[gi * 4 + q] * sg);
            }
            acc_b2 += dz;
            float dzo[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) dzo[o] = __shfl(dz, 16 * o + j, 64);
            // dh^T = W2^T dz^T: one K step (K = the 4 outputs)
            const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
            const f4v dh0 = mfma(adh[0], dz, zero), dh1 = mfma(adh[1], dz, zero);
            float da[2][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float p0 = a0[r] + ub[0][r], p1 = a1[r] + ub[1][r];
                const float h0 = fmaxf(p0, 0.0f), h1 = fmaxf(p1, 0.0f);
                da[0][r] = p0 > 0.0f ? dh0[r] : 0.0f;
                da[1][r] = p1 > 0.0f ? dh1[r] : 0.0f;
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    acc_w2[o][0][r] = fmaf(dzo[o], h0, acc_w2[o][0][r]);
                    acc_w2[o][1][r] = fmaf(dzo[o], h1, acc_w2[o][1][r]);
                }
                acc_b1[0][r] += da[0][r];
                acc_b1[1][r] += da[1][r];
                s_da[wv][16 * ni + j][4 * q + r] = da[0][r];
                s_da[wv][16 * ni + j][16 + 4 * q + r] = da[1][r];
            }
            // dx_g^T = W1g^T dA^T (K = hidden, taken in the lane's own order)
            f4v dx = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r = 0; r < 4; ++r) dx = mfma(ade[0][r], da[0][r], dx);
#pragma unroll
            for (int r = 0; r < 4; ++r) dx = mfma(ade[1][r], da[1][r], dx);
            // through g / max(|g|, eps)
            float dot = eh[0] * dx[0] + eh[1] * dx[1] + eh[2] * dx[2] + eh[3] * dx[3];
            dot += __shfl_xor(dot, 16, 64);
            dot += __shfl_xor(dot, 32, 64);
            if (!above) dot = 0.0f;
            if (valid)
                d_gemb[gi * 4 + q] = make_float4((dx[0] - eh[0] * dot) * inv, (dx[1] - eh[1] * dot) * inv,
                                                 (dx[2] - eh[2] * dot) * inv, (dx[3] - eh[3] * dot) * inv);
        }
        // dW1g += dA^T x_g over the chunk's 64 Gaussians (K = Gaussian)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
        for (int s = 0; s < 16; ++s) {
            const float xv = s_x[wv][4 * s + q][j];
            acc_w1[0] = mfma(s_da[wv][4 * s + q][j], xv, acc_w1[0]);
            acc_w1[1] = mfma(s_da[wv][4 * s + q][16 + j], xv, acc_w1[1]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // sums over the 16 Gaussians of a lane row (j), fixed butterfly order
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc_b1[mi][r] += __shfl_xor(acc_b1[mi][r], off, 64);
#pragma unroll
                for (int o = 0; o < 4; ++o) acc_w2[o][mi][r] += __shfl_xor(acc_w2[o][mi][r], off, 64);
            }
        acc_b2 += __shfl_xor(acc_b2, off, 64);
    }
    // per-wave results into LDS (reusing s_da), then the 4 waves in order
    __syncthreads();
    float* s_part = &s_da[0][0][0];      // [4][kPart] fits in s_da
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_part[wv * kPart + kPW1 + (16 * mi + 4 * q + r) * kGE + j] = acc_w1[mi][r];
    if (j == 0) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int hid = 16 * mi + 4 * q + r;
                s_part[wv * kPart + kPB1 + hid] = acc_b1[mi][r];
#pragma unroll
                for (int o = 0; o < 4; ++o) s_part[wv * kPart + kPW2 + o * kHid + hid] = acc_w2[o][mi][r];
            }
        s_part[wv * kPart + kPB2 + q] = acc_b2;
    }
    __syncthreads();
    // column-major [kPart][gridDim.x], so that each total reads one contiguous run
    for (int i = threadIdx.x; i < kPart; i += kAT)
        partial[(size_t)i * gridDim.x + blockIdx.x] =
            ((s_part[i] + s_part[kPart + i]) + s_part[2 * kPart + i]) + s_part[3 * kPart + i];
}

// tot[c] = sum over workgroups of partial column c (one wave per column,
// double, fixed order)
__global__ __launch_bounds__(64) void k_app_colsum(const float* __restrict__ partial, int blocks,
                                                   double* __restrict__ tot) {
    const int c = blockIdx.x, lane = threadIdx.x;
    double a = 0.0;
    for (int b = lane; b < blocks; b += 64) a += (double)partial[(size_t)c * blocks + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) tot[c] = a;
}

// weight and image-embedding gradients from the column totals (zero when
// there were no Gaussians)
__global__ __launch_bounds__(1024) void k_app_bwd_final(const double* __restrict__ tot, int have,
                                                        const float* __restrict__ iemb, AppMlp w, AppGrad g) {
    __shared__ double s_tot[kPart];
    __shared__ float s_eh[kIE], s_de[kIE];
    __shared__ float s_den;
    __shared__ int s_above;
    const int t = threadIdx.x;
    if (t < kPart) s_tot[t] = have ? tot[t] : 0.0;
    if (t == 0) {
        double ss = 0.0;
        for (int k = 0; k < kIE; ++k) ss += (double)iemb[k] * (double)iemb[k];
        const float nrm = (float)sqrt(ss);
        s_den = fmaxf(nrm, kNormEps);
        s_above = nrm > kNormEps;
    }
    __syncthreads();
    if (t < kIE) s_eh[t] = iemb[t] / s_den;
    __syncthreads();
    if (t < kHid * kGE) g.d_w1[(t / kGE) * kIn + (t % kGE)] = (float)s_tot[kPW1 + t];
    if (t < kHid * kIE) {
        const int hid = t / kIE, k = t % kIE;
        g.d_w1[hid * kIn + kGE + k] = (float)(s_tot[kPB1 + hid] * (double)s_eh[k]);
    }
    if (t < kHid) g.d_b1[t] = (float)s_tot[kPB1 + t];
    if (t < kOut * kHid) g.d_w2[t] = (float)s_tot[kPW2 + t];
    if (t < kOut) g.d_b2[t] = (float)s_tot[kPB2 + t];
    if (t < kIE) {
        double de = 0.0;
        for (int hid = 0; hid < kHid; ++hid) de += (double)w.w1[hid * kIn + kGE + t] * s_tot[kPB1 + hid];
        s_de[t] = (float)de;
    }
    __syncthreads();
    if (t < kIE && g.d_iemb) {
        double dot = 0.0;
        if (s_above)
            for (int k = 0; k < kIE; ++k) dot += (double)s_eh[k] * (double)s_de[k];
        g.d_iemb[t] = (float)(((double)s_de[t] - (double)s_eh[t] * dot) / (double)s_den);
    }
}

// as many workgroups of `kernel` as the device holds at once (at most
// kMaxBlocks), but no more than the n Gaussians need; a grid-stride loop
// gives each wave several chunks (the backward keeps its weight-gradient
// registers over them)
template <class K>
int resident_blocks(K kernel, std::atomic<int>* cache, int64_t n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int res = cache[dev].load(std::memory_order_relaxed);
    if (res <= 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kAT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        res = per_cu * cus;
        res = res > kMaxBlocks ? kMaxBlocks : res;
        cache[dev].store(res, std::memory_order_relaxed);
    }
    const int64_t need = ((n + 63) / 64 + 3) / 4;
    return (int)(need < 1 ? 1 : (need < res ? need : res));
}

std::atomic<int> g_fwd_blocks[64], g_bwd_blocks[64];

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t app_workspace_bytes(int64_t) {
    return align256((size_t)kMaxBlocks * kPart * sizeof(float)) + kPart * sizeof(double);
}

hipError_t launch_app_fwd(const float* gemb, int64_t n, const float* iemb, const AppMlp& w, float reg_weight,
                          float* offsets, float* reg_value, void* ws, hipStream_t s) {
    const int blocks = resident_blocks(k_app_fwd, g_fwd_blocks, n);
    float* part_do = static_cast<float*>(ws);
    if (n > 0)
        hipLaunchKernelGGL(k_app_fwd, dim3(blocks), dim3(kAT), 0, s, gemb, n, iemb, w,
                           reinterpret_cast<float4*>(offsets), part_do);
    if (reg_value)
        hipLaunchKernelGGL(k_app_reg_total, dim3(1), dim3(256), 0, s, part_do, n > 0 ? blocks : 0, n, reg_weight,
                           reg_value);
    return hipGetLastError();
}

hipError_t launch_app_bwd(const float* gemb, int64_t n, const float* iemb, const AppMlp& w, const float* offsets,
                          const float* d_offsets, const float* d_reg, float reg_weight, float* d_gemb,
                          const AppGrad& g, void* ws, hipStream_t s) {
    const int blocks = resident_blocks(k_app_bwd, g_bwd_blocks, n);
    float* partial = static_cast<float*>(ws);
    double* tot = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                            align256((size_t)kMaxBlocks * kPart * sizeof(float)));
    if (n > 0) {
        hipLaunchKernelGGL(k_app_bwd, dim3(blocks), dim3(kAT), 0, s, gemb, n, iemb, w, offsets, d_offsets, d_reg,
                           reg_weight, reinterpret_cast<float4*>(d_gemb), partial);
        hipLaunchKernelGGL(k_app_colsum, dim3(kPart), dim3(64), 0, s, partial, blocks, tot);
    }
    hipLaunchKernelGGL(k_app_bwd_final, dim3(1), dim3(1024), 0, s, tot, n > 0 ? 1 : 0, iemb, w, g);
    return hipGetLastError();
}

}  // namespace gs
