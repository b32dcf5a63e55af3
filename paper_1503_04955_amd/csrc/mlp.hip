// Learned parameter selector: an FP32 multilayer perceptron 3 -> 64 -> 64 -> K (ReLU), whose K
// outputs predict the log of the run time of each candidate parameter tuple.  Forward, backward
// (per-sample gradients reduced in a fixed order, so results are deterministic) and Adam update
// are hand-written kernels; one wavefront (64 lanes) handles one sample, lane i owning hidden
// unit i.
//
// Parameter layout (floats): W1[64][3], b1[64], W2[64][64], b2[64], W3[K][64], b3[K].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dkss.h"
#include "hip_status.hpp"

namespace {

constexpr int kIn = DKSS_MLP_IN, kHid = DKSS_MLP_HID, kOut = DKSS_MLP_OUT;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;
static_assert(kParams == DKSS_MLP_NPARAM, "parameter count");
constexpr int kWaves = 4;                     // samples per workgroup of 256 threads

struct Acts {
    float x[kIn];
    float z1, h1, z2, h2;                     // this lane's hidden unit, both layers
    float y;                                  // output (lanes < K)
};

// forward pass of one sample by one wavefront; sh1/sh2: 64 floats of this wave's LDS
__device__ __forceinline__ void mlp_forward_wave(const float* __restrict__ P, const float* __restrict__ xs,
                                                 float* sh1, float* sh2, int lane, Acts* A) {
#pragma unroll
    for (int c = 0; c < kIn; ++c) A->x[c] = xs[c];
    float z = P[oB1 + lane];
#pragma unroll
    for (int c = 0; c < kIn; ++c) z += P[oW1 + lane * kIn + c] * A->x[c];
    A->z1 = z;
    A->h1 = z > 0.f ? z : 0.f;
    sh1[lane] = A->h1;
    __syncthreads();
    z = P[oB2 + lane];
    for (int j = 0; j < kHid; ++j) z += P[oW2 + lane * kHid + j] * sh1[j];
    A->z2 = z;
    A->h2 = z > 0.f ? z : 0.f;
    sh2[lane] = A->h2;
    __syncthreads();
    A->y = 0.f;
    if (lane < kOut) {
        float y = P[oB3 + lane];
        for (int j = 0; j < kHid; ++j) y += P[oW3 + lane * kHid + j] * sh2[j];
        A->y = y;
    }
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X,
                                                     int n, float* __restrict__ Y) {
    __shared__ float sh[kWaves][2][kHid];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * kWaves + wave;
    const int sc = s < n ? s : n - 1;         // every wave runs (barriers); only valid ones write
    Acts A;
    mlp_forward_wave(P, X + (size_t)sc * kIn, sh[wave][0], sh[wave][1], lane, &A);
    if (s < n && lane < kOut) Y[(size_t)s * kOut + lane] = A.y;
}

// Per-sample gradient of L = (1/msum) sum_n sum_k mask_nk (y_nk - t_nk)^2 into G[s][P], and the
// sample's loss term into Ls[s].
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                  const float* __restrict__ T, const float* __restrict__ Mk,
                                                  int n, float inv_msum, float* __restrict__ G,
                                                  float* __restrict__ Ls) {
    __shared__ float sh[kWaves][4][kHid];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * kWaves + wave;
    const bool valid = s < n;
    const int sc = valid ? s : n - 1;
    float* sh1 = sh[wave][0];
    float* sh2 = sh[wave][1];
    float* sdy = sh[wave][2];
    float* sdz = sh[wave][3];
    Acts A;
    mlp_forward_wave(P, X + (size_t)sc * kIn, sh1, sh2, lane, &A);
    float dy = 0.f, lterm = 0.f;
    if (lane < kOut) {
        const float mk = Mk[(size_t)sc * kOut + lane];
        const float diff = A.y - T[(size_t)sc * kOut + lane];
        dy = 2.f * mk * diff * inv_msum;
        lterm = mk * diff * diff * inv_msum;
    }
    sdy[lane] = dy;
    __syncthreads();
    float* g = G + (size_t)sc * kParams;
    // layer 3
    if (valid) {
        for (int k = 0; k < kOut; ++k) g[oW3 + k * kHid + lane] = sdy[k] * A.h2;
        if (lane < kOut) g[oB3 + lane] = dy;
    }
    float dh2 = 0.f;
    for (int k = 0; k < kOut; ++k) dh2 += P[oW3 + k * kHid + lane] * sdy[k];
    const float dz2 = A.z2 > 0.f ? dh2 : 0.f;
    sdz[lane] = dz2;
    __syncthreads();
    // layer 2
    if (valid) {
        for (int i = 0; i < kHid; ++i) g[oW2 + i * kHid + lane] = sdz[i] * A.h1;
        g[oB2 + lane] = dz2;
    }
    float dh1 = 0.f;
    for (int i = 0; i < kHid; ++i) dh1 += P[oW2 + i * kHid + lane] * sdz[i];
    const float dz1 = A.z1 > 0.f ? dh1 : 0.f;
    if (valid) {
#pragma unroll
        for (int c = 0; c < kIn; ++c) g[oW1 + lane * kIn + c] = dz1 * A.x[c];
        g[oB1 + lane] = dz1;
    }
    // sample loss: sum over the wave's lanes
    sdy[lane] = lterm;
    __syncthreads();
    if (valid && lane == 0) {
        float l = 0.f;
        for (int k = 0; k < kOut; ++k) l += sdy[k];
        Ls[s] = l;
    }
}

// grad[p] = sum_s G[s][p] in sample order; loss = sum_s Ls[s] (thread 0)
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ G, const float* __restrict__ Ls,
                                                    int n, float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float acc = 0.f;
        for (int s = 0; s < n; ++s) acc += G[(size_t)s * kParams + p];
        grad[p] = acc;
    }
    if (p == 0) {
        float l = 0.f;
        for (int s = 0; s < n; ++s) l += Ls[s];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, const float* __restrict__ grad,
                                                  float* __restrict__ m1, float* __restrict__ m2, float lr,
                                                  float b1, float b2, float c1, float c2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.f - b1) * g;
    const float v = b2 * m2[p] + (1.f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    P[p] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
}

}  // namespace

extern "C" {

size_t dkss_mlp_work_floats(int n) { return n > 0 ? (size_t)n * (kParams + 1) : 0; }

int dkss_mlp_forward(const float* params, const float* x, int n, float* y, dkss_stream_t s) {
    if (!params || !x || !y || n <= 0) return DKSS_EINVAL;
    dkss::clear_stale_hip_error();
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + kWaves - 1) / kWaves), dim3(256), 0, (hipStream_t)s, params,
                       x, n, y);
    return dkss::launch_status();
}

int dkss_mlp_loss_grad(const float* params, const float* x, const float* t, const float* mask, int n,
                       float mask_sum, float* grad, float* loss, float* work, dkss_stream_t s) {
    if (!params || !x || !t || !mask || !grad || !loss || !work || n <= 0 || !(mask_sum > 0.f))
        return DKSS_EINVAL;
    dkss::clear_stale_hip_error();
    hipStream_t st = (hipStream_t)s;
    float* G = work;
    float* Ls = work + (size_t)n * kParams;
    hipLaunchKernelGGL(k_mlp_grad, dim3((n + kWaves - 1) / kWaves), dim3(256), 0, st, params, x, t, mask, n,
                       1.f / mask_sum, G, Ls);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, (const float*)G,
                       (const float*)Ls, n, grad, loss);
    return dkss::launch_status();
}

int dkss_mlp_adam(float* params, const float* grad, float* m1, float* m2, int step, float lr,
                  dkss_stream_t s) {
    if (!params || !grad || !m1 || !m2 || step < 1) return DKSS_EINVAL;
    dkss::clear_stale_hip_error();
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f / (1.f - powf(b1, (float)step)), c2 = 1.f / (1.f - powf(b2, (float)step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)s, params, grad,
                       m1, m2, lr, b1, b2, c1, c2, 1e-8f);
    return dkss::launch_status();
}

}  // extern "C"
