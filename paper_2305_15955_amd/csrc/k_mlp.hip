// Learned QP-root seed: MLP 8 -> 64 -> 64 -> 1 (tanh), FP32, with hand-written
// forward, backward (mean squared error) and Adam kernels.
// Parameter layout: W1[64][8], b1[64], W2[64][64], b2[64], W3[1][64], b3[1].
#include "common.h"
#include "kernels.h"

namespace cdwac {

constexpr int kIn = 8, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH;
static_assert(oB3 + 1 == kMlpParams, "parameter count");

// One thread per sample; parameters staged in LDS.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ theta, int n,
                                                     const float* __restrict__ x, float* __restrict__ y) {
    __shared__ float th[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += 256) th[i] = theta[i];
    __syncthreads();
    int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float xi[kIn];
#pragma unroll
    for (int i = 0; i < kIn; ++i) xi[i] = x[(int64_t)s * kIn + i];
    float h1[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = th[oB1 + o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a += th[oW1 + o * kIn + i] * xi[i];
        h1[o] = tanhf(a);
    }
    float out = th[oB3];
    for (int o = 0; o < kH; ++o) {
        float a = th[oB2 + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) a += th[oW2 + o * kH + i] * h1[i];
        out += th[oW3 + o] * tanhf(a);
    }
    y[s] = out;
}

// Gradient of L = (1/n) sum (y - t)^2 over a chunk of 32 samples per block,
// written as one partial gradient per block (reduced deterministically).
constexpr int kChunk = 32;

__global__ __launch_bounds__(256) void k_mlp_grad_partial(const float* __restrict__ theta, int n,
                                                          const float* __restrict__ x,
                                                          const float* __restrict__ t,
                                                          float* __restrict__ partial,
                                                          float* __restrict__ loss_partial) {
    __shared__ float th[kMlpParams];
    __shared__ float X[kChunk][kIn];
    __shared__ float H1[kChunk][kH + 1], H2[kChunk][kH + 1], D2[kChunk][kH + 1], D1[kChunk][kH + 1];
    __shared__ float dy[kChunk], r2[kChunk];
    for (int i = threadIdx.x; i < kMlpParams; i += 256) th[i] = theta[i];
    const int s0 = blockIdx.x * kChunk;
    const int sl = threadIdx.x & (kChunk - 1), part = threadIdx.x / kChunk;   // 8 parts of 8 units
    const int s = s0 + sl;
    const bool valid = s < n;
    if (part == 0) {
#pragma unroll
        for (int i = 0; i < kIn; ++i) X[sl][i] = valid ? x[(int64_t)s * kIn + i] : 0.0f;
    }
    __syncthreads();
    for (int o = part * 8; o < part * 8 + 8; ++o) {
        float a = th[oB1 + o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a += th[oW1 + o * kIn + i] * X[sl][i];
        H1[sl][o] = tanhf(a);
    }
    __syncthreads();
    for (int o = part * 8; o < part * 8 + 8; ++o) {
        float a = th[oB2 + o];
        for (int i = 0; i < kH; ++i) a += th[oW2 + o * kH + i] * H1[sl][i];
        H2[sl][o] = tanhf(a);
    }
    __syncthreads();
    if (part == 0) {
        float yv = th[oB3];
        for (int i = 0; i < kH; ++i) yv += th[oW3 + i] * H2[sl][i];
        float r = valid ? yv - t[s] : 0.0f;
        dy[sl] = 2.0f * r / (float)n;
        r2[sl] = r * r;
    }
    __syncthreads();
    for (int o = part * 8; o < part * 8 + 8; ++o) {
        float h = H2[sl][o];
        D2[sl][o] = dy[sl] * th[oW3 + o] * (1.0f - h * h);
    }
    __syncthreads();
    for (int o = part * 8; o < part * 8 + 8; ++o) {
        float a = 0.0f;
        for (int q = 0; q < kH; ++q) a += th[oW2 + q * kH + o] * D2[sl][q];
        float h = H1[sl][o];
        D1[sl][o] = a * (1.0f - h * h);
    }
    __syncthreads();
    float* g = partial + (int64_t)blockIdx.x * kMlpParams;
    // dW2[o][i] = sum_s D2[s][o] H1[s][i]
    for (int e = threadIdx.x; e < kH * kH; e += 256) {
        int o = e / kH, i = e % kH;
        float a = 0.0f;
        for (int q = 0; q < kChunk; ++q) a += D2[q][o] * H1[q][i];
        g[oW2 + e] = a;
    }
    for (int e = threadIdx.x; e < kH * kIn; e += 256) {
        int o = e / kIn, i = e % kIn;
        float a = 0.0f;
        for (int q = 0; q < kChunk; ++q) a += D1[q][o] * X[q][i];
        g[oW1 + e] = a;
    }
    if (threadIdx.x < kH) {
        int o = threadIdx.x;
        float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
        for (int q = 0; q < kChunk; ++q) {
            a1 += D1[q][o];
            a2 += D2[q][o];
            a3 += dy[q] * H2[q][o];
        }
        g[oB1 + o] = a1;
        g[oB2 + o] = a2;
        g[oW3 + o] = a3;
    }
    if (threadIdx.x == 0) {
        float a = 0.0f, l = 0.0f;
        for (int q = 0; q < kChunk; ++q) {
            a += dy[q];
            l += r2[q];
        }
        g[oB3] = a;
        loss_partial[blockIdx.x] = l / (float)n;
    }
}

__global__ void k_mlp_reduce(const float* __restrict__ partial, const float* __restrict__ loss_partial,
                             int nb, float* __restrict__ grad, float* __restrict__ loss) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float a = 0.0f;
        for (int b = 0; b < nb; ++b) a += partial[(int64_t)b * kMlpParams + p];
        grad[p] = a;
    }
    if (p == 0 && loss) {
        float l = 0.0f;
        for (int b = 0; b < nb; ++b) l += loss_partial[b];
        loss[0] = l;
    }
}

__global__ void k_mlp_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, float c1, float c2, float lr, float b1, float b2, float eps) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float g = grad[p];
    float mm = b1 * m[p] + (1.0f - b1) * g;
    float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    float mh = mm / c1, vh = vv / c2;
    theta[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_mlp_gather(const float* __restrict__ x, const float* __restrict__ t,
                             const int* __restrict__ idx, int n, float* __restrict__ xb,
                             float* __restrict__ tb) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = idx[i];
#pragma unroll
    for (int q = 0; q < kIn; ++q) xb[(int64_t)i * kIn + q] = x[(int64_t)j * kIn + q];
    tb[i] = t[j];
}

int mlp_grad_blocks(int n) { return (n + kChunk - 1) / kChunk; }

void launch_mlp_forward(hipStream_t s, const float* theta, int n, const float* x, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, theta, n, x, y);
}

void launch_mlp_grad(hipStream_t s, const float* theta, int n, const float* x, const float* t, float* partial,
                     float* loss_partial, float* grad, float* loss) {
    int nb = mlp_grad_blocks(n);
    hipLaunchKernelGGL(k_mlp_grad_partial, dim3(nb), dim3(256), 0, s, theta, n, x, t, partial, loss_partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, loss_partial, nb,
                       grad, loss);
}

void launch_mlp_adam(hipStream_t s, float* theta, const float* grad, float* m, float* v, int step, float lr,
                     float b1, float b2, float eps) {
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, theta, grad, m, v, c1, c2, lr,
                       b1, b2, eps);
}

void launch_mlp_gather(hipStream_t s, const float* x, const float* t, const int* idx, int n, float* xb,
                       float* tb) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_gather, dim3((n + 255) / 256), dim3(256), 0, s, x, t, idx, n, xb, tb);
}

}  // namespace cdwac
