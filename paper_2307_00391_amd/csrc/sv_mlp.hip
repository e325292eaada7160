// Learned T0: forward, backward and Adam kernels of a 5 -> 64 -> 64 -> 1
// perceptron with exact GELU activations, FP32.
//
// Parameter layout: W1[64][5] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
#include <math.h>
#include <string.h>

#include "sv_device.h"
#include "sv_internal.h"

namespace sv {

constexpr int MI = SV_MLP_IN, MH = SV_MLP_HIDDEN, MP = SV_MLP_PARAMS;
constexpr int OW1 = 0, OB1 = OW1 + MH * MI, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH;
static_assert(OB3 + 1 == MP, "parameter layout");

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// one thread per sample
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X, int B,
                                                     float *__restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B) return;
    float x[MI];
    for (int i = 0; i < MI; ++i) x[i] = X[(size_t)s * MI + i];
    float h1[MH];
    for (int j = 0; j < MH; ++j) {
        float z = P[OB1 + j];
        for (int i = 0; i < MI; ++i) z += P[OW1 + j * MI + i] * x[i];
        h1[j] = gelu(z);
    }
    float out = P[OB3];
    for (int k = 0; k < MH; ++k) {
        float z = P[OB2 + k];
        for (int j = 0; j < MH; ++j) z += P[OW2 + k * MH + j] * h1[j];
        out += P[OW3 + k] * gelu(z);
    }
    y[s] = out;
}

constexpr int SPB = 32;   // samples per block in the gradient kernel

// per-block partial gradient of sum_i (net(X_i) - t_i)^2 / B and of the loss
__global__ __launch_bounds__(64) void k_mlp_grad_partial(const float *__restrict__ P, const float *__restrict__ X,
                                                         const float *__restrict__ t, int B,
                                                         float *__restrict__ gpart, float *__restrict__ lpart) {
    __shared__ float xs[SPB][MI];
    __shared__ float h1[SPB][MH], g1[SPB][MH];   // g1: gelu'(z1), then d1
    __shared__ float h2[SPB][MH], g2[SPB][MH];   // g2: gelu'(z2), then d2
    __shared__ float d3[SPB], ls[SPB];
    const int s0 = blockIdx.x * SPB;
    const int ns = min(SPB, B - s0);
    const float invB = 1.0f / (float)B;
    // forward: thread j handles hidden unit j for every sample of the block
    for (int e = threadIdx.x; e < SPB * MI; e += blockDim.x) {
        const int s = e / MI, i = e % MI;
        xs[s][i] = s < ns ? X[(size_t)(s0 + s) * MI + i] : 0.f;
    }
    __syncthreads();
    for (int s = 0; s < ns; ++s)
        for (int j = threadIdx.x; j < MH; j += blockDim.x) {
            float z = P[OB1 + j];
            for (int i = 0; i < MI; ++i) z += P[OW1 + j * MI + i] * xs[s][i];
            h1[s][j] = gelu(z);
            g1[s][j] = gelu_d(z);
        }
    __syncthreads();
    for (int s = 0; s < ns; ++s)
        for (int k = threadIdx.x; k < MH; k += blockDim.x) {
            float z = P[OB2 + k];
            for (int j = 0; j < MH; ++j) z += P[OW2 + k * MH + j] * h1[s][j];
            h2[s][k] = gelu(z);
            g2[s][k] = gelu_d(z);
        }
    __syncthreads();
    if (threadIdx.x < SPB) {
        const int s = threadIdx.x;
        float d = 0.f, l = 0.f;
        if (s < ns) {
            float out = P[OB3];
            for (int k = 0; k < MH; ++k) out += P[OW3 + k] * h2[s][k];
            const float r = out - t[s0 + s];
            d = 2.0f * r * invB;
            l = r * r * invB;
        }
        d3[s] = d;
        ls[s] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {   // the block's loss, summed in sample order
        float l = 0.f;
        for (int s = 0; s < ns; ++s) l += ls[s];
        lpart[blockIdx.x] = l;
    }
    // backward through layer 3 and GELU 2
    for (int s = 0; s < ns; ++s)
        for (int k = threadIdx.x; k < MH; k += blockDim.x) g2[s][k] = d3[s] * P[OW3 + k] * g2[s][k];
    __syncthreads();
    // backward through layer 2 and GELU 1
    for (int s = 0; s < ns; ++s)
        for (int j = threadIdx.x; j < MH; j += blockDim.x) {
            float a = 0.f;
            for (int k = 0; k < MH; ++k) a += g2[s][k] * P[OW2 + k * MH + j];
            g1[s][j] = a * g1[s][j];
        }
    __syncthreads();
    // parameter gradients of this block (sums over its samples, fixed order)
    float *G = gpart + (size_t)blockIdx.x * MP;
    for (int p = threadIdx.x; p < MP; p += blockDim.x) {
        float a = 0.f;
        if (p < OB1) {
            const int j = p / MI, i = p % MI;
            for (int s = 0; s < ns; ++s) a += g1[s][j] * xs[s][i];
        } else if (p < OW2) {
            const int j = p - OB1;
            for (int s = 0; s < ns; ++s) a += g1[s][j];
        } else if (p < OB2) {
            const int k = (p - OW2) / MH, j = (p - OW2) % MH;
            for (int s = 0; s < ns; ++s) a += g2[s][k] * h1[s][j];
        } else if (p < OW3) {
            const int k = p - OB2;
            for (int s = 0; s < ns; ++s) a += g2[s][k];
        } else if (p < OB3) {
            const int k = p - OW3;
            for (int s = 0; s < ns; ++s) a += d3[s] * h2[s][k];
        } else {
            for (int s = 0; s < ns; ++s) a += d3[s];
        }
        G[p] = a;
    }
}

// grad[p] = sum over blocks of gpart[b][p] (fixed order); loss = sum of the block losses
__global__ void k_mlp_grad_reduce(const float *__restrict__ gpart, int nb, const float *__restrict__ lpart,
                                  float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MP) {
        float a = 0.f;
        for (int b = 0; b < nb; ++b) a += gpart[(size_t)b * MP + p];
        grad[p] = a;
    }
    if (p == 0) {
        double l = 0.0;
        for (int b = 0; b < nb; ++b) l += lpart[b];
        loss[0] = (float)l;
    }
}

__global__ void k_mlp_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace sv

using namespace sv;

extern "C" {

sv_status sv_mlp_forward(const float *params, const float *X, int B, float *y, void *hip_stream) {
    clear_error();
    if (!params || B < 0) return fail(SV_EINVAL, "bad MLP forward arguments");
    if (!B) return SV_OK;   // X and y may be NULL for an empty batch
    if (!X || !y) return fail(SV_EINVAL, "bad MLP forward arguments");
    hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, params, X, B, y);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

sv_status sv_mlp_backward(const float *params, const float *X, const float *t, int B, float *grad, float *loss,
                          void *hip_stream) {
    clear_error();
    if (!params || !X || !t || !grad || !loss || B < 1) return fail(SV_EINVAL, "bad MLP backward arguments");
    const hipStream_t st = (hipStream_t)hip_stream;
    const int nb = (B + SPB - 1) / SPB;
    void *ws = nullptr;
    SV_HIP(hipMallocAsync(&ws, ((size_t)nb * MP + (size_t)nb) * sizeof(float), st));
    float *gpart = (float *)ws, *lpart = gpart + (size_t)nb * MP;
    hipLaunchKernelGGL(k_mlp_grad_partial, dim3(nb), dim3(64), 0, st, params, X, t, B, gpart, lpart);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((MP + 255) / 256), dim3(256), 0, st, (const float *)gpart, nb,
                       (const float *)lpart, grad, loss);
    const hipError_t e = hipGetLastError();
    hipFreeAsync(ws, st);
    if (e != hipSuccess) return hip_fail(e, "MLP backward");
    return SV_OK;
}

sv_status sv_mlp_adam(float *params, float *m, float *v, const float *grad, int n, int step, float lr, float beta1,
                      float beta2, float eps, void *hip_stream) {
    clear_error();
    if (!params || !m || !v || !grad || n < 0 || step < 1) return fail(SV_EINVAL, "bad Adam arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, params, m, v, grad,
                       n, lr, beta1, beta2, eps, c1, c2);
    SV_HIP(hipGetLastError());
    return SV_OK;
}

}  // extern "C"
