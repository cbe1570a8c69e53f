// Kernels of the variant selector: a 12 -> 32 -> 32 -> 3 fp32 MLP (ReLU) that
// predicts the log device time of one level under each form of the product
// (push, pull, push-bitmap) from the level's frontier / remainder statistics.
// It only picks which form runs; every form returns the same bits.
//
// Weight blob (kMlpTotal floats): W1[32][12] b1[32] W2[32][32] b2[32] W3[3][32]
// b3[3], then the feature mean[12] and inverse std[12] used to normalise the
// raw features (the same blob the level kernel evaluates on the device).
//
// Training: forward + backward of a mean-squared error over the measured
// (masked) log-times, gradients summed per block in LDS then once per block
// into the global gradient, Adam update in place.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bfs_internal.h"

namespace bfsi {

namespace {

constexpr int kW1 = 0, kB1 = kW1 + kMlpIn * kMlpH, kW2 = kB1 + kMlpH, kB2 = kW2 + kMlpH * kMlpH,
              kW3 = kB2 + kMlpH, kB3 = kW3 + kMlpH * kMlpOut, kMean = kMlpParams,
              kIstd = kMean + kMlpIn;

struct Act {
    float x[kMlpIn];
    float z1[kMlpH], h1[kMlpH], z2[kMlpH], h2[kMlpH];
    float y[kMlpOut];
};

__device__ __forceinline__ void forward(const float *w, const float *xr, Act &a) {
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) a.x[i] = (xr[i] - w[kMean + i]) * w[kIstd + i];
#pragma unroll
    for (int o = 0; o < kMlpH; ++o) {
        float s = w[kB1 + o];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) s = fmaf(w[kW1 + o * kMlpIn + i], a.x[i], s);
        a.z1[o] = s;
        a.h1[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int o = 0; o < kMlpH; ++o) {
        float s = w[kB2 + o];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) s = fmaf(w[kW2 + o * kMlpH + i], a.h1[i], s);
        a.z2[o] = s;
        a.h2[o] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kMlpOut; ++u) {
        float s = w[kB3 + u];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) s = fmaf(w[kW3 + u * kMlpH + i], a.h2[i], s);
        a.y[u] = s;
    }
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_mlp_forward(const float *w, const float *x, float *y,
                                                        int32_t rows) {
    __shared__ float sw[kMlpTotal];
    for (int i = threadIdx.x; i < kMlpTotal; i += kBlock) sw[i] = w[i];
    __syncthreads();
    const int32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= rows) return;
    Act a;
    forward(sw, x + (size_t)r * kMlpIn, a);
#pragma unroll
    for (int u = 0; u < kMlpOut; ++u) y[(size_t)r * kMlpOut + u] = a.y[u];
}

// loss = sum(mask * (y - t)^2) / max(1, sum(mask)); grad += d loss / d w
// (weights and biases only; the normalisation constants are fixed).
__global__ __launch_bounds__(kBlock) void k_mlp_grad(const float *w, const float *x, const float *t,
                                                     const float *mask, int32_t rows, float inv_norm,
                                                     float *grad, float *loss) {
    __shared__ float sw[kMlpTotal];
    __shared__ float sg[kMlpParams];
    __shared__ float sl;
    for (int i = threadIdx.x; i < kMlpTotal; i += kBlock) sw[i] = w[i];
    for (int i = threadIdx.x; i < kMlpParams; i += kBlock) sg[i] = 0.f;
    if (threadIdx.x == 0) sl = 0.f;
    __syncthreads();
    const int32_t r = blockIdx.x * kBlock + threadIdx.x;
    if (r < rows) {
        Act a;
        forward(sw, x + (size_t)r * kMlpIn, a);
        float dy[kMlpOut];
        float l = 0.f;
#pragma unroll
        for (int u = 0; u < kMlpOut; ++u) {
            const float m = mask[(size_t)r * kMlpOut + u];
            const float d = a.y[u] - t[(size_t)r * kMlpOut + u];
            l += m * d * d;
            dy[u] = 2.f * m * d * inv_norm;
        }
        atomicAdd(&sl, l * inv_norm);
        float dh2[kMlpH];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) dh2[i] = 0.f;
#pragma unroll
        for (int u = 0; u < kMlpOut; ++u) {
            if (dy[u] == 0.f) continue;
            atomicAdd(&sg[kB3 + u], dy[u]);
#pragma unroll
            for (int i = 0; i < kMlpH; ++i) {
                atomicAdd(&sg[kW3 + u * kMlpH + i], dy[u] * a.h2[i]);
                dh2[i] = fmaf(sw[kW3 + u * kMlpH + i], dy[u], dh2[i]);
            }
        }
        float dh1[kMlpH];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) dh1[i] = 0.f;
#pragma unroll
        for (int o = 0; o < kMlpH; ++o) {
            const float dz = a.z2[o] > 0.f ? dh2[o] : 0.f;
            if (dz == 0.f) continue;
            atomicAdd(&sg[kB2 + o], dz);
#pragma unroll
            for (int i = 0; i < kMlpH; ++i) {
                atomicAdd(&sg[kW2 + o * kMlpH + i], dz * a.h1[i]);
                dh1[i] = fmaf(sw[kW2 + o * kMlpH + i], dz, dh1[i]);
            }
        }
#pragma unroll
        for (int o = 0; o < kMlpH; ++o) {
            const float dz = a.z1[o] > 0.f ? dh1[o] : 0.f;
            if (dz == 0.f) continue;
            atomicAdd(&sg[kB1 + o], dz);
#pragma unroll
            for (int i = 0; i < kMlpIn; ++i) atomicAdd(&sg[kW1 + o * kMlpIn + i], dz * a.x[i]);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMlpParams; i += kBlock)
        if (sg[i] != 0.f) atomicAdd(&grad[i], sg[i]);
    if (threadIdx.x == 0) atomicAdd(loss, sl);
}

// Adam on the weights and biases; the gradient buffer is zeroed for the next step.
__global__ __launch_bounds__(kBlock) void k_mlp_adam(float *w, float *grad, float *m, float *v,
                                                     float lr, float c1, float c2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= kMlpParams) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    grad[i] = 0.f;
}

hipError_t launch_mlp_forward(const float *w, const float *x, float *y, int32_t rows, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s, w, x, y, rows);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *w, const float *x, const float *t, const float *mask,
                           int32_t rows, float inv_norm, float *grad, float *loss, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_grad, dim3((rows + kBlock - 1) / kBlock), dim3(kBlock), 0, s, w, x, t,
                       mask, rows, inv_norm, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *grad, float *m, float *v, int32_t step, float lr,
                           hipStream_t s) {
    const float c1 = 1.f / (1.f - powf(0.9f, (float)step));
    const float c2 = 1.f / (1.f - powf(0.999f, (float)step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, w,
                       grad, m, v, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace bfsi
