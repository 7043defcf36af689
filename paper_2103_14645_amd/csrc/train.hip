// Fine-tuning of the deferred shading network (Section 5.5): the squared
// error between rendered and observed pixels, and the Adam update of the
// network weights (Kingma and Ba, Algorithm 1) with the learning rate of
// Section 5.5.
#include "snerg_launch.h"

namespace snerg {

// grad[i] = (2 / (3 n)) (rgb_i - target_j) for the three colour channels,
// 0 for alpha, with j = ids[i] (or i without ids); each workgroup adds its
// share of (1 / (3 n)) sum (rgb - target)^2 to *loss (which holds zero).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ rgba, const float* __restrict__ target,
                                             const int64_t* __restrict__ ids, int64_t n, float* __restrict__ grad,
                                             float* __restrict__ loss) {
    __shared__ float part[4];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const float inv = 1.0f / (3.0f * float(n));
    float sq = 0.0f;
    if (i < n) {
        const float4 p = reinterpret_cast<const float4*>(rgba)[i];
        const float4 t = reinterpret_cast<const float4*>(target)[ids ? ids[i] : i];
        const float e0 = p.x - t.x, e1 = p.y - t.y, e2 = p.z - t.z;
        reinterpret_cast<float4*>(grad)[i] = make_float4(2.0f * inv * e0, 2.0f * inv * e1, 2.0f * inv * e2, 0.0f);
        sq = (e0 * e0 + e1 * e1) + e2 * e2;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) sq += __shfl_xor(sq, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, ((part[0] + part[1]) + (part[2] + part[3])) * inv);
}

// One Adam step (t >= 1): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_mse(const float* rgba, const float* target, const int64_t* ids, int64_t n, float* grad, float* loss,
                      hipStream_t s) {
    hipError_t e = launch_fill_f32(loss, 1, 0.0f, s);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_mse, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, rgba, target, ids, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace snerg
