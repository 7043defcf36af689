// Adjoint of the render (fine-tuning by a pixel loss, Eq. 3, Section 5.5).
//
// For each ray with output gradient g = dL/d(rgb, alpha):
//  1. MLP backward (Eq. 7): g_C = g_rgb + (J_R^T g_rgb)[0:3],
//     g_V = (J_R^T g_rgb)[3:7]; the weight gradients of the wavefront's 64
//     rays are summed with FP32 MFMA outer products (rays are the K
//     dimension) into per-wavefront accumulators.
//  2. Re-march the same samples (nothing per sample was stored).  With
//     E = g_C . C_d + g_V . V (from the forward's saved C_d, V), the running
//     prefix P_k = sum_{j<=k} w_j e_j, e_k = g_C . c_k + g_V . v_k and
//     dL/dT_N = g_rgb . bg - g_alpha, Eq. 2/5/6 give
//        dL/dsigma_k = delta [T_k e_k - (E - P_k) - T_N dL/dT_N],
//        dL/dc_k = w_k g_C,  dL/dv_k = w_k g_V,
//     (T_k: transmittance after sample k), which the trilinear weights
//     scatter to the 8 corner voxels with float atomics.
#include "march.h"
#include "mlp.h"
#include "snerg_launch.h"

namespace snerg {

typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kStageRow = 52;  // floats per ray in the LDS staging buffer
constexpr int kBwdMaxWaves = 4;

// Adds val to the canonical gradient slot of padded corner (p + c) of block
// (id at block coordinates b).  Corners outside the grid or in empty blocks
// are structural zeros and get nothing.
__device__ __forceinline__ int64_t canonical_voxel(const GridArgs& g, int32_t id, const int32_t b[3],
                                                   int vx, int vy, int vz) {
    const int B = g.B;
    int32_t tid = id;
    if (vx < 0 || vy < 0 || vz < 0 || vx >= B || vy >= B || vz >= B) {
        const int nx = b[0] + (vx < 0 ? -1 : (vx >= B ? 1 : 0));
        const int ny = b[1] + (vy < 0 ? -1 : (vy >= B ? 1 : 0));
        const int nz = b[2] + (vz < 0 ? -1 : (vz >= B ? 1 : 0));
        if (nx < 0 || ny < 0 || nz < 0 || nx >= g.G || ny >= g.G || nz >= g.G) return -1;
        tid = g.ind[(nz * g.G + ny) * g.G + nx];
        if (tid < 0 || tid >= g.n_blocks) return -1;
        vx &= B - 1;
        vy &= B - 1;
        vz &= B - 1;
    }
    return int64_t(tid) * B * B * B + (int64_t(vz) * B + vy) * B + vx;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

template <int MLP>
__global__ __launch_bounds__(256) void k_backward(BackwardArgs a) {
    __shared__ float stage[kBwdMaxWaves][64][kStageRow];
    extern __shared__ uint2 s_occ[];
    for (int w = threadIdx.x; w < a.grid.n_words; w += blockDim.x) s_occ[w] = a.grid.occ[w];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpg = blockDim.x >> 6;
    const GridArgs& g = a.grid;
    const float delta = 1.0f / float(g.N);
    const float kx = g.sigma_scale * delta;
    cfloat* W = as_const(a.mlp);

    float4v acc1[3] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    float4v acc2 = {0.f, 0.f, 0.f, 0.f}, acc3 = {0.f, 0.f, 0.f, 0.f};
    float db2 = 0.f, db3 = 0.f;  // lane j < 16 / < 3 holds the sum

    const int64_t stride = int64_t(gridDim.x) * wpg * 64;
    for (int64_t base = (int64_t(blockIdx.x) * wpg + wave) * 64; base < a.n_rays; base += stride) {
        const int64_t i = base + lane;
        const bool valid = i < a.n_rays;
        int ci = 0, px = 0, py = 0;
        if (valid) {
            const int64_t r = a.ray_ids ? a.ray_ids[i] : i;
            ci = find_camera_by_ray(a.cams, a.n_cams, r);
            const int64_t local = r - a.cams[ci].ray_offset;
            py = int(local / a.cams[ci].W);
            px = int(local - int64_t(py) * a.cams[ci].W);
        }
        int64_t o[3] = {0, 0, 0};
        int32_t s[3] = {0, 0, 0};
        float d[3] = {0.f, 0.f, 1.f};
        float C[3] = {0.f, 0.f, 0.f}, V[4] = {0.f, 0.f, 0.f, 0.f}, TN = 1.0f;
        float gr[4] = {0.f, 0.f, 0.f, 0.f};
        bool gate = false;
        if (valid) {
            ray_setup(a.cams[ci], g.N, px, py, o, s, d);
            const float4 a0 = reinterpret_cast<const float4*>(a.aux)[2 * i];
            const float4 a1 = reinterpret_cast<const float4*>(a.aux)[2 * i + 1];
            C[0] = a0.x; C[1] = a0.y; C[2] = a0.z; V[0] = a0.w;
            V[1] = a1.x; V[2] = a1.y; V[3] = a1.z;
            gate = a1.w >= 0.0f;
            TN = gate ? a1.w : 1.0f;
            const float4 gg = reinterpret_cast<const float4*>(a.grad_rgba)[i];
            gr[0] = gg.x; gr[1] = gg.y; gr[2] = gg.z; gr[3] = gg.w;
        }
        float gC[3] = {gr[0], gr[1], gr[2]};
        float gV[4] = {0.f, 0.f, 0.f, 0.f};

        if (MLP != kMlpOff) {
            const bool use = valid && gate && a.opts.mlp_on;
            float x[kMlpIn];
            encode_x(C, V, d, x);
            float h1[kMlpH], h2[kMlpH], go[kMlpOut], gh1[kMlpH], gh2[kMlpH];
#pragma unroll
            for (int j = 0; j < kMlpH; ++j) {
                float t = W[kOffB1 + j];
#pragma unroll
                for (int q = 0; q < kMlpIn; ++q) t = fmaf(W[kOffW1 + j * kMlpIn + q], x[q], t);
                h1[j] = fmaxf(t, 0.0f);
            }
#pragma unroll
            for (int j = 0; j < kMlpH; ++j) {
                float t = W[kOffB2 + j];
#pragma unroll
                for (int q = 0; q < kMlpH; ++q) t = fmaf(W[kOffW2 + j * kMlpH + q], h1[q], t);
                h2[j] = fmaxf(t, 0.0f);
            }
#pragma unroll
            for (int j = 0; j < kMlpOut; ++j) {
                float t = W[kOffB3 + j];
#pragma unroll
                for (int q = 0; q < kMlpH; ++q) t = fmaf(W[kOffW3 + j * kMlpH + q], h2[q], t);
                const float R = sigmoid_f32(t);
                go[j] = use ? gr[j] * R * (1.0f - R) : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) {
                float t = 0.f;
#pragma unroll
                for (int j = 0; j < kMlpOut; ++j) t = fmaf(W[kOffW3 + j * kMlpH + q], go[j], t);
                gh2[q] = h2[q] > 0.0f ? t : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) {
                float t = 0.f;
#pragma unroll
                for (int j = 0; j < kMlpH; ++j) t = fmaf(W[kOffW2 + j * kMlpH + q], gh2[j], t);
                gh1[q] = h1[q] > 0.0f ? t : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                float t = 0.f;
#pragma unroll
                for (int j = 0; j < kMlpH; ++j) t = fmaf(W[kOffW1 + j * kMlpIn + q], gh1[j], t);
                if (q < 3) gC[q] += t; else gV[q - 3] = t;
            }

            // Weight gradients: dW = sum_r gA_r (x) act_r as 16x16x4 FP32 MFMAs,
            // A = gradient rows (16 x 4 rays), B = activations (4 rays x 16).
            float* st = &stage[wave][0][0];
            float* me = &stage[wave][lane][0];
            // phase 1: gh1 (16) | x (34) | 1 (bias column) | 0
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) me[q] = gh1[q];
#pragma unroll
            for (int q = 0; q < kMlpIn; ++q) me[16 + q] = x[q];
            me[16 + 34] = use ? 1.0f : 0.0f;
            me[16 + 35] = 0.0f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int li = lane & 15, lk = lane >> 4;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const float* rr = st + (4 * kk + lk) * kStageRow;
                const float av = rr[li];
#pragma unroll
                for (int nt = 0; nt < 3; ++nt) {
                    const int col = 16 * nt + li;
                    const float bv = col < 36 ? rr[16 + col] : 0.0f;
                    acc1[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc1[nt], 0, 0, 0);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // phase 2: gh2 (16) | h1 (16) | go (3) | h2 (16)
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) me[q] = gh2[q];
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) me[16 + q] = use ? h1[q] : 0.0f;
#pragma unroll
            for (int q = 0; q < kMlpOut; ++q) me[32 + q] = go[q];
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) me[35 + q] = use ? h2[q] : 0.0f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const float* rr = st + (4 * kk + lk) * kStageRow;
                acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(rr[li], rr[16 + li], acc2, 0, 0, 0);
                const float a3 = li < 3 ? rr[32 + li] : 0.0f;
                acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, rr[35 + li], acc3, 0, 0, 0);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) {
                const float sq = wave_sum(gh2[q]);
                if (lane == q) db2 += sq;
            }
#pragma unroll
            for (int q = 0; q < kMlpOut; ++q) {
                const float sq = wave_sum(go[q]);
                if (lane == q) db3 += sq;
            }
            if (!a.opts.mlp_on) {
                gC[0] = gr[0]; gC[1] = gr[1]; gC[2] = gr[2];
                gV[0] = gV[1] = gV[2] = gV[3] = 0.0f;
            }
        }

        if (valid && gate) {
            const float E = gC[0] * C[0] + gC[1] * C[1] + gC[2] * C[2] +
                            (gV[0] * V[0] + gV[1] * V[1] + gV[2] * V[2] + gV[3] * V[3]);
            const float gTN = gr[0] * a.opts.bg[0] + gr[1] * a.opts.bg[1] + gr[2] * a.opts.bg[2] - gr[3];
            const float tail = TN * gTN;
            float T = 1.0f, Pk = 0.0f;
            const float t_stop = a.opts.t_stop;
            const bool early = a.opts.early_stop != 0;
            march_ray(
                g, s_occ, o, s, [](int32_t, bool) {}, [](int32_t) {},
                [&](int64_t, int32_t rk, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
                    Sample smp;
                    gather_f32(vox, g.Bp, p, fr, smp);
                    if (!smp.active) return false;
                    const float x = smp.sigma_raw * kx;
                    const float e = __expf(-x);
                    const float alpha = 1.0f - e;
                    const float w = T * alpha;
                    const float ek = gC[0] * smp.rgb[0] + gC[1] * smp.rgb[1] + gC[2] * smp.rgb[2] +
                                     (gV[0] * smp.feat[0] + gV[1] * smp.feat[1] + gV[2] * smp.feat[2] +
                                      gV[3] * smp.feat[3]);
                    Pk += w * ek;
                    T *= e;
                    const float gsig = delta * (T * ek - (E - Pk) - tail);
                    // scatter through the trilinear weights
                    const int32_t lin = g.rank_lin[rk];
                    const int32_t id = g.rank_id[rk];
                    const int32_t b[3] = {lin % g.G, (lin / g.G) % g.G, lin / (g.G * g.G)};
                    float wc[8];
                    corner_weights(fr, wc);
                    const float gd = g.sigma_scale * gsig;
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        if (!corner_live(c, fr)) continue;
                        const int64_t vi = canonical_voxel(g, id, b, p[0] + (c & 1) - 1,
                                                           p[1] + ((c >> 1) & 1) - 1, p[2] + (c >> 2) - 1);
                        if (vi < 0) continue;
                        const float ww = wc[c] * w;
                        unsafeAtomicAdd(a.grad_dens + vi, wc[c] * gd);
                        unsafeAtomicAdd(a.grad_rgb + 3 * vi + 0, ww * gC[0]);
                        unsafeAtomicAdd(a.grad_rgb + 3 * vi + 1, ww * gC[1]);
                        unsafeAtomicAdd(a.grad_rgb + 3 * vi + 2, ww * gC[2]);
                        if (MLP != kMlpOff) {
                            unsafeAtomicAdd(a.grad_feat + 4 * vi + 0, ww * gV[0]);
                            unsafeAtomicAdd(a.grad_feat + 4 * vi + 1, ww * gV[1]);
                            unsafeAtomicAdd(a.grad_feat + 4 * vi + 2, ww * gV[2]);
                            unsafeAtomicAdd(a.grad_feat + 4 * vi + 3, ww * gV[3]);
                        }
                    }
                    return early && T < t_stop;
                });
        }
    }

    if (MLP != kMlpOff) {
        // this wavefront's partial MLP gradient, in parameter order
        float* out = a.g_mlp_partial + (int64_t(blockIdx.x) * wpg + wave) * kMlpParams;
        const int li = lane & 15, lr = 4 * (lane >> 4);
#pragma unroll
        for (int nt = 0; nt < 3; ++nt) {
            const int col = 16 * nt + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = lr + v;
                if (col < kMlpIn) out[kOffW1 + row * kMlpIn + col] = acc1[nt][v];
                else if (col == kMlpIn) out[kOffB1 + row] = acc1[nt][v];
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            out[kOffW2 + (lr + v) * kMlpH + li] = acc2[v];
            if (lr + v < kMlpOut) out[kOffW3 + (lr + v) * kMlpH + li] = acc3[v];
        }
        if (lane < kMlpH) out[kOffB2 + lane] = db2;
        if (lane < kMlpOut) out[kOffB3 + lane] = db3;
    }
}

__global__ void k_reduce_rows(const float* __restrict__ partial, int rows, float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= kMlpParams) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += partial[int64_t(r) * kMlpParams + j];
    out[j] = s;
}

hipError_t launch_backward(const BackwardArgs& a, int n_groups, hipStream_t s) {
    if (n_groups <= 0) return hipSuccess;
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2);
    if (a.mlp_mode == kMlpOff)
        hipLaunchKernelGGL(k_backward<kMlpOff>, dim3(n_groups), dim3(64 * kBwdMaxWaves), lds, s, a);
    else
        hipLaunchKernelGGL(k_backward<kMlpF32>, dim3(n_groups), dim3(64 * kBwdMaxWaves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_mlp(const float* partial, int rows, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_rows, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, rows, out);
    return hipGetLastError();
}

}  // namespace snerg
