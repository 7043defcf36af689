// The non-deferred render (the performance ablation of Section 7.1): the
// view-dependent network of Eq. 7 runs on every composited sample, with that
// sample's own colour and features and the ray direction, and its residual
// is added to the sample's colour before compositing, as NeRF queries its
// MLP at every sample.  No network runs per pixel.  Each lane holds its ray's
// direction encoding (FP16 path: staged once per ray in the MFMA input rows;
// FP32 path: the direction part of layer 1, b1 + W1[:, 7:34] x[7:34], once
// per ray in LDS); the march is wavefront-convergent so that a sample found
// by any lane is shaded at the next convergent point, on MFMA tiles for all
// 64 lanes at once or per lane in FP32.
#include "march.h"
#include "mlp.h"
#include "snerg_launch.h"

namespace snerg {

namespace {

struct PsAccum {
    float C[3], T;
    bool gate;
};

__device__ __forceinline__ int64_t wave_uniform_ps(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Ray of lane `lane` for wavefront index t (tile or first list entry).
__device__ __forceinline__ bool locate_ps(const RenderArgs& a, int64_t t, int lane, int& ci, int& px, int& py,
                                          int64_t& out_idx) {
    if (a.mode == kModeList) {
        out_idx = t + lane;
        if (out_idx >= a.n_rays) return false;
        const int64_t r = a.ray_ids[out_idx];
        ci = find_camera_by_ray(a.cams, a.n_cams, r);
        const int64_t local = r - a.cams[ci].ray_offset;
        py = int(local / a.cams[ci].W);
        px = int(local - int64_t(py) * a.cams[ci].W);
        return true;
    }
    if (a.tile_order) t = a.tile_order[t];
    ci = find_camera_by_tile(a.cams, a.n_cams, t);
    const DevCamera& c = a.cams[ci];
    const int64_t tl = t - c.tile_offset;
    px = int(tl % c.tiles_x) * a.tile_w + lane % a.tile_w;
    py = int(tl / c.tiles_x) * a.tile_h + lane / a.tile_w;
    out_idx = c.ray_offset + int64_t(py) * c.W + px;
    return px < c.W && py < c.H;
}

}  // namespace

template <int VT, bool F16>
__global__ __launch_bounds__(256) void k_render_ps(RenderArgs a) {
    extern __shared__ uint2 s_occ[];
    __shared__ _Float16 xs[F16 ? kMaxWavesF16 : 1][64][kXRow];   // FP16: network inputs per lane
    __shared__ float u1[F16 ? 1 : kMaxWavesF16][64][kMlpH + 1];  // FP32: direction part of layer 1
    const GridArgs& g = a.grid;
    for (int w = threadIdx.x; w < g.n_words; w += blockDim.x) s_occ[w] = g.occ[w];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpg = blockDim.x >> 6;
    cfloat* W = as_const(a.mlp);
    const bool use_mlp = a.opts.mlp_on != 0;
    // FP16 path: the weights as MFMA fragments, once per wavefront
    MlpFragsF16 frags;
    if (F16 && use_mlp) frags = mlp_frags_f16(W);
    const float cs = VT == 0 ? (1.0f / 255.0f) : 1.0f;
    const float kx = g.sigma_scale * cs / float(g.N);
    const float t_stop = a.opts.t_stop;
    const bool early = a.opts.early_stop != 0;
    const bool nn_gate = a.opts.nn_gate != 0;
    const bool persist = a.mode == kModePersistent;
    int64_t t = a.mode == kModeList ? int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63)
                                    : int64_t(xcd_grouped(blockIdx.x, gridDim.x)) * wpg + wave;
    for (;;) {
        if (persist) {
            int64_t v = 0;
            if (lane == 0) v = atomicAdd(a.tile_counter, 1);
            t = __shfl(v, 0);
        }
        t = wave_uniform_ps(t);
        if (t >= (a.mode == kModeList ? a.n_rays : a.total_tiles)) break;  // wave-uniform
        int ci = 0, px = 0, py = 0;
        int64_t out_idx = 0;
        const bool valid = locate_ps(a, t, lane, ci, px, py, out_idx);
        int64_t o[3] = {0, 0, 0};
        int32_t s[3] = {0, 0, 1 << 15};
        float d[3] = {0.f, 0.f, 1.f};
        if (valid) ray_setup(a.cams[ci], g.N, px, py, o, s, d);
        // this ray's direction encoding, once
        {
            float x[kMlpIn];
            const float z3[3] = {0.f, 0.f, 0.f}, z4[4] = {0.f, 0.f, 0.f, 0.f};
            encode_x(z3, z4, d, x);
            if (F16) {
#pragma unroll
                for (int i = 0; i < kXPad; ++i) xs[wave][lane][i] = _Float16(i < kMlpIn ? x[i] : 0.0f);
            } else {
                for (int j = 0; j < kMlpH; ++j) {
                    float acc = W[kOffB1 + j];
#pragma unroll
                    for (int i = 7; i < kMlpIn; ++i) acc = fmaf(W[kOffW1 + j * kMlpIn + i], x[i], acc);
                    u1[wave][lane][j] = acc;
                }
            }
        }
        PsAccum st = {{0.f, 0.f, 0.f}, 1.0f, false};
        bool pending = false;
        float pc[3] = {0.f, 0.f, 0.f}, pv[4] = {0.f, 0.f, 0.f, 0.f}, psig = 0.f;
        march_ray_flat_sync(
            g, s_occ, valid, o, s,
            [&](int64_t, int32_t, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
                Sample smp;
                if (VT == 0) {
                    Corners8 cn;
                    load_corners_u8(vox + (uint64_t(cell_index(p, uint32_t(g.Bp), uint32_t(g.Bp * g.Bp))) << 3),
                                    g.Bp, cn);
                    interp_u8(cn, fr, smp);
                    if (nn_gate) smp.active = nearest_nonzero_u8(cn, fr);
                } else {
                    gather_f32(vox, g.Bp, p, fr, smp, nn_gate);
                }
                if (!smp.active) return false;
                pending = true;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) pc[ch] = smp.rgb[ch] * cs;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) pv[ch] = smp.feat[ch] * cs;
                psig = smp.sigma_raw;
                return false;
            },
            [&]() -> bool {
                if (!__any(pending)) return false;
                float R[3] = {0.f, 0.f, 0.f};
                if (use_mlp) {
                    if (F16) {
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) xs[wave][lane][ch] = _Float16(pc[ch]);
#pragma unroll
                        for (int ch = 0; ch < 4; ++ch) xs[wave][lane][3 + ch] = _Float16(pv[ch]);
                        mlp_eval_f16_wave(frags, xs[wave], pending, R);
                    } else if (pending) {
                        const float xi[7] = {pc[0], pc[1], pc[2], pv[0], pv[1], pv[2], pv[3]};
                        float h2[kMlpH];
#pragma unroll
                        for (int k = 0; k < kMlpH; ++k) h2[k] = W[kOffB2 + k];
#pragma nounroll
                        for (int j = 0; j < kMlpH; ++j) {
                            float acc = u1[wave][lane][j];
#pragma unroll
                            for (int i = 0; i < 7; ++i) acc = fmaf(W[kOffW1 + j * kMlpIn + i], xi[i], acc);
                            const float h1j = fmaxf(acc, 0.0f);
#pragma unroll
                            for (int k = 0; k < kMlpH; ++k) h2[k] = fmaf(W[kOffW2 + k * kMlpH + j], h1j, h2[k]);
                        }
#pragma unroll
                        for (int q = 0; q < kMlpOut; ++q) {
                            float z = W[kOffB3 + q];
#pragma unroll
                            for (int k = 0; k < kMlpH; ++k) z = fmaf(W[kOffW3 + q * kMlpH + k], fmaxf(h2[k], 0.0f), z);
                            R[q] = sigmoid_f32(z);
                        }
                    }
                }
                bool stop = false;
                if (pending) {
                    const float e = __expf(-psig * kx);
                    const float w = st.T * (1.0f - e);
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) st.C[ch] += w * (pc[ch] + R[ch]);
                    st.T *= e;
                    st.gate = true;
                    stop = early && st.T < t_stop;
                    pending = false;
                }
                return stop;
            });
        if (valid) {
            float T = st.T;
            float C[3] = {st.C[0], st.C[1], st.C[2]};
            if (a.opts.unpremultiply) {
                const float al = 1.0f - T;
                if (al > 0.0f) {
                    const float sc = fminf(1.0f, 1.5f * al) / al;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) C[ch] *= sc;
                    T = 1.0f - al * sc;
                }
            }
            reinterpret_cast<float4*>(a.out)[out_idx] =
                make_float4(C[0] + T * a.opts.bg[0], C[1] + T * a.opts.bg[1], C[2] + T * a.opts.bg[2], 1.0f - T);
        }
        if (!persist) break;
    }
}

hipError_t launch_render_ps(const RenderArgs& a, int vt, bool f16, int wpg, int n_groups, hipStream_t s) {
    const int threads = 64 * wpg;
    unsigned blocks;
    if (a.mode == kModeList) blocks = unsigned((a.n_rays + threads - 1) / threads);
    else if (a.mode == kModeTiles) blocks = unsigned((a.total_tiles + wpg - 1) / wpg);
    else blocks = unsigned(n_groups);
    if (blocks == 0) return hipSuccess;
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2);
    if (vt == 0) {
        if (f16) hipLaunchKernelGGL((k_render_ps<0, true>), dim3(blocks), dim3(threads), lds, s, a);
        else hipLaunchKernelGGL((k_render_ps<0, false>), dim3(blocks), dim3(threads), lds, s, a);
    } else {
        if (f16) hipLaunchKernelGGL((k_render_ps<1, true>), dim3(blocks), dim3(threads), lds, s, a);
        else hipLaunchKernelGGL((k_render_ps<1, false>), dim3(blocks), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace snerg
