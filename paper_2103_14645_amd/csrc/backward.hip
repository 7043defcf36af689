// Adjoint of the render (fine-tuning by a pixel loss, Eq. 3, Section 5.5).
//
// For each ray with output gradient g = dL/d(rgb, alpha):
//  K1 (k_mlp_backward, only with the MLP on): MLP backward (Eq. 7):
//     g_C = g_rgb + (J_R^T g_rgb)[0:3], g_V = (J_R^T g_rgb)[3:7], written per
//     ray; the weight gradients of the wavefront's 64 rays are summed with
//     FP32 MFMA outer products (rays are the K dimension) into per-wavefront
//     partial rows, reduced afterwards.
//  K2 (k_march_backward): re-march the same samples (nothing per sample was
//     stored).  With E = g_C . C_d + g_V . V (from the forward's saved C_d,
//     V), the running prefix P_k = sum_{j<=k} w_j e_j, e_k = g_C . c_k +
//     g_V . v_k and dL/dT_N = g_rgb . bg - g_alpha, Eq. 2/5/6 give
//        dL/dsigma_k = delta [T_k e_k - (E - P_k) - T_N dL/dT_N],
//        dL/dc_k = w_k g_C,  dL/dv_k = w_k g_V,
//     (T_k: transmittance after sample k).  Through the trilinear weights
//     w_c(k) a corner voxel receives sum_k w_c(k) dL/dsigma_k (density) and
//     g_C, g_V times A = sum_k w_c(k) w_k (colour, features).  Along one ray
//     each cell coordinate is monotone, so the 8 corners of the current cell
//     are kept as running (A, D) sums and a voxel is handed over once, when
//     the ray's cell window leaves it: into a per-wavefront LDS table that
//     sums the hand-overs of the wavefront's rays (whole views in 8x8 pixel
//     tiles, patch lists), or an LDS log (scattered ray lists), flushed to
//     the gradient arrays with float atomics grouped by cache line.
//  Short ray lists (up to 2^18 rays) run K2 in two phases: k_backward_record
//     lists each ray's samples, k_backward_from_list runs the same adjoint
//     over the lists (the single re-march is as slow as its slowest
//     wavefront when the wavefronts are few).
#include "march.h"
#include "mlp.h"
#include "snerg_launch.h"

namespace snerg {

typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kBwdWaves = 2;  // wavefronts per K1 workgroup
// K1 staging row per ray (floats): gh1 | x (34) 1 0 | gh2 | h1 | go (3) 0 | h2
constexpr int kSGh1 = 0, kSX = 16, kSGh2 = 52, kSH1 = 68, kSGo = 84, kSH2 = 88;
constexpr int kStageRow = 105;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ void locate(const BackwardArgs& a, int64_t r, int& ci, int& px, int& py) {
    ci = find_camera_by_ray(a.cams, a.n_cams, r);
    const int64_t local = r - a.cams[ci].ray_offset;
    py = int(local / a.cams[ci].W);
    px = int(local - int64_t(py) * a.cams[ci].W);
}

// ------------------------------------------------------------------ K1: MLP

// A-operand fragment of the transpose of a row-major [rows][cols] matrix M
// (a 16x16 tile of M^T): lane l holds M^T[l%16][4(l/16) + j] = M[4(l/16) + j][l%16].
__device__ __forceinline__ half4_t a_frag_t(cfloat* M, int rows, int cols, int lane) {
    const int c = lane & 15;
    const int r = 4 * (lane >> 4);
    half4_t v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (r + j < rows && c < cols) ? _Float16(M[(r + j) * cols + c]) : _Float16(0.0f);
    return v;
}

__device__ __forceinline__ half4_t to_half4(float4_t v) {
    half4_t h;
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = _Float16(v[j]);
    return h;
}

// The MLP chain of 64 rays on FP16 MFMA tiles.  xs: the rays' inputs
// ([64][kXRow] halves), gsm: per ray g_rgb and the gate, stage: per-ray
// rows that receive h1, h2, go, gh2, gh1 (float).  Tile layouts (16x16x16):
// A lane l = [m = l%16][k = 4(l/16)+j], B lane l = [k = 4(l/16)+j][n = l%16],
// D lane l = [m = 4(l/16)+v][n = l%16]; hidden units are rows, rays columns,
// so every D tile (after its element-wise step) is the next B operand.
__device__ __forceinline__ void mlp_backward_f16_wave(const BackwardArgs& a, cfloat* W, const _Float16* xs,
                                                      const float* gsm, float* stage, int64_t base, int lane) {
    const half8_t w1[2] = {a_frag32(W + kOffW1, kMlpIn, 0, lane), a_frag32(W + kOffW1, kMlpIn, 1, lane)};
    const half4_t w2 = a_frag(W + kOffW2, kMlpH, kMlpH, 0, 0, lane);
    const half4_t w3 = a_frag(W + kOffW3, kMlpOut, kMlpH, 0, 0, lane);
    const half4_t w3t = a_frag_t(W + kOffW3, kMlpOut, kMlpH, lane);
    const half4_t w2t = a_frag_t(W + kOffW2, kMlpH, kMlpH, lane);
    const half4_t w1t = a_frag_t(W + kOffW1, kMlpH, kMlpIn, lane);  // input rows 0..15
    const float4_t bb1 = bias_frag(W + kOffB1, kMlpH, lane);
    const float4_t bb2 = bias_frag(W + kOffB2, kMlpH, lane);
    const float4_t bb3 = bias_frag(W + kOffB3, kMlpOut, lane);
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    const int n = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int ray = 16 * g + n;  // this lane's column
        const _Float16 (*rows)[kXRow] = reinterpret_cast<const _Float16 (*)[kXRow]>(xs);
        float4_t h1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(w1[0], x_frag32(rows, g, 0, lane), bb1, 0, 0, 0);
        h1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(w1[1], x_frag32(rows, g, 1, lane), h1, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) h1[v] = fmaxf(h1[v], 0.0f);
        float4_t h2 = __builtin_amdgcn_mfma_f32_16x16x16f16(w2, to_half4(h1), bb2, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) h2[v] = fmaxf(h2[v], 0.0f);
        const float4_t o = __builtin_amdgcn_mfma_f32_16x16x16f16(w3, to_half4(h2), bb3, 0, 0, 0);
        const float use = gsm[ray * 4 + 3];
        float4_t go = zero;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            if (lane < 16) {
                const float R = sigmoid_f32(o[v]);
                go[v] = use * gsm[ray * 4 + v] * R * (1.0f - R);
            }
        }
        float4_t gh2 = __builtin_amdgcn_mfma_f32_16x16x16f16(w3t, to_half4(go), zero, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) gh2[v] = h2[v] > 0.0f ? gh2[v] : 0.0f;
        float4_t gh1 = __builtin_amdgcn_mfma_f32_16x16x16f16(w2t, to_half4(gh2), zero, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) gh1[v] = h1[v] > 0.0f ? gh1[v] : 0.0f;
        const float4_t gx = __builtin_amdgcn_mfma_f32_16x16x16f16(w1t, to_half4(gh1), zero, 0, 0, 0);
        float* sr = stage + ray * kStageRow;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            sr[kSH1 + rq + v] = use * h1[v];
            sr[kSH2 + rq + v] = use * h2[v];
            sr[kSGh2 + rq + v] = gh2[v];
            sr[kSGh1 + rq + v] = gh1[v];
            if (lane < 16) sr[kSGo + v] = go[v];
        }
        // g_C = g_rgb + gx[0:3], g_V = gx[3:7]: rows 0..3 sit in lanes 0..15,
        // rows 4..7 in lanes 16..31
        const int64_t i = base + ray;
        if (i < a.n_rays && lane < 32) {
            float4* gcv = reinterpret_cast<float4*>(a.gcv) + 2 * i;
            if (lane < 16)
                gcv[0] = make_float4(gsm[ray * 4 + 0] + gx[0], gsm[ray * 4 + 1] + gx[1], gsm[ray * 4 + 2] + gx[2], gx[3]);
            else
                gcv[1] = make_float4(gx[0], gx[1], gx[2], 0.0f);
        }
    }
}

// F16: the MLP chain (forward and backward through the three layers) runs as
// v_mfma_f32_16x16x16_f16 tiles over the wavefront's 64 rays (FP16 operands,
// FP32 accumulation); the per-ray activations and gradients land in the same
// staging rows as in the FP32 path, and the weight gradients are summed by
// the same FP32 MFMA outer products.
template <bool F16>
__global__ __launch_bounds__(64 * kBwdWaves) void k_mlp_backward(BackwardArgs a) {
    __shared__ float stage[kBwdWaves][64][kStageRow];
    __shared__ _Float16 xs[F16 ? kBwdWaves : 1][64][kXRow];
    __shared__ float gsm[F16 ? kBwdWaves : 1][64][4];  // g_rgb (3), gate
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    cfloat* W = as_const(a.mlp);
    float* me = &stage[wave][lane][0];
    const float* st = &stage[wave][0][0];
    const int li = lane & 15, lk = lane >> 4;

    float4v acc1[3] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    float4v acc2 = {0.f, 0.f, 0.f, 0.f}, acc3 = {0.f, 0.f, 0.f, 0.f};
    float db2 = 0.f, db3 = 0.f;  // lane j < 16 / < 3 holds the sum

    const int64_t stride = int64_t(gridDim.x) * kBwdWaves * 64;
    for (int64_t base = (int64_t(blockIdx.x) * kBwdWaves + wave) * 64; base < a.n_rays; base += stride) {
        const int64_t i = base + lane;
        const bool valid = i < a.n_rays;
        float C[3] = {0.f, 0.f, 0.f}, V[4] = {0.f, 0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
        float gr[4] = {0.f, 0.f, 0.f, 0.f};
        bool gate = false;
        if (valid) {
            const int64_t r = a.ray_ids ? a.ray_ids[i] : i;
            int ci, px, py;
            locate(a, r, ci, px, py);
            int64_t o[3];
            int32_t s[3];
            ray_setup(a.cams[ci], a.grid.N, px, py, o, s, d);
            const float4 a0 = reinterpret_cast<const float4*>(a.aux)[2 * i];
            const float4 a1 = reinterpret_cast<const float4*>(a.aux)[2 * i + 1];
            C[0] = a0.x; C[1] = a0.y; C[2] = a0.z; V[0] = a0.w;
            V[1] = a1.x; V[2] = a1.y; V[3] = a1.z;
            gate = a1.w >= 0.0f;
            const float4 gg = reinterpret_cast<const float4*>(a.grad_rgba)[i];
            gr[0] = gg.x; gr[1] = gg.y; gr[2] = gg.z; gr[3] = gg.w;
        }
        const bool use = valid && gate;

        // forward, staging x, h1, h2 for the weight gradients
        float x[kMlpIn];
        encode_x(C, V, d, x);
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q) me[kSX + q] = x[q];
        me[kSX + 34] = use ? 1.0f : 0.0f;
        me[kSX + 35] = 0.0f;
        if (F16) {
#pragma unroll
            for (int q = 0; q < kXPad; ++q) xs[F16 ? wave : 0][lane][q] = _Float16(q < kMlpIn ? x[q] : 0.0f);
            gsm[F16 ? wave : 0][lane][0] = gr[0];
            gsm[F16 ? wave : 0][lane][1] = gr[1];
            gsm[F16 ? wave : 0][lane][2] = gr[2];
            gsm[F16 ? wave : 0][lane][3] = use ? 1.0f : 0.0f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            mlp_backward_f16_wave(a, W, &xs[F16 ? wave : 0][0][0], &gsm[F16 ? wave : 0][0][0],
                                  &stage[wave][0][0], base, lane);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < kMlpH) {
                float t = 0.f;
                for (int r = 0; r < 64; ++r) t += st[r * kStageRow + kSGh2 + lane];
                db2 += t;
            }
            if (lane < kMlpOut) {
                float t = 0.f;
                for (int r = 0; r < 64; ++r) t += st[r * kStageRow + kSGo + lane];
                db3 += t;
            }
        } else {
        float h2[kMlpH];
#pragma unroll
        for (int k = 0; k < kMlpH; ++k) h2[k] = W[kOffB2 + k];
#pragma nounroll
        for (int j = 0; j < kMlpH; ++j) {
            float t = W[kOffB1 + j];
#pragma unroll
            for (int q = 0; q < kMlpIn; ++q) t = fmaf(W[kOffW1 + j * kMlpIn + q], x[q], t);
            const float h1j = fmaxf(t, 0.0f);
            me[kSH1 + j] = use ? h1j : 0.0f;
#pragma unroll
            for (int k = 0; k < kMlpH; ++k) h2[k] = fmaf(W[kOffW2 + k * kMlpH + j], h1j, h2[k]);
        }
#pragma unroll
        for (int k = 0; k < kMlpH; ++k) {
            h2[k] = fmaxf(h2[k], 0.0f);
            me[kSH2 + k] = use ? h2[k] : 0.0f;
        }
        float go[kMlpOut];
#pragma unroll
        for (int j = 0; j < kMlpOut; ++j) {
            float t = W[kOffB3 + j];
#pragma unroll
            for (int q = 0; q < kMlpH; ++q) t = fmaf(W[kOffW3 + j * kMlpH + q], h2[q], t);
            const float R = sigmoid_f32(t);
            go[j] = use ? gr[j] * R * (1.0f - R) : 0.0f;
            me[kSGo + j] = go[j];
        }
        me[kSGo + 3] = 0.0f;
        // backward through layers 3 and 2 (the ReLU masks come from h2, h1)
#pragma unroll
        for (int q = 0; q < kMlpH; ++q) {
            float t = 0.f;
#pragma unroll
            for (int j = 0; j < kMlpOut; ++j) t = fmaf(W[kOffW3 + j * kMlpH + q], go[j], t);
            h2[q] = h2[q] > 0.0f ? t : 0.0f;  // h2 now holds gh2
            me[kSGh2 + q] = h2[q];
        }
        float gx[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma nounroll
        for (int j = 0; j < kMlpH; ++j) {
            float t = 0.f;
#pragma unroll
            for (int k = 0; k < kMlpH; ++k) t = fmaf(W[kOffW2 + k * kMlpH + j], h2[k], t);
            const float gh1j = me[kSH1 + j] > 0.0f ? t : 0.0f;
            me[kSGh1 + j] = gh1j;
#pragma unroll
            for (int q = 0; q < 7; ++q) gx[q] = fmaf(W[kOffW1 + j * kMlpIn + q], gh1j, gx[q]);
        }
        if (valid) {
            float4* gcv = reinterpret_cast<float4*>(a.gcv) + 2 * i;
            gcv[0] = make_float4(gr[0] + gx[0], gr[1] + gx[1], gr[2] + gx[2], gx[3]);
            gcv[1] = make_float4(gx[4], gx[5], gx[6], 0.0f);
        }
#pragma unroll
        for (int q = 0; q < kMlpH; ++q) {
            const float sq = wave_sum(h2[q]);
            if (lane == q) db2 += sq;
        }
#pragma unroll
        for (int q = 0; q < kMlpOut; ++q) {
            const float sq = wave_sum(go[q]);
            if (lane == q) db3 += sq;
        }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // dW = sum_r gA_r (x) act_r as 16x16x4 FP32 MFMAs: A = gradient rows
        // (16 x 4 rays), B = activations (4 rays x 16); D lane l holds row
        // 4(l/16) + v, column l % 16.
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const float* rr = st + (4 * kk + lk) * kStageRow;
            const float a1v = rr[kSGh1 + li];
#pragma unroll
            for (int nt = 0; nt < 3; ++nt) {
                const int col = 16 * nt + li;
                const float bv = col < 36 ? rr[kSX + col] : 0.0f;
                acc1[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1v, bv, acc1[nt], 0, 0, 0);
            }
            acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(rr[kSGh2 + li], rr[kSH1 + li], acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(li < 4 ? rr[kSGo + li] : 0.0f, rr[kSH2 + li], acc3, 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // this wavefront's partial MLP gradient, in parameter order
    float* out = a.g_mlp_partial + (int64_t(blockIdx.x) * kBwdWaves + wave) * kMlpParams;
    const int lr = 4 * (lane >> 4);
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

// --------------------------------------------------------------- K2: march

// Canonical gradient slot of padded corner voxel (vx, vy, vz) (local
// coordinates in [-1, B]) of the block with atlas id `id` at block
// coordinates b.  Voxels outside the grid or in empty blocks are structural
// zeros and have no slot (-1).
__device__ __forceinline__ int64_t canonical_voxel(const GridArgs& g, int32_t id, const int32_t b[3],
                                                   int vx, int vy, int vz, int32_t& nb_lin, int32_t& nb_id) {
    const int B = g.B;
    int32_t tid = id;
    if (tid < 0 || tid >= g.n_blocks) return -1;
    if (vx < 0 || vy < 0 || vz < 0 || vx >= B || vy >= B || vz >= B) {
        const int nx = b[0] + (vx < 0 ? -1 : (vx >= B ? 1 : 0));
        const int ny = b[1] + (vy < 0 ? -1 : (vy >= B ? 1 : 0));
        const int nz = b[2] + (vz < 0 ? -1 : (vz >= B ? 1 : 0));
        if (nx < 0 || ny < 0 || nz < 0 || nx >= g.G || ny >= g.G || nz >= g.G) return -1;
        // the last neighbour looked up (a ray runs along a face for a while)
        const int32_t nlin = (nz * g.G + ny) * g.G + nx;
        if (nlin != nb_lin) {
            nb_lin = nlin;
            nb_id = g.ind[nlin];
        }
        tid = nb_id;
        if (tid < 0 || tid >= g.n_blocks) return -1;
        vx &= B - 1;
        vy &= B - 1;
        vz &= B - 1;
    }
    return int64_t(tid) * B * B * B + (int64_t(vz) * B + vy) * B + vx;
}

// Running gradient sums for the 8 corner voxels of the ray's current cell.
struct CellWindow {
    int32_t c[3];  // padded cell coordinates
    int32_t rank;  // block record, -1 when empty
    int32_t id;    // atlas id of the block
    int32_t b[3];  // block coordinates
    float A[8], D[8];
};

// Per-wavefront gradient aggregation in LDS.  The rays of an 8x8 pixel tile
// share most of the voxels they touch, so each voxel's eight gradient values
// (density, RGB, features) are first summed in an open-addressed table of
// kAggSlots entries and reach device memory with one set of atomics per
// table flush instead of one per ray.  Keys are canonical voxel indices
// (< 2^31; the launch falls back to direct atomics otherwise).
//
// The colour and feature sums are kept in 32-bit fixed point: on gfx950 an
// LDS float add (ds_add_f32) retires about one lane every three cycles, an
// LDS integer add (ds_add_u32) more than forty times faster.  A ray hands a
// voxel its colour gradient A g_C with A = sum_k w_c(k) w_k, and the A of all
// of a ray's hand-overs add up to at most sum_k w_k <= 1, so with
// M = max over the wavefront's rays of |g_C|, |g_V| all that one ray hands to
// one voxel is at most M and a table entry (64 rays between flushes) at most
// 64 M.  Values are scaled by 2^S, the largest power of two with M 2^S < 2^24,
// and rounded to integers: an entry stays below 2^30 (plus its rounding),
// and each hand-over carries a rounding error of at most 2^-24 M.  The
// density sums, whose size depends on the grid values, stay in float.
constexpr int kAggSlots = 512;
constexpr int kAggLog = 9;
constexpr int kAggProbes = 16;
// Flush once this many keys are in.  Every flush sends each held voxel's
// eight sums to device memory as float atomics, which gfx950 executes at the
// memory side, about 21 G cache lines per second, so the fewer flushes the
// better: at 7/8 full the adjoint frame runs 18% faster than at 1/2 (the
// table then holds most of a tile's voxels at once); a key that finds no
// free slot within kAggProbes probes goes to device memory directly.
constexpr int kAggFlushAt = kAggSlots * 7 / 8;
constexpr int kAggWaves = 4;                 // wavefronts per workgroup
constexpr int kAggWords = kAggSlots * 9;     // keys, 8 value planes
// dynamic LDS of the re-march kernels after the occupancy words: kAggWaves tables
constexpr int kAggLdsWords = kAggWaves * kAggWords;

struct AggTable {
    int32_t* key;  // [kAggSlots], -1 = free
    float* val;    // [8][kAggSlots]: plane 0 float (density), planes 1..7 int32 fixed point
    float q;       // wave-uniform 2^S: fixed-point scale of the colour and feature planes
    float dq;      // 2^-S
};

// The same LDS as an append-only log, for rays that share few voxels
// (scattered ray lists): entry e holds a key and its eight float values,
// written once, with no probing and no LDS atomics (AdjointRay::commit
// places the entries).  Flushed by cache line as the table is.

// Fixed-point scale for a wavefront whose largest |g_C|, |g_V| is m (m >= 0,
// the same value in every lane): 2^S with m 2^S < 2^24 <= 2 m 2^S.
__device__ __forceinline__ void agg_scale(AggTable& t, float m) {
    int e = 0;
    (void)__builtin_frexpf(m, &e);  // 2^(e-1) <= m < 2^e
    int sh = 24 - e;
    sh = m > 0.0f ? (sh < 126 ? (sh > -126 ? sh : -126) : 126) : 0;
    t.q = __builtin_ldexpf(1.0f, sh);
    t.dq = __builtin_ldexpf(1.0f, -sh);
}

__device__ __forceinline__ void add_global(const BackwardArgs& a, int64_t vi, const float v[8], bool feat) {
    if (a.grad_packed) {
        float* g = a.grad_dens + 8 * vi;
        for (int c = 0; c < (feat ? 8 : 4); ++c) unsafeAtomicAdd(g + c, v[c]);
        return;
    }
    unsafeAtomicAdd(a.grad_dens + vi, v[0]);
    unsafeAtomicAdd(a.grad_rgb + 3 * vi + 0, v[1]);
    unsafeAtomicAdd(a.grad_rgb + 3 * vi + 1, v[2]);
    unsafeAtomicAdd(a.grad_rgb + 3 * vi + 2, v[3]);
    if (feat) {
        unsafeAtomicAdd(a.grad_feat + 4 * vi + 0, v[4]);
        unsafeAtomicAdd(a.grad_feat + 4 * vi + 1, v[5]);
        unsafeAtomicAdd(a.grad_feat + 4 * vi + 2, v[6]);
        unsafeAtomicAdd(a.grad_feat + 4 * vi + 3, v[7]);
    }
}

// Adds v to the table entry of `key` (lanes may diverge); false when no slot
// was found within kAggProbes probes.  `fresh` counts the lane's new keys.
__device__ __forceinline__ bool agg_add(const AggTable& t, int32_t key, const float v[8], bool feat, int& fresh) {
    const uint32_t h = (uint32_t(key) * 2654435761u) >> (32 - kAggLog);
    for (int pr = 0; pr < kAggProbes; ++pr) {
        const uint32_t sl = (h + pr) & (kAggSlots - 1);
        // one round trip per probe: the compare-and-swap claims a free slot
        // and otherwise returns the key that holds it
        int32_t k = atomicCAS(t.key + sl, -1, key);
        if (k == -1) {
            ++fresh;
            k = key;
        }
        if (k == key) {
            const int nv = feat ? 8 : 4;
            atomicAdd(t.val + sl, v[0]);
            int32_t* iv = reinterpret_cast<int32_t*>(t.val);
            for (int c = 1; c < nv; ++c) atomicAdd(iv + c * kAggSlots + sl, int32_t(__builtin_rintf(v[c] * t.q)));
            return true;
        }
    }
    return false;
}

// The device address of channel c (0 density, 1..3 RGB, 4..7 features) of
// voxel key in the three separate gradient arrays.
__device__ __forceinline__ float* grad_channel(const BackwardArgs& a, int32_t key, int c) {
    return c == 0 ? a.grad_dens + key
                  : (c < 4 ? a.grad_rgb + 3 * int64_t(key) + (c - 1) : a.grad_feat + 4 * int64_t(key) + (c - 4));
}

// All 64 lanes together: the log's first n entries go to device memory and
// the log is emptied.  Lanes are laid across each entry's channels as in
// agg_flush.
template <bool FEAT>
__device__ __forceinline__ void log_flush(const BackwardArgs& a, const AggTable& t, int lane, int n) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (a.grad_packed) {
        constexpr int kC = FEAT ? 8 : 4;  // lanes per entry, one channel each
        const int c = lane % kC;
        for (int e = lane / kC; e < n; e += 64 / kC) {
            const float v = t.val[c * kAggSlots + e];
            if (v != 0.0f) unsafeAtomicAdd(a.grad_dens + 8 * int64_t(t.key[e]) + c, v);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        return;
    }
    const int c = lane & 3;
    for (int e = lane >> 2; e < n; e += 16) {
        const int32_t key = t.key[e];
        const float v0 = t.val[c * kAggSlots + e];
        if (v0 != 0.0f) unsafeAtomicAdd(grad_channel(a, key, c), v0);
        if (FEAT) {
            const float v1 = t.val[(c + 4) * kAggSlots + e];
            if (v1 != 0.0f) unsafeAtomicAdd(grad_channel(a, key, c + 4), v1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// All 64 lanes together: every used entry goes to device memory, the table
// is cleared.  gfx950 serves a wavefront's float atomics per 64-byte line
// (measured: about 21 G lines per second whether a line carries one lane's
// add or sixteen), so the lanes are laid across the entries' channels, not
// the entries: lane l takes entry l / 4 of a group of 16 and within it
// channels l % 4 and l % 4 + 4, so that one instruction adds an entry's
// density and colour (two lines) and the next its four features (one
// line), where one lane per entry would touch seven lines.  With packed
// gradients an entry's eight sums share one line: eight lanes per entry (four
// without features), one instruction per group.
template <bool FEAT>
__device__ __forceinline__ void agg_flush(const BackwardArgs& a, const AggTable& t, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    int32_t* iv = reinterpret_cast<int32_t*>(t.val);
    if (a.grad_packed) {
        constexpr int kC = FEAT ? 8 : 4;
        const int c = lane % kC;
        for (int sl = lane / kC; sl < kAggSlots; sl += 64 / kC) {
            const int32_t key = t.key[sl];
            if (key >= 0) {
                float v;
                if (c == 0) {
                    v = t.val[sl];
                    t.val[sl] = 0.0f;
                } else {
                    v = float(iv[c * kAggSlots + sl]) * t.dq;
                    iv[c * kAggSlots + sl] = 0;
                }
                if (v != 0.0f) unsafeAtomicAdd(a.grad_dens + 8 * int64_t(key) + c, v);
            }
        }
    } else {
        const int c = lane & 3;
        for (int sl = lane >> 2; sl < kAggSlots; sl += 16) {
            const int32_t key = t.key[sl];
            if (key >= 0) {
                float v0;
                if (c == 0) {
                    v0 = t.val[sl];
                    t.val[sl] = 0.0f;
                } else {
                    v0 = float(iv[c * kAggSlots + sl]) * t.dq;
                    iv[c * kAggSlots + sl] = 0;
                }
                if (v0 != 0.0f) unsafeAtomicAdd(grad_channel(a, key, c), v0);
                if (FEAT) {
                    const float v1 = float(iv[(c + 4) * kAggSlots + sl]) * t.dq;
                    iv[(c + 4) * kAggSlots + sl] = 0;
                    if (v1 != 0.0f) unsafeAtomicAdd(grad_channel(a, key, c + 4), v1);
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int sl = lane; sl < kAggSlots; sl += 64) t.key[sl] = -1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return __builtin_amdgcn_readfirstlane(v);
}

template <bool FEAT, bool AGG>
__device__ __forceinline__ void flush_corner(const BackwardArgs& a, const AggTable& t, const CellWindow& w, int c,
                                             const float gC[3], const float gV[4], int& fresh, int32_t& nb_lin,
                                             int32_t& nb_id) {
    const float A = w.A[c], D = w.D[c];
    if (A == 0.0f && D == 0.0f) return;
    const GridArgs& g = a.grid;
    const int64_t vi = canonical_voxel(g, w.id, w.b, w.c[0] + (c & 1) - 1, w.c[1] + ((c >> 1) & 1) - 1,
                                       w.c[2] + (c >> 2) - 1, nb_lin, nb_id);
    if (vi < 0) return;
    float v[8] = {g.sigma_scale * D, A * gC[0], A * gC[1], A * gC[2], 0.f, 0.f, 0.f, 0.f};
    if (FEAT) {
        v[4] = A * gV[0]; v[5] = A * gV[1]; v[6] = A * gV[2]; v[7] = A * gV[3];
    }
    if (AGG && agg_add(t, int32_t(vi), v, FEAT, fresh)) return;
    add_global(a, vi, v, FEAT);
}

// The adjoint state of one ray's re-march: its output gradient and the
// forward's per-ray results (E, the T_N tail), the running transmittance T
// and prefix P_k, and the corner window.  sample() takes the samples in
// march order, as march_ray hands them over (inactive ones included), and
// returns true once the early-stop rule ends the ray; finish() hands over
// the last window.
template <bool FEAT, bool AGG, bool LOG = false>
struct AdjointRay {
    float gC[3], gV[4];
    float E, tail, T, Pk;
    float delta, kx, t_stop;
    bool early, nn_gate;
    CellWindow win;
    int fresh;  // this lane's new table keys since the last count
    int32_t nb_lin, nb_id;  // the last neighbouring block looked up: linear index, atlas id
    // LOG: the corners handed over since the last commit, by corner index
    uint32_t pmask;
    int32_t pvi[8];
    float pA[8], pD[8];

    // Reads list position i's state; false when the ray composited nothing
    // (no grid gradient) or `live` is false.
    __device__ __forceinline__ bool setup(const BackwardArgs& a, int64_t i, bool live) {
        float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = make_float4(0.f, 0.f, 0.f, -1.f);
        float4 gg = make_float4(0.f, 0.f, 0.f, 0.f);
        if (live) {
            a1 = reinterpret_cast<const float4*>(a.aux)[2 * i + 1];
            live = a1.w >= 0.0f;  // nothing was composited: no grid gradient
        }
        gC[0] = gC[1] = gC[2] = 0.f;
        gV[0] = gV[1] = gV[2] = gV[3] = 0.f;
        if (live) {
            a0 = reinterpret_cast<const float4*>(a.aux)[2 * i];
            gg = reinterpret_cast<const float4*>(a.grad_rgba)[i];
            gC[0] = gg.x; gC[1] = gg.y; gC[2] = gg.z;
            if (FEAT) {
                const float4 c0 = reinterpret_cast<const float4*>(a.gcv)[2 * i];
                const float4 c1 = reinterpret_cast<const float4*>(a.gcv)[2 * i + 1];
                gC[0] = c0.x; gC[1] = c0.y; gC[2] = c0.z;
                gV[0] = c0.w; gV[1] = c1.x; gV[2] = c1.y; gV[3] = c1.z;
            }
        }
        E = gC[0] * a0.x + gC[1] * a0.y + gC[2] * a0.z + (gV[0] * a0.w + gV[1] * a1.x + gV[2] * a1.y + gV[3] * a1.z);
        const float gTN = gg.x * a.opts.bg[0] + gg.y * a.opts.bg[1] + gg.z * a.opts.bg[2] - gg.w;
        tail = a1.w * gTN;
        T = 1.0f;
        Pk = 0.0f;
        delta = 1.0f / float(a.grid.N);
        kx = a.grid.sigma_scale * delta;
        t_stop = a.opts.t_stop;
        early = a.opts.early_stop != 0;
        nn_gate = a.opts.nn_gate != 0;
        win.rank = -1;
        win.id = 0;
        win.c[0] = win.c[1] = win.c[2] = 0;
        win.b[0] = win.b[1] = win.b[2] = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) win.A[c] = win.D[c] = 0.0f;
        fresh = 0;
        pmask = 0;
        nb_lin = -1;
        nb_id = -1;
        return live;
    }

    // LOG: keeps corner c's hand-over (lanes may diverge) for commit().
    __device__ __forceinline__ void stash(const GridArgs& g, int c) {
        const float A = win.A[c], D = win.D[c];
        if (A == 0.0f && D == 0.0f) return;
        const int64_t vi = canonical_voxel(g, win.id, win.b, win.c[0] + (c & 1) - 1, win.c[1] + ((c >> 1) & 1) - 1,
                                           win.c[2] + (c >> 2) - 1, nb_lin, nb_id);
        if (vi < 0) return;
        pvi[c] = int32_t(vi);  // LOG runs only on grids of fewer than 2^31 voxels
        pA[c] = A;
        pD[c] = D;
        pmask |= 1u << c;
    }

    // LOG, all 64 lanes together: appends the stashed hand-overs to the log,
    // corner by corner.  The lanes appending a corner take the next entries
    // in lane order (a ballot and a prefix count), so the fill count n stays
    // the same in every lane and nothing needs an LDS atomic; the log is
    // flushed whenever another corner might not fit.
    template <bool F>
    __device__ __forceinline__ void commit(const BackwardArgs& a, const AggTable& t, int lane, int& n) {
        const GridArgs& g = a.grid;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const bool want = (pmask >> c) & 1u;
            const uint64_t m = __ballot(want);
            if (m == 0) continue;  // wave-uniform
            if (n > kAggSlots - 64) {
                log_flush<F>(a, t, lane, n);
                n = 0;
            }
            if (want) {
                const int e = n + int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
                const float A = pA[c];
                t.key[e] = pvi[c];
                t.val[e] = g.sigma_scale * pD[c];
                t.val[kAggSlots + e] = A * gC[0];
                t.val[2 * kAggSlots + e] = A * gC[1];
                t.val[3 * kAggSlots + e] = A * gC[2];
                if (F) {
                    t.val[4 * kAggSlots + e] = A * gV[0];
                    t.val[5 * kAggSlots + e] = A * gV[1];
                    t.val[6 * kAggSlots + e] = A * gV[2];
                    t.val[7 * kAggSlots + e] = A * gV[3];
                }
            }
            n += __builtin_popcountll(m);
        }
        pmask = 0;
    }

    // Wavefront-wide (all 64 lanes, the same value in each): the largest
    // |g_C|, |g_V| sets the table's fixed-point scale.
    __device__ __forceinline__ void table_scale(AggTable& tab) const {
        float m = fmaxf(fmaxf(fabsf(gC[0]), fabsf(gC[1])), fmaxf(fabsf(gC[2]), fabsf(gV[0])));
        m = fmaxf(m, fmaxf(fmaxf(fabsf(gV[1]), fabsf(gV[2])), fabsf(gV[3])));
#pragma unroll
        for (int sh = 32; sh >= 1; sh >>= 1) m = fmaxf(m, __shfl_xor(m, sh));
        agg_scale(tab, m);  // the butterfly leaves the same maximum in every lane
    }

    __device__ __forceinline__ bool sample(const BackwardArgs& a, const AggTable& tab, int32_t rk, const uint8_t* vox,
                                           const int32_t p[3], const int32_t fr[3]) {
        Sample smp;
        gather_f32(vox, a.grid.Bp, p, fr, smp, nn_gate);
        return take(a, tab, rk, smp, p, fr);
    }

    // The sample with its corners already interpolated.
    __device__ __forceinline__ bool take(const BackwardArgs& a, const AggTable& tab, int32_t rk, const Sample& smp,
                                         const int32_t p[3], const int32_t fr[3]) {
        const GridArgs& g = a.grid;
        if (!smp.active) return false;
        const float e = __expf(-smp.sigma_raw * kx);
        const float w = T * (1.0f - e);
        const float ek = gC[0] * smp.rgb[0] + gC[1] * smp.rgb[1] + gC[2] * smp.rgb[2] +
                         (gV[0] * smp.feat[0] + gV[1] * smp.feat[1] + gV[2] * smp.feat[2] + gV[3] * smp.feat[3]);
        Pk += w * ek;
        T *= e;
        const float gsig = delta * (T * ek - (E - Pk) - tail);
        // Slide the corner window to this sample's cell: corners on a
        // trailing face (or all of them after a jump) are flushed once, the
        // survivors shift to their new corner index.
        const bool jump = win.rank != rk || abs(p[0] - win.c[0]) > 1 || abs(p[1] - win.c[1]) > 1 ||
                          abs(p[2] - win.c[2]) > 1;
        int dd[3] = {p[0] - win.c[0], p[1] - win.c[1], p[2] - win.c[2]};
        uint32_t leave = 0;
        if (jump) {
            leave = win.rank >= 0 ? 0xFFu : 0u;
        } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                // corners with bit ax clear: 0x55, 0x33, 0x0F for ax = 0, 1, 2
                const uint32_t clear = ax == 0 ? 0x55u : (ax == 1 ? 0x33u : 0x0Fu);
                if (dd[ax] > 0) leave |= clear;
                if (dd[ax] < 0) leave |= ~clear & 0xFFu;
            }
        }
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if ((leave >> c) & 1u) {
                if (LOG) stash(g, c);
                else flush_corner<FEAT, AGG>(a, tab, win, c, gC, gV, fresh, nb_lin, nb_id);
            }
        if (jump) {
#pragma unroll
            for (int c = 0; c < 8; ++c) win.A[c] = win.D[c] = 0.0f;
            win.rank = rk;
            win.id = g.rank_id[rk];
            const int32_t lin = g.rank_lin[rk];
            win.b[0] = lin % g.G;
            win.b[1] = (lin / g.G) % g.G;
            win.b[2] = lin / (g.G * g.G);
            win.c[0] = p[0]; win.c[1] = p[1]; win.c[2] = p[2];
        } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int bit = 1 << ax;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (c & bit) continue;
                    const int c1 = c | bit;
                    const float a0v = win.A[c], d0v = win.D[c], a1v = win.A[c1], d1v = win.D[c1];
                    win.A[c] = dd[ax] > 0 ? a1v : (dd[ax] < 0 ? 0.0f : a0v);
                    win.D[c] = dd[ax] > 0 ? d1v : (dd[ax] < 0 ? 0.0f : d0v);
                    win.A[c1] = dd[ax] < 0 ? a0v : (dd[ax] > 0 ? 0.0f : a1v);
                    win.D[c1] = dd[ax] < 0 ? d0v : (dd[ax] > 0 ? 0.0f : d1v);
                }
                win.c[ax] += dd[ax];
            }
        }
        float wc[8];
        corner_weights(fr, wc);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            win.A[c] = fmaf(wc[c], w, win.A[c]);
            win.D[c] = fmaf(wc[c], gsig, win.D[c]);
        }
        return early && T < t_stop;
    }

    __device__ __forceinline__ void finish(const BackwardArgs& a, const AggTable& tab) {
        if (win.rank >= 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (LOG) stash(a.grid, c);
                else flush_corner<FEAT, AGG>(a, tab, win, c, gC, gV, fresh, nb_lin, nb_id);
            }
        }
    }
};

// The table of the calling wavefront in dynamic LDS (after the occupancy
// words), cleared.
__device__ __forceinline__ AggTable agg_table(uint2* s_occ, int n_words, int wave, int lane, bool clear) {
    AggTable tab;
    int32_t* base = reinterpret_cast<int32_t*>(s_occ + n_words) + wave * kAggWords;
    tab.key = base;
    tab.val = reinterpret_cast<float*>(base + kAggSlots);
    if (clear) {
        for (int sl = lane; sl < kAggSlots; sl += 64) {
            tab.key[sl] = -1;
#pragma unroll
            for (int c = 0; c < 8; ++c) tab.val[c * kAggSlots + sl] = 0.0f;
        }
    }
    return tab;
}

// Wavefront-wide, after each step of the lanes: counts the table's new keys
// and flushes it once it is full enough.
struct TableSync {
    int in_table = 0;  // wave-uniform: keys in the table
    template <bool FEAT>
    __device__ __forceinline__ void step(const BackwardArgs& a, const AggTable& tab, int lane, int& fresh) {
        if (__any(fresh != 0)) {
            in_table += wave_sum_i32(fresh);
            fresh = 0;
            if (in_table >= kAggFlushAt) {
                agg_flush<FEAT>(a, tab, lane);
                in_table = 0;
            }
        }
    }
};

// One lane per ray.  Without a ray list the wavefronts walk the cameras'
// tt_w x tt_h pixel tiles (neighbouring rays, shared voxels); with a list,
// 64 consecutive list entries.  AGG: gradients go through the per-wavefront
// LDS table.  Every lane stays to the end (the flushes need all 64).
template <bool FEAT, bool AGG>
__global__ __launch_bounds__(64 * kAggWaves) void k_march_backward(BackwardArgs a) {
    extern __shared__ uint2 s_occ[];
    const GridArgs& g = a.grid;
    for (int w = threadIdx.x; w < g.n_words; w += blockDim.x) s_occ[w] = g.occ[w];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    AggTable tab = agg_table(s_occ, g.n_words, wave, lane, AGG);
    __syncthreads();

    // this lane's ray: list position i (indexes aux, grad_rgba, gcv) and id r
    bool live;
    int64_t i, r;
    const int64_t wt = int64_t(a.ray_ids ? blockIdx.x : xcd_grouped(blockIdx.x, gridDim.x)) * kAggWaves + wave;
    if (a.ray_ids) {
        i = wt * 64 + lane;
        live = i < a.n_rays;
        r = live ? a.ray_ids[i] : 0;
    } else {
        live = wt < a.total_tiles;
        i = r = 0;
        if (live) {
            const int ci = find_camera_by_tile(a.cams, a.n_cams, wt);
            const DevCamera& c = a.cams[ci];
            const int64_t tl = wt - c.tile_offset;
            const int px = int(tl % c.tiles_x) * a.tile_w + lane % a.tile_w;
            const int py = int(tl / c.tiles_x) * a.tile_h + lane / a.tile_w;
            live = px < c.W && py < c.H;
            i = r = c.ray_offset + int64_t(py) * c.W + px;
        }
    }
    AdjointRay<FEAT, AGG> st;
    live = st.setup(a, i, live);
    if (AGG) st.table_scale(tab);

    int64_t o[3] = {0, 0, 0};
    int32_t s[3] = {0, 0, 1 << 15};
    if (live) {
        int ci, px, py;
        locate(a, r, ci, px, py);
        float d[3];
        ray_setup(a.cams[ci], g.N, px, py, o, s, d);
    }
    TableSync sync;
    march_ray_flat_sync(
        g, s_occ, live, o, s,
        [&](int64_t, int32_t rk, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
            return st.sample(a, tab, rk, vox, p, fr);
        },
        [&]() {
            if (AGG) sync.step<FEAT>(a, tab, lane, st.fresh);
            return false;
        });
    st.finish(a, tab);
    if (AGG) agg_flush<FEAT>(a, tab, lane);
}

// Short ray lists in two phases.  With few rays the wavefronts are few and
// the backward is as slow as its slowest wavefront, whose 64 rays march in
// lock step: at nearly every step some lane takes a sample, so every step
// pays for the whole gradient code.  Phase 1 (k_backward_record) walks each
// ray alone and lists the samples the walk hands over (cell position and
// macroblock record: cells with a zero distance byte, nearly all of them
// active; the gradient code decides); phase 2
// (k_backward_from_list) runs the gradient code over the lists, one listed
// sample per lane per step, with the same per-ray arithmetic in the same
// order as k_march_backward.  A ray with more than kBackwardListCap listed
// samples walks on from its start in phase 2, skipping the listed ones.
constexpr int kListCap = kBackwardListCap;

__global__ __launch_bounds__(256) void k_backward_record(BackwardArgs a, int4* __restrict__ list,
                                                         int32_t* __restrict__ count, int64_t* __restrict__ klast) {
    extern __shared__ uint2 s_occ[];
    const GridArgs& g = a.grid;
    for (int w = threadIdx.x; w < g.n_words; w += blockDim.x) s_occ[w] = g.occ[w];
    __syncthreads();
    // a.list_rpw rays per wavefront, as in the gradient pass
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * a.list_rpw + lane;
    if (lane >= a.list_rpw || i >= a.n_rays) return;
    int32_t n = 0;
    int64_t kl = 0;
    // rays that composited nothing have no grid gradient (phase 2 skips them)
    if (reinterpret_cast<const float4*>(a.aux)[2 * i + 1].w >= 0.0f) {
        int ci, px, py;
        locate(a, a.ray_ids[i], ci, px, py);
        int64_t o[3];
        int32_t s[3];
        float d[3];
        ray_setup(a.cams[ci], g.N, px, py, o, s, d);
        int4* mine = list + i * kListCap;
        march_ray_flat(g, s_occ, o, s,
                       [&](int64_t k, int32_t rk, const uint8_t*, const int32_t p[3], const int32_t fr[3]) {
                           if (n < kListCap) {
                               mine[n] = make_int4((p[0] << 16) | fr[0], (p[1] << 16) | fr[1], (p[2] << 16) | fr[2], rk);
                               kl = k;
                           }
                           ++n;
                           return false;
                       });
    }
    count[i] = n;
    klast[i] = kl;
}

template <bool FEAT, bool LOG>
__global__ __launch_bounds__(64 * kAggWaves) void k_backward_from_list(BackwardArgs a, const int4* __restrict__ list,
                                                                       const int32_t* __restrict__ count,
                                                                       const int64_t* __restrict__ klast) {
    extern __shared__ uint2 s_occ[];
    const GridArgs& g = a.grid;
    for (int w = threadIdx.x; w < g.n_words; w += blockDim.x) s_occ[w] = g.occ[w];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    AggTable tab = agg_table(s_occ, g.n_words, wave, lane, true);
    __syncthreads();
    // a.list_rpw rays per wavefront (lanes past them idle)
    const int64_t i = (int64_t(blockIdx.x) * kAggWaves + wave) * a.list_rpw + lane;
    bool live = lane < a.list_rpw && i < a.n_rays;
    AdjointRay<FEAT, true, LOG> st;
    live = st.setup(a, i, live);
    if (!LOG) st.table_scale(tab);
    const int32_t total = live ? count[i] : 0;
    const int32_t n = total < kListCap ? total : kListCap;
    const int4* mine = list + i * kListCap;
    TableSync sync;
    int n_log = 0;  // LOG: entries in the log, the same in every lane
    bool going = live;
    // Software pipeline (at these sizes one wavefront per SIMD, so nothing
    // else hides a step's loads): list entries are read two steps ahead and
    // the next sample's corners are loaded before the current sample's
    // gradient work, in two corner buffers with the loop unrolled by two so
    // that neither is copied.
    const int4 none = make_int4(0, 0, 0, 0);
    int4 e0 = n > 0 ? mine[0] : none;
    int4 e1 = n > 1 ? mine[1] : none;
    CornersF32 cb[2];
    auto load = [&](const int4& e, CornersF32& cn) {
        const int32_t p[3] = {e.x >> 16, e.y >> 16, e.z >> 16};
        load_corners_f32(g.rec + int64_t(e.w) * g.rec_stride + g.dist_bytes, g.Bp, p, cn);
    };
    if (n > 0) load(e0, cb[0]);
    auto step = [&](int32_t j, const int4& e, const CornersF32& cn) {
        if (going && j < n) {
            const int32_t p[3] = {e.x >> 16, e.y >> 16, e.z >> 16};
            const int32_t fr[3] = {e.x & 0xFFFF, e.y & 0xFFFF, e.z & 0xFFFF};
            Sample smp;
            interp_f32(cn, fr, smp, st.nn_gate);
            if (st.take(a, tab, e.w, smp, p, fr)) going = false;
        }
        if (LOG) st.template commit<FEAT>(a, tab, lane, n_log);
        else sync.step<FEAT>(a, tab, lane, st.fresh);
    };
    for (int32_t j = 0; __any(going && j < n); j += 2) {
        if (going && j + 1 < n) load(e1, cb[1]);
        const int4 e2 = going && j + 2 < n ? mine[j + 2] : none;
        step(j, e0, cb[0]);
        if (!__any(going && j + 1 < n)) break;
        if (going && j + 2 < n) load(e2, cb[0]);
        const int4 e3 = going && j + 3 < n ? mine[j + 3] : none;
        step(j + 1, e1, cb[1]);
        e0 = e2;
        e1 = e3;
    }
    // past the list: walk from the start and take the samples after the last listed one
    const bool more = going && total > kListCap;
    if (__any(more)) {
        int64_t o[3] = {0, 0, 0};
        int32_t s[3] = {0, 0, 1 << 15};
        const int64_t k_listed = more ? klast[i] : 0;
        if (more) {
            int ci, px, py;
            locate(a, a.ray_ids[i], ci, px, py);
            float d[3];
            ray_setup(a.cams[ci], g.N, px, py, o, s, d);
        }
        march_ray_flat_sync(
            g, s_occ, more, o, s,
            [&](int64_t k, int32_t rk, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
                return k > k_listed && st.sample(a, tab, rk, vox, p, fr);
            },
            [&]() {
                if (LOG) st.template commit<FEAT>(a, tab, lane, n_log);
                else sync.step<FEAT>(a, tab, lane, st.fresh);
                return false;
            });
    }
    st.finish(a, tab);
    if (LOG) {
        st.template commit<FEAT>(a, tab, lane, n_log);
        log_flush<FEAT>(a, tab, lane, n_log);
    } else {
        agg_flush<FEAT>(a, tab, lane);
    }
}

// Column sums of the [rows][883] partial-gradient matrix into out (which
// holds zeros): each workgroup takes 64 columns x kReduceRows rows, four
// row phases of 64 threads, combines them in LDS and adds its sum to out.
constexpr int kReduceRows = 256;

__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ partial, int rows,
                                                     float* __restrict__ out) {
    __shared__ float part[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + tx;
    const int r0 = blockIdx.y * kReduceRows;
    const int r1 = min(rows, r0 + kReduceRows);
    float acc = 0.f;
    if (col < kMlpParams)
        for (int r = r0 + ty; r < r1; r += 4) acc += partial[int64_t(r) * kMlpParams + col];
    part[ty][tx] = acc;
    __syncthreads();
    if (ty == 0 && col < kMlpParams) atomicAdd(out + col, (part[0][tx] + part[1][tx]) + (part[2][tx] + part[3][tx]));
}

int backward_partial_rows(int n_groups) { return n_groups * kBwdWaves; }

bool backward_aggregates(const GridArgs& g) {
    return int64_t(g.n_blocks) * g.B * g.B * g.B < (int64_t(1) << 31);
}

hipError_t launch_backward(const BackwardArgs& a, int n_groups, hipStream_t s) {
    if (a.n_rays <= 0) return hipSuccess;
    hipError_t e;
    if (a.mlp_mode == kMlpF16) {
        hipLaunchKernelGGL(k_mlp_backward<true>, dim3(n_groups), dim3(64 * kBwdWaves), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (a.mlp_mode == kMlpF32) {
        hipLaunchKernelGGL(k_mlp_backward<false>, dim3(n_groups), dim3(64 * kBwdWaves), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (a.mlp_only) return hipSuccess;
    // aggregation keys are int32 voxel indices
    const int64_t n_vox = int64_t(a.grid.n_blocks) * a.grid.B * a.grid.B * a.grid.B;
    const bool agg = backward_aggregates(a.grid);
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2) + (agg ? size_t(kAggLdsWords) * 4 : 0);
    const int64_t waves = a.ray_ids ? (a.n_rays + 63) / 64 : a.total_tiles;
    const unsigned blocks = unsigned((waves + kAggWaves - 1) / kAggWaves);
    const bool feat = a.mlp_mode != kMlpOff;
    (void)n_vox;
    if (a.list) {  // short ray list: record, then the gradient from the lists
        // A scattered list of up to 2^16 rays fills at most one wavefront
        // per SIMD at 64 rays each, and a lone wavefront waits on its own
        // latencies: with 32 rays (up to 2^16) or 16 (up to 2^15), the other
        // lanes idle, two or more share each SIMD.  Patch lists keep 64, the
        // 8x8 patches whose voxels the table sums.
        BackwardArgs b = a;
        b.list_rpw = a.patch_rays ? 64 : (a.n_rays <= (int64_t(1) << 15) ? 16 : (a.n_rays <= (int64_t(1) << 16) ? 32 : 64));
        const unsigned lblocks = unsigned(((a.n_rays + b.list_rpw - 1) / b.list_rpw + kAggWaves - 1) / kAggWaves);
        const size_t occ = size_t(a.grid.n_words) * sizeof(uint2);
        const unsigned rblocks = unsigned(((a.n_rays + b.list_rpw - 1) / b.list_rpw + 3) / 4);
        hipLaunchKernelGGL(k_backward_record, dim3(rblocks), dim3(256), occ, s, b, b.list, b.list_count,
                           b.list_klast);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // scattered rays share few voxels: the log; patches: the aggregating table
        if (feat && a.patch_rays)
            hipLaunchKernelGGL((k_backward_from_list<true, false>), dim3(lblocks), dim3(64 * kAggWaves), lds, s, b,
                               b.list, b.list_count, b.list_klast);
        else if (feat)
            hipLaunchKernelGGL((k_backward_from_list<true, true>), dim3(lblocks), dim3(64 * kAggWaves), lds, s, b,
                               b.list, b.list_count, b.list_klast);
        else if (a.patch_rays)
            hipLaunchKernelGGL((k_backward_from_list<false, false>), dim3(lblocks), dim3(64 * kAggWaves), lds, s, b,
                               b.list, b.list_count, b.list_klast);
        else
            hipLaunchKernelGGL((k_backward_from_list<false, true>), dim3(lblocks), dim3(64 * kAggWaves), lds, s, b,
                               b.list, b.list_count, b.list_klast);
        return hipGetLastError();
    }
    if (feat && agg)
        hipLaunchKernelGGL((k_march_backward<true, true>), dim3(blocks), dim3(64 * kAggWaves), lds, s, a);
    else if (feat)
        hipLaunchKernelGGL((k_march_backward<true, false>), dim3(blocks), dim3(64 * kAggWaves), lds, s, a);
    else if (agg)
        hipLaunchKernelGGL((k_march_backward<false, true>), dim3(blocks), dim3(64 * kAggWaves), lds, s, a);
    else
        hipLaunchKernelGGL((k_march_backward<false, false>), dim3(blocks), dim3(64 * kAggWaves), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_mlp(const float* partial, int rows, float* out, hipStream_t s) {
    const dim3 grid((kMlpParams + 63) / 64, (rows + kReduceRows - 1) / kReduceRows);
    hipLaunchKernelGGL(k_reduce_rows, grid, dim3(256), 0, s, partial, rows, out);
    return hipGetLastError();
}

}  // namespace snerg
