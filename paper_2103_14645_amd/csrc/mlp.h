// Deferred shading MLP (Eq. 7, Section 4.2): x = [C_d, V, d, PE(d)] (34),
// two ReLU layers of 16 channels, sigmoid output (3).  Weights are the
// 883-float vector W1[16][34] b1 W2[16][16] b2 W3[3][16] b3 ([out][in]).
//
//  - mlp_forward_f32: one ray per lane, FP32 FMAs; wave-uniform weight
//    addresses become scalar loads.
//  - mlp_forward_f16_wave: the 64 rays of a wavefront as MFMA tiles (FP16
//    operands, FP32 accumulation), computing H^T = W X^T with hidden units
//    as rows and 16 rays per column tile: layer 1 as two gfx950
//    v_mfma_f32_16x16x32_f16 tiles (K = 34 padded to 64), layers 2 and 3 as
//    v_mfma_f32_16x16x16_f16.  x is moved into the B-operand layout through
//    LDS; each layer's FP32 result, after bias and ReLU, is already in the
//    next layer's B-operand layout.  Sigmoid stays FP32.
#pragma once

#include "snerg_dev.h"

namespace snerg {

__device__ __forceinline__ void encode_x(const float C[3], const float V[4], const float d[3],
                                         float x[kMlpIn]) {
    x[0] = C[0]; x[1] = C[1]; x[2] = C[2];
    x[3] = V[0]; x[4] = V[1]; x[5] = V[2]; x[6] = V[3];
    x[7] = d[0]; x[8] = d[1]; x[9] = d[2];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const float sc = float(1 << l);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float sn, cn;
            sincospif(sc * d[a], &sn, &cn);  // sin(2^l pi d), cos(2^l pi d)
            x[10 + 6 * l + a] = sn;
            x[13 + 6 * l + a] = cn;
        }
    }
}

__device__ __forceinline__ float sigmoid_f32(float z) { return 1.0f / (1.0f + __expf(-z)); }

// One ray per lane.  Layer 1 runs hidden unit by hidden unit in a rolled
// loop; each h1_j is folded into the 16 layer-2 accumulators as soon as it
// exists, so only x, the accumulators and one weight row are live (the
// weights arrive through scalar loads; unrolled, their hoisting overflows
// the scalar register file).  Summation order per output is unchanged:
// bias first, then inputs in index order.
__device__ __forceinline__ void mlp_forward_f32(cfloat* W, const float C[3],
                                                const float V[4], const float d[3], float R[3]) {
    float x[kMlpIn];
    encode_x(C, V, d, x);
    float h2[kMlpH];
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) h2[k] = W[kOffB2 + k];
#pragma nounroll
    for (int j = 0; j < kMlpH; ++j) {
        cfloat* row = W + kOffW1 + j * kMlpIn;
        float s = W[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) s = fmaf(row[i], x[i], s);
        const float h1j = fmaxf(s, 0.0f);
#pragma unroll
        for (int k = 0; k < kMlpH; ++k) h2[k] = fmaf(W[kOffW2 + k * kMlpH + j], h1j, h2[k]);
    }
#pragma unroll
    for (int k = 0; k < kMlpH; ++k) h2[k] = fmaxf(h2[k], 0.0f);
#pragma unroll
    for (int j = 0; j < kMlpOut; ++j) {
        float s = W[kOffB3 + j];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) s = fmaf(W[kOffW3 + j * kMlpH + i], h2[i], s);
        R[j] = sigmoid_f32(s);
    }
}

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kXPad = 48;              // 34 inputs padded with zeros to 48
constexpr int kXRow = kXPad + 8;       // LDS row stride in halves (112 B: 16-byte aligned, breaks bank alignment)
constexpr int kMaxWavesF16 = 4;

// Tile layouts (lane l, n = l % 16, q = l / 16):
//  v_mfma_f32_16x16x32_f16: A lane l = M[m = n][k = 8q + j], j = 0..7;
//                           B lane l = X[k = 8q + j][n]
//  v_mfma_f32_16x16x16f16:  A lane l = M[m = n][k = 4q + j], j = 0..3;
//                           B lane l = X[k = 4q + j][n]
//  both:                    D lane l = Y[m = 4q + v][n], v = 0..3
// Hidden units are rows and the 16 rays of a column group are columns, so a
// layer's D tile, after bias and ReLU and conversion to half, is the next
// layer's 16x16x16 B operand as it stands.

// A-operand fragment (16x16x16) of a row-major [rows][cols] FP32 matrix for
// the tile at (r0, c0), zero outside [rows, cols).
__device__ __forceinline__ half4_t a_frag(cfloat* M, int rows, int cols, int r0, int c0, int lane) {
    const int r = r0 + (lane & 15);
    const int c = c0 + 4 * (lane >> 4);
    half4_t v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (r < rows && c + j < cols) ? _Float16(M[r * cols + c + j]) : _Float16(0.0f);
    return v;
}

// A-operand fragment (16x16x32) of W1 [16][34] for K chunk kc (inputs 32 kc ..).
__device__ __forceinline__ half8_t a_frag32(cfloat* M, int cols, int kc, int lane) {
    const int r = lane & 15;
    const int c = 32 * kc + 8 * (lane >> 4);
    half8_t v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = c + j < cols ? _Float16(M[r * cols + c + j]) : _Float16(0.0f);
    return v;
}

// Accumulator initialised with a bias: lane l holds rows 4(l/16) + v.
__device__ __forceinline__ float4_t bias_frag(cfloat* b, int rows, int lane) {
    float4_t v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = 4 * (lane >> 4) + j;
        v[j] = r < rows ? b[r] : 0.0f;
    }
    return v;
}

__device__ __forceinline__ half4_t relu_to_half(float4_t v) {
    half4_t h;
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = _Float16(fmaxf(v[j], 0.0f));
    return h;
}

// The network's weights as this lane's MFMA fragments, converted to half
// once per wavefront (not once per evaluation).
struct MlpFragsF16 {
    half8_t w1[2];  // layer 1, K chunks 0..31 and 32..63 (inputs >= 34 are zero)
    half4_t w2, w3;
    float4_t b1, b2, b3;
};

__device__ __forceinline__ MlpFragsF16 mlp_frags_f16(cfloat* W) {
    const int lane = threadIdx.x & 63;
    MlpFragsF16 f;
    f.w1[0] = a_frag32(W + kOffW1, kMlpIn, 0, lane);
    f.w1[1] = a_frag32(W + kOffW1, kMlpIn, 1, lane);
    f.w2 = a_frag(W + kOffW2, kMlpH, kMlpH, 0, 0, lane);
    f.w3 = a_frag(W + kOffW3, kMlpOut, kMlpH, 0, 0, lane);
    f.b1 = bias_frag(W + kOffB1, kMlpH, lane);
    f.b2 = bias_frag(W + kOffB2, kMlpH, lane);
    f.b3 = bias_frag(W + kOffB3, kMlpOut, lane);
    return f;
}

// B operand (16x16x32) of layer 1 for column group g and K chunk kc: lane l
// reads inputs 32 kc + 8 q .. + 7 of ray 16 g + n from the staged rows.  The
// rows hold 48 inputs, so in chunk 1 the lanes with q >= 2 (inputs 48..63,
// whose weights are zero) take zeros instead of reading past the row.
__device__ __forceinline__ half8_t x_frag32(const _Float16 (*xs)[kXRow], int g, int kc, int lane) {
    const int q = lane >> 4;
    if (kc == 1 && q >= 2) {
        half8_t z;
#pragma unroll
        for (int j = 0; j < 8; ++j) z[j] = _Float16(0.0f);
        return z;
    }
    return *reinterpret_cast<const half8_t*>(&xs[16 * g + (lane & 15)][32 * kc + 8 * q]);
}

// The network on FP16 MFMA tiles for the inputs staged in xs ([64][kXRow]
// halves, one row per lane: x padded with zeros to kXPad).  All 64 lanes of
// the wavefront call this together; lanes with use == false get R = 0.
// Per 16-ray column group: two 16x16x32 tiles for layer 1 (K = 34 in 64),
// one 16x16x16 tile each for layers 2 and 3.
__device__ __forceinline__ void mlp_eval_f16_wave(const MlpFragsF16& f, _Float16 (*xs)[kXRow], bool use, float R[3]) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float4_t out[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        float4_t acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(f.w1[0], x_frag32(xs, g, 0, lane), f.b1, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(f.w1[1], x_frag32(xs, g, 1, lane), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16f16(f.w2, relu_to_half(acc), f.b2, 0, 0, 0);
        out[g] = __builtin_amdgcn_mfma_f32_16x16x16f16(f.w3, relu_to_half(acc), f.b3, 0, 0, 0);
    }
    // Output row i (0..2) of ray 16g + n sits in lane n, element i, of out[g].
    const int src = lane & 15;
    const int my_g = lane >> 4;
#pragma unroll
    for (int i = 0; i < kMlpOut; ++i) {
        float v0 = __shfl(out[0][i], src), v1 = __shfl(out[1][i], src);
        float v2 = __shfl(out[2][i], src), v3 = __shfl(out[3][i], src);
        float z = my_g == 0 ? v0 : (my_g == 1 ? v1 : (my_g == 2 ? v2 : v3));
        R[i] = use ? sigmoid_f32(z) : 0.0f;
    }
    __builtin_amdgcn_wave_barrier();  // xs is rewritten by the next call
}

// All 64 lanes of the wavefront must call this together.  Lanes with
// use == false get R = 0 (their inputs still flow through the tiles).
__device__ __forceinline__ void mlp_forward_f16_wave(cfloat* W, bool use, const float C[3],
                                                     const float V[4], const float d[3], float R[3]) {
    __shared__ _Float16 xs[kMaxWavesF16][64][kXRow];
    const int lane = threadIdx.x & 63;
    const int wave = (threadIdx.x >> 6) & (kMaxWavesF16 - 1);
    float x[kMlpIn];
    encode_x(C, V, d, x);
#pragma unroll
    for (int i = 0; i < kXPad; ++i) xs[wave][lane][i] = _Float16(i < kMlpIn ? x[i] : 0.0f);
    mlp_eval_f16_wave(mlp_frags_f16(W), xs[wave], use, R);
}

}  // namespace snerg
