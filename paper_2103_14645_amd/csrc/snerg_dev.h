// Device-side data layouts and helpers of the gfx950 SNeRG renderer.
//
// Packed grid (written by the pack kernels, read by render/backward):
//   [occ:      n_words x {uint32 bits, int32 rank}]  n_words = ceil(G^3 / 32)
//       bit j of word w is set when macroblock lin = 32 w + j (indirection
//       order) holds a valid atlas id; `rank` counts the set bits of all
//       earlier words.  The rank of an occupied macroblock (its position in
//       scan order) indexes the per-block records below.
//   [rank_lin: n_blocks int32]  indirection index of rank r
//   [rank_id:  n_blocks int32]  atlas id of rank r (canonical layout)
//   [records:  n_blocks x rec_stride bytes], rank order, each:
//       dist: (B+1)^3 bytes.  Cell (cx, cy, cz), c in [0, B], is the
//           trilinear cell whose lower corner is local voxel c - 1; it is
//           active when any of its 8 corner voxels has non-zero density.
//           dist holds the Chebyshev (L-inf) distance, in cells, from the
//           cell to the nearest active cell of the same record (0 = active,
//           capped at 255), at ((cz*(B+1) + cy)*(B+1) + cx).
//       vox (16-byte aligned): padded copy of the block, local voxel v in
//           [-1, B] per axis at ((v_z+1)*(B+2) + (v_y+1))*(B+2) + (v_x+1);
//           voxels of neighbouring occupied blocks are copied in,
//           outside/empty ones are zero.  Channels interleaved per voxel:
//           density, r, g, b, f0..f3 (8 bytes for uint8, 32 for float32).
// Sections start on 256-byte boundaries; records are 256-byte aligned.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snerg {

constexpr int kMlpIn = 34;
constexpr int kMlpH = 16;
constexpr int kMlpOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB3 + kMlpOut;  // 883

// Camera as the kernels see it (host fills it from snerg_camera).
struct DevCamera {
    double eye[3], fwd[3], right[3], up[3];
    double focal;
    int32_t W, H;
    int64_t ray_offset;   // id of the camera's first ray
    int64_t tile_offset;  // index of the camera's first wavefront tile
    int32_t tiles_x, tiles_y;
};

struct PackedLayout {
    int32_t N, B, logB, G;
    int32_t Bp;          // B + 2
    int32_t Bc;          // B + 1
    int32_t n_words;     // occupancy words
    int32_t vsize;       // bytes per voxel
    int64_t off_occ, off_rank_lin, off_rank_id, off_rec;
    int64_t dist_bytes;  // (B+1)^3 rounded up to 16
    int64_t rec_stride;  // bytes per block record
    int64_t total;
};

inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

inline PackedLayout make_layout(int32_t N, int32_t B, int32_t n_blocks, int32_t vsize) {
    PackedLayout L;
    L.N = N;
    L.B = B;
    int lb = 0;
    while ((1 << lb) < B) ++lb;
    L.logB = lb;
    L.G = N / B;
    L.Bp = B + 2;
    L.Bc = B + 1;
    const int64_t G3 = int64_t(L.G) * L.G * L.G;
    L.n_words = int32_t((G3 + 31) / 32);
    L.vsize = vsize;
    L.off_occ = 0;
    L.off_rank_lin = align256(int64_t(L.n_words) * 8);
    L.off_rank_id = L.off_rank_lin + align256(int64_t(n_blocks) * 4);
    L.off_rec = L.off_rank_id + align256(int64_t(n_blocks) * 4);
    L.dist_bytes = (int64_t(L.Bc) * L.Bc * L.Bc + 15) & ~int64_t(15);
    L.rec_stride = align256(L.dist_bytes + int64_t(L.Bp) * L.Bp * L.Bp * vsize);
    L.total = L.off_rec + int64_t(n_blocks) * L.rec_stride;
    return L;
}

// Largest grid whose occupancy table is staged in LDS: (N/B)^3 <= 2^18.
constexpr int kMaxOccWords = (1 << 18) / 32;

// Grid as a kernel argument.
struct GridArgs {
    const int32_t* ind;       // canonical indirection (atlas ids)
    const uint2* occ;         // {bits, rank} per 32 macroblocks
    const int32_t* rank_lin;
    const int32_t* rank_id;
    const uint8_t* rec;       // block records in rank order
    int32_t N, B, logB, G, Bp, Bc, n_words, n_blocks;
    int64_t rec_stride, dist_bytes;
    float sigma_scale;
};

// Read-only parameters viewed through the constant address space: loads at
// wavefront-uniform addresses become scalar (SMEM) loads into SGPRs.
typedef const __attribute__((address_space(4))) float cfloat;
__device__ __forceinline__ cfloat* as_const(const float* p) { return (cfloat*)p; }

struct RenderOpts {
    float bg[3];
    float t_stop;
    int32_t early_stop;
    int32_t mlp_on;
    int32_t nn_gate;        // composite only samples whose nearest voxel has density
    int32_t unpremultiply;  // Eq. 9 after compositing
    int32_t per_sample_mlp; // not deferred: the network on every composited sample
};

// ---------------------------------------------------------------- integers

// floor(a / b) for b > 0 and |a| < 2^53: the correctly rounded double
// quotient is within |a| 2^-53 / b < 1/b of a/b, and a non-integer a/b is at
// least 1/b away from every integer, so floor() never crosses one.
__host__ __device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
    return (int64_t)__builtin_floor((double)a / (double)b);
}
__host__ __device__ __forceinline__ int64_t ceil_div64(int64_t a, int64_t b) {
    return (int64_t)__builtin_ceil((double)a / (double)b);
}

// Smallest n >= 1 with n * s >= D (0 < D < 2^23, 0 < s < 2^16), from a float
// estimate corrected in integers (the estimate is off by at most one).
__host__ __device__ __forceinline__ int32_t steps_to_reach(int32_t D, int32_t s, float inv_s) {
    int32_t n = (int32_t)__builtin_ceilf((float)D * inv_s);
    if (n * s < D) ++n;
    if (n > 1 && (n - 1) * s >= D) --n;
    return n < 1 ? 1 : n;
}
// Smallest n >= 1 with n * s > D (0 <= D < 2^23, 0 < s < 2^16).
__host__ __device__ __forceinline__ int32_t steps_to_pass(int32_t D, int32_t s, float inv_s) {
    int32_t n = (int32_t)__builtin_floorf((float)D * inv_s) + 1;
    if (n * s <= D) ++n;
    if (n > 1 && (n - 1) * s > D) --n;
    return n < 1 ? 1 : n;
}

// ------------------------------------------------------------ ray prologue

// FP64 ray setup with the operation order of the ABI contract (no
// contraction): Q16 origin o, Q16 step s (half a voxel along d), direction d.
__host__ __device__ __forceinline__ void ray_setup(const DevCamera& c, int32_t N, int32_t px, int32_t py,
                                          int64_t o[3], int32_t s[3], float d[3]) {
#pragma clang fp contract(off)
    double x = (((double)px + 0.5) - (double)c.W * 0.5) / c.focal;
    double y = (((double)py + 0.5) - (double)c.H * 0.5) / c.focal;
    double D[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = x * c.right[a];
        t = c.fwd[a] + t;
        double u = y * c.up[a];
        D[a] = t - u;
    }
    double n2 = D[0] * D[0];
    n2 = n2 + D[1] * D[1];
    n2 = n2 + D[2] * D[2];
    double n = __builtin_sqrt(n2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double da = D[a] / n;
        d[a] = (float)da;
        s[a] = (int32_t)__builtin_rint(da * 32768.0);
        double e = c.eye[a] + 1.0;
        e = e * (0.5 * (double)N);
        e = e * 65536.0;
        o[a] = (int64_t)__builtin_rint(e);
    }
}

// Inclusive range [klo, khi] of lattice indices inside [0, L)^3; false if empty.
__host__ __device__ __forceinline__ bool entry_range(const int64_t o[3], const int32_t s[3], int64_t L,
                                            int64_t& klo, int64_t& khi) {
    klo = 0;
    khi = INT64_MAX;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t sa = s[a], oa = o[a];
        if (sa == 0) {
            if (oa < 0 || oa >= L) return false;
        } else if (sa > 0) {
            const int64_t lo = ceil_div64(-oa, sa), hi = floor_div64(L - 1 - oa, sa);
            klo = lo > klo ? lo : klo;
            khi = hi < khi ? hi : khi;
        } else {
            const int64_t lo = ceil_div64(oa - (L - 1), -sa), hi = floor_div64(oa, -sa);
            klo = lo > klo ? lo : klo;
            khi = hi < khi ? hi : khi;
        }
    }
    return klo <= khi;
}

// Lattice steps from position P (inside macroblock b, edge shift
// bs = 16 + log2 B) until the ray leaves the macroblock on some axis.
__host__ __device__ __forceinline__ int32_t block_steps(const int32_t P[3], const int32_t s[3], const float inv_abs_s[3],
                                               const int32_t b[3], int bs) {
    int32_t n = 0x7fffffff;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (s[a] > 0) {
            const int32_t D = ((b[a] + 1) << bs) - P[a];  // in (0, B 2^16]
            const int32_t m = steps_to_reach(D, s[a], inv_abs_s[a]);
            n = m < n ? m : n;
        } else if (s[a] < 0) {
            const int32_t D = P[a] - (b[a] << bs);  // in [0, B 2^16)
            const int32_t m = steps_to_pass(D, -s[a], inv_abs_s[a]);
            n = m < n ? m : n;
        }
    }
    return n;
}

// Workgroup w of a launch of n goes to XCD w mod 8 (each of the eight XCDs
// has its own L2), so consecutive workgroups of a tile order, which render
// neighbouring tiles and read the same macroblocks, would land in eight
// different L2s.  This permutation of [0, n) gives each XCD runs of 8
// consecutive workgroups while the XCDs still advance through the order
// together; the last n mod 64 stay in place.  Only the speed depends on the
// dispatch order, never the result.
__device__ __forceinline__ uint32_t xcd_grouped(uint32_t w, uint32_t n) {
    constexpr uint32_t kRun = 8, kChunk = 8 * kRun;
    if (w >= n / kChunk * kChunk) return w;
    const uint32_t r = w % kChunk;
    return w - r + (r % 8) * kRun + r / 8;
}

// Camera of a global tile / ray index (binary search over the table).
__device__ __forceinline__ int find_camera_by_tile(const DevCamera* cams, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_camera_by_ray(const DevCamera* cams, int n, int64_t r) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cams[mid].ray_offset <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace snerg
