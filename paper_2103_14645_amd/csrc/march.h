// The per-ray march shared by the forward, trace and backward kernels:
// integer lattice traversal with macroblock skipping and distance-field
// skipping inside macroblocks (march_ray, and the single-loop walk
// FlatWalk that the render and adjoint kernels run), the 8-corner gather
// from the padded block, the exact active-sample predicate and trilinear
// weights.
#pragma once

#include "snerg_dev.h"

namespace snerg {

// One trilinear sample: weights, corner values and the exact active flag.
struct Sample {
    float sigma_raw;  // sum_c w_c * density_c (stored units)
    float rgb[3];     // sum_c w_c * rgb_c (stored units)
    float feat[4];
    bool active;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16 bytes at an 8-byte aligned address: one dwordx4 load (global memory
// needs only dword alignment for multi-dword accesses).
__device__ __forceinline__ u32x4 ld_pair(const uint8_t* p) {
    u32x4 v;
    __builtin_memcpy(&v, __builtin_assume_aligned(p, 8), 16);
    return v;
}

__device__ __forceinline__ float ubyte(uint32_t v, int i) {
    return float((v >> (8 * i)) & 0xFFu);
}

// Corner weights from 16-bit fractions; order c = cx + 2 cy + 4 cz, product (wx*wy)*wz.
__device__ __forceinline__ void corner_weights(const int32_t fr[3], float w[8]) {
    const float fx = float(fr[0]) * (1.0f / 65536.0f);
    const float fy = float(fr[1]) * (1.0f / 65536.0f);
    const float fz = float(fr[2]) * (1.0f / 65536.0f);
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    w[0] = (gx * gy) * gz;
    w[1] = (fx * gy) * gz;
    w[2] = (gx * fy) * gz;
    w[3] = (fx * fy) * gz;
    w[4] = (gx * gy) * fz;
    w[5] = (fx * gy) * fz;
    w[6] = (gx * fy) * fz;
    w[7] = (fx * fy) * fz;
}

// Corner c may have non-zero weight: every axis with c_a = 1 needs f_a != 0.
__device__ __forceinline__ bool corner_live(int c, const int32_t fr[3]) {
    return ((c & 1) == 0 || fr[0] != 0) && ((c & 2) == 0 || fr[1] != 0) && ((c & 4) == 0 || fr[2] != 0);
}

// The 8 corners of a padded cell of a uint8 block: the corners (x, x+1) of
// each of the four (y, z) rows are 16 adjacent bytes, so four 16-byte loads
// issued together bring all of them.
struct Corners8 {
    u32x4 row[4];
};

__device__ __forceinline__ void load_corners_u8(const uint8_t* __restrict__ cell, int Bp, Corners8& cn) {
    const int sy = Bp * 8, sz = Bp * Bp * 8;
    cn.row[0] = ld_pair(cell);
    cn.row[1] = ld_pair(cell + sy);
    cn.row[2] = ld_pair(cell + sz);
    cn.row[3] = ld_pair(cell + sz + sy);
}

// Trilinear sample from loaded uint8 corners.  Every non-zero weight is a
// product of fractions >= 2^-16 (no underflow) and densities are
// non-negative, so "some corner has non-zero density and non-zero weight"
// is exactly "the FP32 density sum is positive".
__device__ __forceinline__ void interp_u8(const Corners8& cn, const int32_t fr[3], Sample& smp) {
    uint2 v[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[2 * r] = make_uint2(cn.row[r].x, cn.row[r].y);
        v[2 * r + 1] = make_uint2(cn.row[r].z, cn.row[r].w);
    }
    float w[8];
    corner_weights(fr, w);
    float sd = 0.f, r0 = 0.f, r1 = 0.f, r2 = 0.f, f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        sd += w[c] * ubyte(v[c].x, 0);
        r0 += w[c] * ubyte(v[c].x, 1);
        r1 += w[c] * ubyte(v[c].x, 2);
        r2 += w[c] * ubyte(v[c].x, 3);
        f0 += w[c] * ubyte(v[c].y, 0);
        f1 += w[c] * ubyte(v[c].y, 1);
        f2 += w[c] * ubyte(v[c].y, 2);
        f3 += w[c] * ubyte(v[c].y, 3);
    }
    smp.sigma_raw = sd;
    smp.rgb[0] = r0; smp.rgb[1] = r1; smp.rgb[2] = r2;
    smp.feat[0] = f0; smp.feat[1] = f1; smp.feat[2] = f2; smp.feat[3] = f3;
    smp.active = sd > 0.0f;
}

// Index of the corner nearest to the sample (the voxel floor(x) in voxel
// units): on each axis the upper corner when the fraction is >= 1/2.
__host__ __device__ __forceinline__ int nearest_corner(const int32_t fr[3]) {
    return (fr[0] >= 32768 ? 1 : 0) | (fr[1] >= 32768 ? 2 : 0) | (fr[2] >= 32768 ? 4 : 0);
}

// Density byte of the nearest corner is non-zero (the WebGL renderer's test).
__device__ __forceinline__ bool nearest_nonzero_u8(const Corners8& cn, const int32_t fr[3]) {
    const int c = nearest_corner(fr);
    const u32x4 r = (c & 6) == 0 ? cn.row[0] : ((c & 6) == 2 ? cn.row[1] : ((c & 6) == 4 ? cn.row[2] : cn.row[3]));
    return (((c & 1) ? r.z : r.x) & 0xFFu) != 0u;
}

// Gather at padded cell p (each in [0, B]) of a uint8 block.
__device__ __forceinline__ void gather_u8(const uint8_t* __restrict__ blk, int Bp, const int32_t p[3],
                                          const int32_t fr[3], Sample& smp) {
    Corners8 cn;
    load_corners_u8(blk + (int64_t((p[2] * Bp + p[1]) * Bp + p[0]) << 3), Bp, cn);
    interp_u8(cn, fr, smp);
}

// The 8 corners of a padded cell of a float32 block (32 bytes per voxel:
// density, RGB, features), loaded by load_corners_f32 and sampled by
// interp_f32: gather_f32 in two parts, so that a caller can issue the loads
// of its next sample before it works on the current one.
struct CornersF32 {
    float4 a[8], b[8];
};

__device__ __forceinline__ void load_corners_f32(const uint8_t* __restrict__ blk, int Bp, const int32_t p[3],
                                                 CornersF32& cn) {
    const float4* base = reinterpret_cast<const float4*>(blk) + (int64_t((p[2] * Bp + p[1]) * Bp + p[0]) << 1);
    const int sy = Bp * 2, sz = Bp * Bp * 2;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4* q = base + ((c & 4) ? sz : 0) + ((c & 2) ? sy : 0) + ((c & 1) ? 2 : 0);
        cn.a[c] = q[0];
        cn.b[c] = q[1];
    }
}

// The same arithmetic in the same order as gather_f32.
__device__ __forceinline__ void interp_f32(const CornersF32& cn, const int32_t fr[3], Sample& smp, bool nn_gate) {
    float w[8];
    corner_weights(fr, w);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool act = false;
    const int cnn = nearest_corner(fr);
    float dnn = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4 a = cn.a[c], b = cn.b[c];
        act |= (a.x != 0.f) && corner_live(c, fr);
        dnn = c == cnn ? a.x : dnn;
        acc[0] += w[c] * a.x; acc[1] += w[c] * a.y; acc[2] += w[c] * a.z; acc[3] += w[c] * a.w;
        acc[4] += w[c] * b.x; acc[5] += w[c] * b.y; acc[6] += w[c] * b.z; acc[7] += w[c] * b.w;
    }
    smp.sigma_raw = acc[0];
    smp.rgb[0] = acc[1]; smp.rgb[1] = acc[2]; smp.rgb[2] = acc[3];
    smp.feat[0] = acc[4]; smp.feat[1] = acc[5]; smp.feat[2] = acc[6]; smp.feat[3] = acc[7];
    smp.active = nn_gate ? dnn != 0.f : act;
}

// Gather at padded cell p of a float32 block (32 bytes per voxel).
// With nn_gate the sample counts as active only when the nearest corner's
// density is non-zero (the WebGL renderer's test; that corner always has
// non-zero weight).
__device__ __forceinline__ void gather_f32(const uint8_t* __restrict__ blk, int Bp, const int32_t p[3],
                                           const int32_t fr[3], Sample& smp, bool nn_gate = false) {
    const float4* base = reinterpret_cast<const float4*>(blk) + (int64_t((p[2] * Bp + p[1]) * Bp + p[0]) << 1);
    const int sy = Bp * 2, sz = Bp * Bp * 2;
    float w[8];
    corner_weights(fr, w);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool act = false;
    const int cnn = nearest_corner(fr);
    float dnn = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float4* q = base + ((c & 4) ? sz : 0) + ((c & 2) ? sy : 0) + ((c & 1) ? 2 : 0);
        const float4 a = q[0], b = q[1];
        act |= (a.x != 0.f) && corner_live(c, fr);
        dnn = c == cnn ? a.x : dnn;
        acc[0] += w[c] * a.x; acc[1] += w[c] * a.y; acc[2] += w[c] * a.z; acc[3] += w[c] * a.w;
        acc[4] += w[c] * b.x; acc[5] += w[c] * b.y; acc[6] += w[c] * b.z; acc[7] += w[c] * b.w;
    }
    smp.sigma_raw = acc[0];
    smp.rgb[0] = acc[1]; smp.rgb[1] = acc[2]; smp.rgb[2] = acc[3];
    smp.feat[0] = acc[4]; smp.feat[1] = acc[5]; smp.feat[2] = acc[6]; smp.feat[3] = acc[7];
    smp.active = nn_gate ? dnn != 0.f : act;
}

// Occupancy lookup: rank of macroblock `lin` in scan order, or -1 if empty.
__host__ __device__ __forceinline__ int32_t block_rank(const uint2* occ, int32_t lin, int32_t n_blocks) {
    const uint2 e = occ[lin >> 5];
    const uint32_t j = uint32_t(lin) & 31u;
    if (!((e.x >> j) & 1u)) return -1;
    const int32_t r = int32_t(e.y) + __builtin_popcount(e.x & ((1u << j) - 1u));
    return r < n_blocks ? r : -1;
}

// Samples the ray may skip from a cell at Chebyshev distance d >= 1 from the
// nearest active cell: after j steps every coordinate has moved by at most
// j*smax in Q16, so the cell index by at most ceil(j*smax / 2^16), and all
// j with j*smax <= (d-1) 2^16 land in inactive cells.  Returns that largest
// j plus one (the current sample is inactive too).
// (d <= 255 and smax <= 2^15, so m stays far below 2^24 and the products
// below 2^32: the masks only tell the compiler that 24-bit multiplies do.)
__host__ __device__ __forceinline__ int32_t skip_steps(int32_t d, int32_t smax, float inv_smax) {
    const uint32_t D = uint32_t(d - 1) << 16;
    const uint32_t sm = uint32_t(smax) & 0xFFFFFFu;
    uint32_t m = uint32_t(__builtin_floorf((float)D * inv_smax)) & 0xFFFFFFu;
    if (((m + 1) & 0xFFFFFFu) * sm <= D) ++m;
    m &= 0xFFFFFFu;
    if (m > 0 && m * sm > D) --m;
    return int32_t(m) + 1;
}

// Linear index of cell p (each coordinate in [0, n)) of an n^3 array, nn = n*n;
// all operands fit 24 bits.
__host__ __device__ __forceinline__ uint32_t cell_index(const int32_t p[3], uint32_t n, uint32_t nn) {
    return (uint32_t(p[2]) & 0x3FFu) * (nn & 0xFFFFFFu) + (uint32_t(p[1]) & 0x3FFu) * (n & 0xFFFFu) +
           (uint32_t(p[0]) & 0x3FFu);
}

// Visits, in order, every lattice sample of a ray that lies in an occupied
// macroblock and in an active cell (cells closer than their distance value
// to the current one are skipped in one step).  on_sample(k, rank, vox, p,
// fr) gets the block's rank, its padded voxels, the padded cell p and the
// 16-bit fractions, and returns true to stop the march.  on_block(lin, occ)
// and on_inblock(n) (n samples inside an occupied block passed) feed the
// visit trace.  `occ` is the occupancy table (usually staged in LDS).
// Sample indices run relative to the ray's first lattice index inside the
// grid (a ray has at most ~3.5 N samples there); callbacks get absolute k.
// Returns the k at which on_sample stopped the march, or -1.
template <typename OnBlock, typename OnInBlock, typename OnSample>
__host__ __device__ __forceinline__ int64_t march_ray(const GridArgs& g, const uint2* occ, const int64_t o[3],
                                                      const int32_t s[3], OnBlock&& on_block,
                                                      OnInBlock&& on_inblock, OnSample&& on_sample) {
    const int bs = 16 + g.logB;
    const int64_t L = int64_t(g.N) << 16;
    const uint32_t nc = uint32_t(g.Bc), ncc = nc * nc;
    int64_t klo, khi;
    if (!entry_range(o, s, L, klo, khi)) return -1;
    float inv[3];
    int32_t P[3];
    int32_t smax = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t sa = s[a] < 0 ? -s[a] : s[a];
        smax = sa > smax ? sa : smax;
        inv[a] = sa != 0 ? 1.0f / float(sa) : 0.0f;
        P[a] = int32_t(o[a] + klo * int64_t(s[a]));  // inside [0, N 2^16)
    }
    const float inv_smax = 1.0f / float(smax);
    const int32_t kend = int32_t(khi - klo);  // relative, inclusive
    int32_t k = 0;
    while (k <= kend) {
        int32_t b[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) b[a] = P[a] >> bs;
        // Guards: the exact integer arithmetic keeps P inside the grid and
        // every sample of [k, kn) inside block b; these checks end the ray
        // instead of indexing outside the buffers should that ever fail.
        if ((unsigned)b[0] >= (unsigned)g.G || (unsigned)b[1] >= (unsigned)g.G || (unsigned)b[2] >= (unsigned)g.G)
            return -1;
        int32_t nstep = block_steps(P, s, inv, b, bs);
        while (nstep > 1 && (((P[0] + (nstep - 1) * s[0]) >> bs) != b[0] ||
                             ((P[1] + (nstep - 1) * s[1]) >> bs) != b[1] ||
                             ((P[2] + (nstep - 1) * s[2]) >> bs) != b[2]))
            --nstep;
        const int32_t kn = (k + nstep) < (kend + 1) ? (k + nstep) : (kend + 1);
        const int32_t lin = (b[2] * g.G + b[1]) * g.G + b[0];
        const int32_t r = block_rank(occ, lin, g.n_blocks);
        on_block(lin, r >= 0);
        if (r >= 0) {
            const uint8_t* __restrict__ dist = g.rec + int64_t(r) * g.rec_stride;
            const uint8_t* __restrict__ vox = dist + g.dist_bytes;
            int32_t q[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] = P[a] - (b[a] << bs) + 32768;  // padded Q16 coordinate
            int32_t left = kn - k;
            int32_t kk = k;
            while (left > 0) {
                const int32_t p[3] = {q[0] >> 16, q[1] >> 16, q[2] >> 16};
                const int32_t d = dist[cell_index(p, nc, ncc)];
                int32_t adv = 1;
                if (d == 0) {
                    on_inblock(1);
                    const int32_t fr[3] = {q[0] & 0xFFFF, q[1] & 0xFFFF, q[2] & 0xFFFF};
                    if (on_sample(klo + kk, r, vox, p, fr)) return klo + kk;
                } else {
                    adv = skip_steps(d, smax, inv_smax);
                    adv = adv < left ? adv : left;
                    on_inblock(adv);
                }
                kk += adv;
                left -= adv;
#pragma unroll
                for (int a = 0; a < 3; ++a) q[a] += adv * s[a];
            }
        }
        const int32_t adv = kn - k;
#pragma unroll
        for (int a = 0; a < 3; ++a) P[a] += adv * s[a];  // |adv s| <= B 2^16 + |s|
        k = kn;
    }
    return -1;
}

// a * b for operands that fit 24-bit signed integers (|a|, |b| < 2^23) with
// a product inside int32: the sign-extension from bit 23 is an identity on
// such values and lets the compiler use the 24-bit multiplier.
__host__ __device__ __forceinline__ int32_t mul_s24(int32_t a, int32_t b) {
    return (int32_t(uint32_t(a) << 8) >> 8) * (int32_t(uint32_t(b) << 8) >> 8);
}

// The samples march_ray visits, in the same order, from one flat loop: on
// each trip a lane either enters its next macroblock (and, when that one is
// occupied, goes on to read the distance byte of its first cell) or reads
// the distance byte of its next cell; a zero byte is an active cell and the
// lane takes the sample on the same trip.  With the macroblock walk and the
// in-block steps in one loop the lanes of a wavefront no longer wait for
// each other at every macroblock face, so the sample code runs with more
// lanes at once.  on_sample as for march_ray.
//
// The macroblock walk is incremental.  With X_a(k) = P_a + k s_a the Q16
// position of relative sample k and W = B 2^16 the macroblock edge, the ray
// leaves its macroblock along axis a at kc_a, the smallest k with
// k |s_a| >= F_a, where F_a = (b_a + 1) W - P_a for s_a > 0 and
// F_a = P_a - b_a W + 1 for s_a < 0.  Crossing that face adds W to F_a, and
// with Q_a = floor(W / |s_a|) the next crossing is kc_a + Q_a or
// kc_a + Q_a + 1, whichever is the first to satisfy the inequality.  The
// next macroblock starts at min_a kc_a, as in march_ray, and every axis
// whose kc_a equals it changes macroblock there.
// Counting hooks of FlatWalk::trip: block(occupied) on every macroblock the
// walk enters, inblock(n) when it passes n samples inside an occupied one
// (the sample it takes, or the cells it skips).  NoCount compiles to nothing.
struct NoCount {
    __host__ __device__ __forceinline__ void block(bool) {}
    __host__ __device__ __forceinline__ void inblock(int32_t) {}
};

struct FlatWalk {
    int32_t kc[3], F[3], Q[3];
    int32_t smax, lin, kend;
    int32_t k;     // first relative sample of the next macroblock to enter
    int32_t kk;    // relative sample at q
    int32_t left;  // samples of the current occupied macroblock from q on
    int32_t r;
    int32_t q[3];
    int64_t klo;
    float inv_smax;
    const uint8_t* __restrict__ dist;

    // Sets up the walk of a ray; false when it misses the grid.
    __host__ __device__ __forceinline__ bool init(const GridArgs& g, const int64_t o[3], const int32_t s[3]) {
        const int bs = 16 + g.logB;
        const int32_t W = int32_t(1) << bs;
        int64_t khi;
        if (!entry_range(o, s, int64_t(g.N) << 16, klo, khi)) return false;
        const int32_t gstride[3] = {1, g.G, g.G * g.G};
        smax = 1;
        lin = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int32_t sa = s[a] < 0 ? -s[a] : s[a];
            smax = sa > smax ? sa : smax;
            const int32_t P = int32_t(o[a] + klo * int64_t(s[a]));  // inside [0, N 2^16)
            const int32_t b = P >> bs;
            lin += b * gstride[a];
            const float inv = sa != 0 ? 1.0f / float(sa) : 0.0f;
            // F as defined above; for s = 0 the s < 0 form, which then only
            // serves to place the sample inside its macroblock
            F[a] = s[a] > 0 ? ((b + 1) << bs) - P : P - (b << bs) + 1;  // in [1, W]
            kc[a] = sa != 0 ? steps_to_reach(F[a], sa, inv) : 0x7fffffff;
            // Q = floor(W / |s|)
            int32_t qa = sa != 0 ? int32_t(__builtin_floorf(float(W) * inv)) : 0;
            if (sa != 0 && (qa + 1) * sa <= W) ++qa;
            if (sa != 0 && qa * sa > W) --qa;
            Q[a] = qa;
        }
        inv_smax = 1.0f / float(smax);
        kend = int32_t(khi - klo);  // relative, inclusive
        k = 0;
        kk = 0;
        left = 0;
        r = -1;
        q[0] = q[1] = q[2] = 0;
        dist = g.rec;
        return true;
    }

    // One trip: enter the next macroblock (going on to its first cell when
    // it is occupied) or step to the next cell; on an active cell hand the
    // sample to on_sample.  One if-region per kind of work and no early
    // exit keep the caller's loop flat in the generated code.  Returns false
    // once the ray has ended or on_sample asked to stop.
    template <typename OnSample>
    __host__ __device__ __forceinline__ bool trip(const GridArgs& g, const uint2* occ, const int32_t s[3],
                                                  OnSample&& on_sample) {
        NoCount nc;
        return trip(g, occ, s, on_sample, nc);
    }

    template <typename OnSample, typename Count>
    __host__ __device__ __forceinline__ bool trip(const GridArgs& g, const uint2* occ, const int32_t s[3],
                                                  OnSample&& on_sample, Count& cnt) {
        const int bs = 16 + g.logB;
        const int32_t W = int32_t(1) << bs;
        const uint32_t nc = uint32_t(g.Bc), ncc = nc * nc;
        const uint32_t G3 = uint32_t(g.G) * uint32_t(g.G) * uint32_t(g.G);
        const int32_t gstride[3] = {1, g.G, g.G * g.G};
        bool live = true;
        bool inside = left > 0;
        if (!inside) {
            // the end of the ray; the index guard keeps the table reads in
            // bounds should the exact walk ever leave the grid
            if (k > kend || uint32_t(lin) >= G3) {
                live = false;
            } else {
                int32_t kn = kc[0] < kc[1] ? kc[0] : kc[1];
                kn = kn < kc[2] ? kn : kc[2];
                kn = kn < kend + 1 ? kn : kend + 1;
                r = block_rank(occ, lin, g.n_blocks);
                cnt.block(r >= 0);
                if (r >= 0) {
                    dist = g.rec + int64_t(r) * g.rec_stride;
                    // Q16 position of sample k inside the macroblock, + 2^15 for the padding
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        q[a] = (s[a] > 0 ? W - F[a] : F[a] - 1) + mul_s24(k, s[a]) + 32768;
                    left = kn - k;
                    kk = k;
                    inside = true;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (kc[a] == kn) {
                        lin += s[a] > 0 ? gstride[a] : -gstride[a];
                        F[a] += W;
                        const int32_t c = kc[a] + Q[a];
                        const int32_t cs = mul_s24(c, s[a]);  // c |s| = sign(s) c s
                        kc[a] = (s[a] > 0 ? cs : -cs) >= F[a] ? c : c + 1;
                    }
                }
                k = kn;
            }
        }
        if (inside) {
            const int32_t p[3] = {q[0] >> 16, q[1] >> 16, q[2] >> 16};
            const int32_t d = dist[cell_index(p, nc, ncc)];
            int32_t adv = 1;
            if (d == 0) {
                const int32_t fr[3] = {q[0] & 0xFFFF, q[1] & 0xFFFF, q[2] & 0xFFFF};
                if (on_sample(klo + kk, r, dist + g.dist_bytes, p, fr)) live = false;
            } else {
                adv = skip_steps(d, smax, inv_smax);
                adv = adv < left ? adv : left;
            }
            cnt.inblock(adv);
            kk += adv;
            left -= adv;
#pragma unroll
            for (int a = 0; a < 3; ++a) q[a] += mul_s24(adv, s[a]);
        }
        return live;
    }
};

template <typename OnSample, typename Count>
__host__ __device__ __forceinline__ void march_ray_flat(const GridArgs& g, const uint2* occ, const int64_t o[3],
                                                        const int32_t s[3], OnSample&& on_sample, Count& cnt) {
    FlatWalk w;
    bool live = w.init(g, o, s);
    while (live) live = w.trip(g, occ, s, on_sample, cnt);
}

template <typename OnSample>
__host__ __device__ __forceinline__ void march_ray_flat(const GridArgs& g, const uint2* occ, const int64_t o[3],
                                                        const int32_t s[3], OnSample&& on_sample) {
    NoCount nc;
    march_ray_flat(g, occ, o, s, on_sample, nc);
}

// march_ray_flat made convergent across the wavefront: every live lane
// makes one trip per iteration, then all 64 lanes call on_sync() together,
// which may therefore use wavefront-wide operations.  `live` false marks a
// lane without a ray.  on_sample as for march_ray; returning true ends the
// lane's march, and so does on_sync() returning true (after the samples
// handed over so far).
template <typename OnSample, typename OnSync>
__device__ __forceinline__ void march_ray_flat_sync(const GridArgs& g, const uint2* occ, bool live,
                                                    const int64_t o[3], const int32_t s[3], OnSample&& on_sample,
                                                    OnSync&& on_sync) {
    FlatWalk w;
    if (live) live = w.init(g, o, s);
    while (__any(live)) {
        if (live) live = w.trip(g, occ, s, on_sample);
        if (on_sync()) live = false;
    }
}

// Samples of the ray inside occupied macroblocks, counted for the blocks
// whose first sample on the ray's lattice lies in the part [k0, k1] of the
// lattice indices inside the grid: the macroblock walk of march_ray alone,
// without visiting samples and without early stop (a cost estimate for
// scheduling, not part of any result).  A block is counted whole by the part
// its first sample lies in, so adding the parts' counts gives the ray's
// count exactly.
__host__ __device__ __forceinline__ int32_t occupied_samples_on_ray(const GridArgs& g, const uint2* occ,
                                                                   const int64_t o[3], const int32_t s[3], int part,
                                                                   int n_parts) {
    const int bs = 16 + g.logB;
    const int64_t L = int64_t(g.N) << 16;
    int64_t klo, khi;
    if (!entry_range(o, s, L, klo, khi)) return 0;
    const int64_t len = khi - klo + 1;
    const int64_t k0 = klo + len * part / n_parts, k1 = klo + len * (part + 1) / n_parts - 1;
    if (k0 > k1) return 0;
    float inv[3];
    int32_t P[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t sa = s[a] < 0 ? -s[a] : s[a];
        inv[a] = sa != 0 ? 1.0f / float(sa) : 0.0f;
        P[a] = int32_t(o[a] + k0 * int64_t(s[a]));
    }
    const int32_t kend = int32_t(k1 - k0);       // the part's last sample, relative
    const int32_t krest = int32_t(khi - k0);     // the ray's last sample, relative
    int32_t k = 0, count = 0;
    bool first = k0 > klo;
    while (k <= kend) {
        int32_t b[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) b[a] = P[a] >> bs;
        if ((unsigned)b[0] >= (unsigned)g.G || (unsigned)b[1] >= (unsigned)g.G || (unsigned)b[2] >= (unsigned)g.G)
            break;
        const int32_t nstep = block_steps(P, s, inv, b, bs);
        const int32_t lin = (b[2] * g.G + b[1]) * g.G + b[0];
        bool counted = ((occ[lin >> 5].x >> (lin & 31)) & 1u) != 0;
        if (first) {  // entered in an earlier part?
            counted = counted && (((P[0] - s[0]) >> bs) != b[0] || ((P[1] - s[1]) >> bs) != b[1] ||
                                  ((P[2] - s[2]) >> bs) != b[2]);
            first = false;
        }
        // the whole block up to the ray's end, also past the part's end
        const int32_t n = (k + nstep) <= krest + 1 ? nstep : krest + 1 - k;
        count += counted ? n : 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) P[a] += nstep * s[a];
        k += nstep;
    }
    return count;
}

}  // namespace snerg
