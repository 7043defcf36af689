// Baking side of the method (Section 5.3, 5.4): which macroblocks of a
// densely evaluated field are stored, and their 8-bit values.
//
//  k_bake_block_max   largest density of every macroblock (HBM-bound
//                     streaming pass over the N^3 field); also resets the
//                     per-block visibility words.
//  k_bake_visibility  every training ray marched over the dense field on
//                     the render's sample lattice (step 1/N), one lane per
//                     ray and one wavefront per 8x8 pixel tile; the density
//                     prefix sum before the first sample of each macroblock
//                     the ray enters is folded into that block's minimum
//                     (64-bit atomic min on the bits of a non-negative
//                     double, which orders like the value).  The ray stops
//                     once the prefix sum passes the visibility threshold:
//                     later samples cannot make a block visible.
//  k_bake_compact     the two culls and the atlas numbering in scan order
//                     (one workgroup: a ballot prefix per wavefront, then
//                     across wavefronts).
//  k_bake_quantize    8-bit quantisation of the kept blocks into the
//                     canonical atlas, four voxels per lane along x.
#include <type_traits>

#include "snerg_launch.h"

namespace snerg {

namespace {

constexpr uint64_t kInfBits = 0x7ff0000000000000ull;  // +inf as double bits

struct f32x4 {
    float v[4];
};
__device__ __forceinline__ f32x4 ld4(const float* p) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    return {{q.x, q.y, q.z, q.w}};
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m));
    return v;
}

}  // namespace

// One workgroup per macroblock (grid.x = G^3).  V = voxels per load (4 when
// B >= 4, else 1).
template <int V>
__global__ __launch_bounds__(256) void k_bake_block_max(const float* __restrict__ sigma, int32_t N, int32_t logB,
                                                        int32_t G, float* __restrict__ bmax,
                                                        uint64_t* __restrict__ depth_bits) {
    __shared__ float part[4];
    const int64_t lin = blockIdx.x;
    const int32_t bx = int32_t(lin % G), by = int32_t((lin / G) % G), bz = int32_t(lin / (int64_t(G) * G));
    const int32_t B = 1 << logB;
    const int32_t rowq = B / V;  // loads per row
    const int32_t n_loads = B * B * rowq;
    float m = -INFINITY;
    for (int32_t e = threadIdx.x; e < n_loads; e += blockDim.x) {
        const int32_t q = e % rowq, r = e / rowq;
        const int32_t ly = r & (B - 1), lz = r >> logB;
        const int64_t base = (int64_t(bz * B + lz) * N + (by * B + ly)) * N + bx * B + q * V;
        if (V == 4) {
            const f32x4 x = ld4(sigma + base);
            m = fmaxf(m, fmaxf(fmaxf(x.v[0], x.v[1]), fmaxf(x.v[2], x.v[3])));
        } else {
            m = fmaxf(m, sigma[base]);
        }
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = part[0];
        for (int w = 1; w < int(blockDim.x >> 6); ++w) r = fmaxf(r, part[w]);
        bmax[lin] = r;
        depth_bits[lin] = kInfBits;
    }
}

struct BakeVisArgs {
    const float* sigma;
    const DevCamera* cams;
    int32_t n_cams;
    int32_t N, logB, G;
    int64_t total_tiles;
    int32_t tile_w, tile_h;
    double sum_thr;  // stop once the density prefix sum exceeds this
    uint64_t* depth_bits;
};

// Samples loaded ahead of the sequential prefix sum.
constexpr int kVisAhead = 4;

// Voxel index arithmetic of the march: kIdx64 for any N, kIdx32 when
// N^3 < 2^32 (24-bit multiplies), kIdxPow2 when N is a power of two up to
// 1024 (bit fields: the voxel index is vx | vy << lg | vz << 2 lg, and the
// macroblock is that index with the low logB bits of each field masked off,
// one AND per sample).
enum { kIdx64 = 0, kIdx32 = 1, kIdxPow2 = 2 };

template <int IDX>
__global__ __launch_bounds__(256) void k_bake_visibility(BakeVisArgs a) {
    // Per-workgroup cache of bounds on the blocks' minima: 256 slots indexed
    // by the low 8 bits of the block index, each one 32-bit word (read and
    // written whole, so no reader sees half an update): the block index's
    // high 10 bits, then a 22-bit code whose value is an upper bound of a
    // prefix sum already folded into that block's minimum (the sum rounded
    // up to float, then its bits rounded up to a multiple of 2^10).  A block
    // entry whose prefix sum is at least that bound needs no global access:
    // the block's minimum is already no larger.  A racing overwrite only
    // costs a later global check.
    __shared__ uint32_t vcache[256];
    vcache[threadIdx.x & 255] = (0x3ffu << 22) | (0x7f800000u >> 10);  // bound +inf: never skips
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t t = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= a.total_tiles) return;  // wave-uniform
    const int ci = find_camera_by_tile(a.cams, a.n_cams, t);
    const DevCamera& c = a.cams[ci];
    const int64_t tl = t - c.tile_offset;
    const int px = int(tl % c.tiles_x) * a.tile_w + lane % a.tile_w;
    const int py = int(tl / c.tiles_x) * a.tile_h + lane / a.tile_w;
    if (px >= c.W || py >= c.H) return;
    int64_t o[3];
    int32_t s[3];
    float d[3];
    ray_setup(c, a.N, px, py, o, s, d);
    const int64_t L = int64_t(a.N) << 16;
    int64_t klo, khi;
    if (!entry_range(o, s, L, klo, khi)) return;
    int32_t P[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) P[q] = int32_t(o[q] + klo * int64_t(s[q]));  // inside [0, N 2^16)
    const int32_t n = int32_t(khi - klo + 1);
    const uint32_t N = uint32_t(a.N), G = uint32_t(a.G);
    const int bs = 16 + a.logB;
    int lg = 0;
    while ((1 << lg) < a.N) ++lg;
    const uint32_t fmask = (G - 1) << a.logB;  // block bits of one coordinate field
    const uint32_t bmask = fmask | (fmask << lg) | (fmask << (2 * lg));
    const double thr = a.sum_thr;
    double sum = 0.0;
    uint32_t prev = 0xffffffffu;
    // One chunk of kVisAhead samples: all loads first, then the sequential
    // prefix sum.  With FULL every sample of the chunk is inside the grid;
    // otherwise the ones past the last inside sample are clamped onto it, so
    // that every load stays in bounds.
    auto chunk = [&](auto full_tag, int32_t last) {
        constexpr bool FULL = decltype(full_tag)::value;
        float sv[kVisAhead];
        uint32_t bk[kVisAhead];
        uint32_t Q[3] = {uint32_t(P[0]), uint32_t(P[1]), uint32_t(P[2])};
#pragma unroll
        for (int u = 0; u < kVisAhead; ++u) {
            if (u > 0) {
                const uint32_t m = (FULL || u <= last) ? 0xffffffffu : 0u;
#pragma unroll
                for (int q = 0; q < 3; ++q) Q[q] += uint32_t(s[q]) & m;
            }
            if (IDX == kIdxPow2) {
                const uint32_t v = (Q[0] >> 16) | ((Q[1] >> 16) << lg) | ((Q[2] >> 16) << (2 * lg));
                sv[u] = a.sigma[v];
                bk[u] = v & bmask;
            } else {
                if (IDX == kIdx32) {  // every factor and partial sum below 2^24
                    const uint32_t v = __umul24(__umul24(Q[2] >> 16, N) + (Q[1] >> 16), N) + (Q[0] >> 16);
                    sv[u] = a.sigma[v];
                } else {
                    const uint64_t v = (uint64_t(Q[2] >> 16) * N + (Q[1] >> 16)) * N + (Q[0] >> 16);
                    sv[u] = a.sigma[v];
                }
                // macroblock coordinates packed 8 bits each (G <= 64)
                bk[u] = (Q[0] >> bs) | ((Q[1] >> bs) << 8) | ((Q[2] >> bs) << 16);
            }
        }
#pragma unroll
        for (int u = 0; u < kVisAhead; ++u) {
            if (FULL || u <= last) {
                // first sample of a macroblock: the ray's smallest prefix sum in
                // it; past the threshold no later block is visible from this ray
                if (bk[u] != prev) {
                    prev = bk[u];
                    if (sum <= thr) {
                        const uint64_t bits = uint64_t(__double_as_longlong(sum));
                        uint32_t bx, by, bz;
                        if (IDX == kIdxPow2) {
                            bx = (bk[u] >> a.logB) & (G - 1);
                            by = (bk[u] >> (lg + a.logB)) & (G - 1);
                            bz = bk[u] >> (2 * lg + a.logB);
                        } else {
                            bx = bk[u] & 0xff;
                            by = (bk[u] >> 8) & 0xff;
                            bz = bk[u] >> 16;
                        }
                        const uint32_t lin = __umul24(__umul24(bz, G) + by, G) + bx;
                        const uint32_t key = vcache[lin & 255];
                        if ((key >> 22) != (lin >> 8) || double(__uint_as_float((key & 0x3fffffu) << 10)) > sum) {
                            uint64_t* w = a.depth_bits + lin;
                            uint64_t g = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if (bits < g) {
                                atomicMin(reinterpret_cast<unsigned long long*>(w), (unsigned long long)bits);
                                g = bits;
                            }
                            const double gv = __longlong_as_double((long long)g);
                            float gf = float(gv);
                            if (double(gf) < gv) gf = __uint_as_float(__float_as_uint(gf) + 1u);
                            const uint32_t code = (__float_as_uint(gf) + 0x3ffu) >> 10;
                            vcache[lin & 255] = ((lin >> 8) << 22) | code;
                        }
                    }
                }
                sum += double(sv[u]);
            }
        }
    };
    for (int32_t j = 0;; j += kVisAhead) {
        const int32_t last = n - 1 - j;
        if (__all(last >= kVisAhead - 1))
            chunk(std::true_type{}, last);
        else
            chunk(std::false_type{}, last);
        if (sum > thr || last < kVisAhead) break;
#pragma unroll
        for (int q = 0; q < 3; ++q) P[q] += kVisAhead * s[q];
    }
}

struct BakeCompactArgs {
    const float* bmax;
    const uint64_t* depth_bits;
    int64_t n_lin;        // G^3
    int32_t N;
    double sigma_thr;     // keep when max sigma >= this (alpha >= tau_alpha)
    double sum_thr;       // keep when min prefix sum <= this (T >= tau_vis)
    float* block_alpha;   // nullable
    float* block_vis;     // nullable
    int32_t* indirection;
    int32_t* n_blocks;    // device, one int
};

__global__ __launch_bounds__(1024) void k_bake_compact(BakeCompactArgs a) {
    __shared__ int32_t wtot[16];
    __shared__ int32_t base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    const double inv_n = 1.0 / double(a.N);
    for (int64_t c0 = 0; c0 < a.n_lin; c0 += blockDim.x) {
        const int64_t lin = c0 + threadIdx.x;
        bool keep = false;
        if (lin < a.n_lin) {
            const double sm = double(a.bmax[lin]);
            const double dm = __longlong_as_double((long long)a.depth_bits[lin]);
            keep = sm >= a.sigma_thr && dm <= a.sum_thr;
            if (a.block_alpha) a.block_alpha[lin] = float(1.0 - exp(-sm * inv_n));
            if (a.block_vis) a.block_vis[lin] = dm <= a.sum_thr ? float(exp(-dm * inv_n)) : 0.0f;
        }
        const uint64_t bal = __ballot(keep);
        const int32_t below = __popcll(bal & ((uint64_t(1) << lane) - 1));
        if (lane == 0) wtot[wave] = __popcll(bal);
        __syncthreads();
        int32_t off = base;
        for (int w = 0; w < wave; ++w) off += wtot[w];
        if (lin < a.n_lin) a.indirection[lin] = keep ? off + below : -1;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t tot = 0;
            for (int w = 0; w < n_waves; ++w) tot += wtot[w];
            base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.n_blocks = base;
}

// lin_of[id] = indirection index of atlas id (ids outside [0, n_blocks) are
// ignored); lin_of holds -1 beforehand.
__global__ __launch_bounds__(256) void k_bake_invert(const int32_t* __restrict__ ind, int64_t n_lin, int32_t n_blocks,
                                                     int32_t* __restrict__ lin_of) {
    const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lin >= n_lin) return;
    const int32_t id = ind[lin];
    if (id >= 0 && id < n_blocks) lin_of[id] = int32_t(lin);
}

struct BakeQuantArgs {
    const float* sigma;
    const float* rgb;
    const float* feat;
    const int32_t* lin_of;
    int32_t N, logB, G;
    float k_sigma;  // 255 / sigma_scale, float32
    uint8_t* dens8;
    uint8_t* rgb8;
    uint8_t* feat8;
};

__device__ __forceinline__ uint32_t qbyte(float x, float k) {
    const float q = __builtin_rintf(__fmul_rn(x, k));
    return uint32_t(fminf(fmaxf(q, 0.0f), 255.0f));
}

// grid.x = atlas id, grid.y = chunk of 256 lanes x V voxels of the block.
template <int V>
__global__ __launch_bounds__(256) void k_bake_quantize(BakeQuantArgs a) {
    const int32_t id = blockIdx.x;
    const int32_t B = 1 << a.logB;
    const int64_t B3 = int64_t(B) * B * B;
    const int64_t e0 = (int64_t(blockIdx.y) * blockDim.x + threadIdx.x) * V;  // first voxel, canonical order
    if (e0 >= B3) return;
    const int32_t lx = int32_t(e0 & (B - 1)), ly = int32_t((e0 >> a.logB) & (B - 1)), lz = int32_t(e0 >> (2 * a.logB));
    const int64_t out = int64_t(id) * B3 + e0;
    const int32_t lin = a.lin_of[id];
    uint32_t dq[V], rq[3 * V], fq[4 * V];
    if (lin < 0) {
#pragma unroll
        for (int i = 0; i < V; ++i) dq[i] = 0;
#pragma unroll
        for (int i = 0; i < 3 * V; ++i) rq[i] = 0;
#pragma unroll
        for (int i = 0; i < 4 * V; ++i) fq[i] = 0;
    } else {
        const int32_t bx = lin % a.G, by = (lin / a.G) % a.G, bz = lin / (a.G * a.G);
        const int64_t v = (int64_t(bz * B + lz) * a.N + (by * B + ly)) * a.N + bx * B + lx;
        const float kr = 255.0f;
        if (V == 4) {
            const f32x4 sg = ld4(a.sigma + v);
#pragma unroll
            for (int i = 0; i < 4; ++i) dq[i] = qbyte(sg.v[i], a.k_sigma);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const f32x4 x = ld4(a.rgb + 3 * v + 4 * c);
#pragma unroll
                for (int i = 0; i < 4; ++i) rq[4 * c + i] = qbyte(x.v[i], kr);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const f32x4 x = ld4(a.feat + 4 * v + 4 * c);
#pragma unroll
                for (int i = 0; i < 4; ++i) fq[4 * c + i] = qbyte(x.v[i], kr);
            }
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                dq[i] = qbyte(a.sigma[v + i], a.k_sigma);
#pragma unroll
                for (int c = 0; c < 3; ++c) rq[3 * i + c] = qbyte(a.rgb[3 * (v + i) + c], kr);
#pragma unroll
                for (int c = 0; c < 4; ++c) fq[4 * i + c] = qbyte(a.feat[4 * (v + i) + c], kr);
            }
        }
    }
    if (V == 4) {
        *reinterpret_cast<uint32_t*>(a.dens8 + out) = dq[0] | (dq[1] << 8) | (dq[2] << 16) | (dq[3] << 24);
        uint32_t* r = reinterpret_cast<uint32_t*>(a.rgb8 + 3 * out);
#pragma unroll
        for (int w = 0; w < 3; ++w)
            r[w] = rq[4 * w] | (rq[4 * w + 1] << 8) | (rq[4 * w + 2] << 16) | (rq[4 * w + 3] << 24);
        uint32_t* f = reinterpret_cast<uint32_t*>(a.feat8 + 4 * out);
#pragma unroll
        for (int w = 0; w < 4; ++w)
            f[w] = fq[4 * w] | (fq[4 * w + 1] << 8) | (fq[4 * w + 2] << 16) | (fq[4 * w + 3] << 24);
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) {
            a.dens8[out + i] = uint8_t(dq[i]);
#pragma unroll
            for (int c = 0; c < 3; ++c) a.rgb8[3 * (out + i) + c] = uint8_t(rq[3 * i + c]);
#pragma unroll
            for (int c = 0; c < 4; ++c) a.feat8[4 * (out + i) + c] = uint8_t(fq[4 * i + c]);
        }
    }
}

hipError_t launch_bake_cull(const BakeCullPlan& p, hipStream_t s) {
    const int64_t G3 = int64_t(p.G) * p.G * p.G;
    if (p.vec4)
        hipLaunchKernelGGL(k_bake_block_max<4>, dim3(unsigned(G3)), dim3(256), 0, s, p.sigma, p.N, p.logB, p.G,
                           p.bmax, p.depth_bits);
    else
        hipLaunchKernelGGL(k_bake_block_max<1>, dim3(unsigned(G3)), dim3(256), 0, s, p.sigma, p.N, p.logB, p.G,
                           p.bmax, p.depth_bits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (p.total_tiles > 0) {
        BakeVisArgs v;
        v.sigma = p.sigma;
        v.cams = p.cams;
        v.n_cams = p.n_cams;
        v.N = p.N;
        v.logB = p.logB;
        v.G = p.G;
        v.total_tiles = p.total_tiles;
        v.tile_w = p.tile_w;
        v.tile_h = p.tile_h;
        v.sum_thr = p.sum_thr;
        v.depth_bits = p.depth_bits;
        const unsigned blocks = unsigned((p.total_tiles + 3) / 4);
        if ((p.N & (p.N - 1)) == 0 && p.N <= 1024)
            hipLaunchKernelGGL(k_bake_visibility<kIdxPow2>, dim3(blocks), dim3(256), 0, s, v);
        else if (int64_t(p.N) * p.N * p.N <= int64_t(0xffffffffu))
            hipLaunchKernelGGL(k_bake_visibility<kIdx32>, dim3(blocks), dim3(256), 0, s, v);
        else
            hipLaunchKernelGGL(k_bake_visibility<kIdx64>, dim3(blocks), dim3(256), 0, s, v);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    BakeCompactArgs c;
    c.bmax = p.bmax;
    c.depth_bits = p.depth_bits;
    c.n_lin = G3;
    c.N = p.N;
    c.sigma_thr = p.sigma_thr;
    c.sum_thr = p.sum_thr;
    c.block_alpha = p.block_alpha;
    c.block_vis = p.block_vis;
    c.indirection = p.indirection;
    c.n_blocks = p.n_blocks_dev;
    hipLaunchKernelGGL(k_bake_compact, dim3(1), dim3(1024), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_bake_quantize(const BakeQuantPlan& p, hipStream_t s) {
    const int64_t G3 = int64_t(p.G) * p.G * p.G;
    hipError_t e = launch_fill_i32(p.lin_of, p.n_blocks, -1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bake_invert, dim3(unsigned((G3 + 255) / 256)), dim3(256), 0, s, p.indirection, G3,
                       p.n_blocks, p.lin_of);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    BakeQuantArgs q;
    q.sigma = p.sigma;
    q.rgb = p.rgb;
    q.feat = p.feat;
    q.lin_of = p.lin_of;
    q.N = p.N;
    q.logB = p.logB;
    q.G = p.G;
    q.k_sigma = p.k_sigma;
    q.dens8 = p.dens8;
    q.rgb8 = p.rgb8;
    q.feat8 = p.feat8;
    const int64_t B3 = int64_t(1) << (3 * p.logB);
    const int V = p.vec4 ? 4 : 1;
    const unsigned chunks = unsigned((B3 / V + 255) / 256);
    if (p.vec4)
        hipLaunchKernelGGL(k_bake_quantize<4>, dim3(unsigned(p.n_blocks), chunks), dim3(256), 0, s, q);
    else
        hipLaunchKernelGGL(k_bake_quantize<1>, dim3(unsigned(p.n_blocks), chunks), dim3(256), 0, s, q);
    return hipGetLastError();
}

}  // namespace snerg
