// Packing of a canonical SNeRG atlas into the layout the render kernels read
// (described in snerg_dev.h).  Atlas ids outside [0, n_blocks) in the
// indirection grid count as empty macroblocks, and ranks beyond n_blocks
// (only possible when atlas ids repeat) are dropped, so no kernel can index
// past the packed buffer whatever the indirection holds.
#include "snerg_dev.h"
#include "snerg_launch.h"

namespace snerg {

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_occ_bits(const int32_t* __restrict__ ind, int64_t G3, int32_t n_blocks, int32_t n_words,
                           uint2* __restrict__ occ) {
    const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_words) return;
    uint32_t bits = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t lin = int64_t(w) * 32 + j;
        if (lin >= G3) break;
        const int32_t id = ind[lin];
        bits |= uint32_t(id >= 0 && id < n_blocks) << j;
    }
    occ[w] = make_uint2(bits, 0u);
}

// Exclusive prefix sum of the popcounts (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_occ_scan(uint2* __restrict__ occ, int32_t n_words) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (n_words + 1023) / 1024;
    const int w0 = t * per;
    int32_t sum = 0;
    for (int i = 0; i < per; ++i)
        if (w0 + i < n_words) sum += __popc(occ[w0 + i].x);
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int i = 0; i < per; ++i)
        if (w0 + i < n_words) {
            occ[w0 + i].y = uint32_t(run);
            run += __popc(occ[w0 + i].x);
        }
}

__global__ void k_rank_maps(const int32_t* __restrict__ ind, const uint2* __restrict__ occ, int64_t G3,
                            int32_t n_blocks, int32_t* __restrict__ rank_lin, int32_t* __restrict__ rank_id) {
    const int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lin >= G3) return;
    const uint2 e = occ[lin >> 5];
    const int j = int(lin & 31);
    if (!((e.x >> j) & 1u)) return;
    const int32_t r = int32_t(e.y) + __popc(e.x & ((1u << j) - 1u));
    if (r < n_blocks) {
        rank_lin[r] = int32_t(lin);
        rank_id[r] = ind[lin];
    }
}

// One thread per padded voxel of every block record.
template <typename T>
__global__ void k_pack_vox(const int32_t* __restrict__ ind, const int32_t* __restrict__ rank_lin,
                           const T* __restrict__ dens, const T* __restrict__ rgb, const T* __restrict__ feat,
                           int32_t N, int32_t B, int32_t logB, int32_t n_blocks, int64_t total,
                           int64_t rec_stride, int64_t dist_bytes, uint8_t* __restrict__ rec) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int32_t Bp = B + 2;
    const int64_t per_block = int64_t(Bp) * Bp * Bp;
    const int32_t r = int32_t(t / per_block);
    const int32_t v = int32_t(t - int64_t(r) * per_block);
    const int32_t px = v % Bp, py = (v / Bp) % Bp, pz = v / (Bp * Bp);
    const int32_t G = N >> logB;
    T val[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    const int32_t lin = rank_lin[r];
    if (lin >= 0) {
        const int32_t bx = lin % G, by = (lin / G) % G, bz = lin / (G * G);
        const int32_t gx = bx * B + px - 1, gy = by * B + py - 1, gz = bz * B + pz - 1;
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < N && gy < N && gz < N) {
            const int32_t nb = ((gz >> logB) * G + (gy >> logB)) * G + (gx >> logB);
            const int32_t gid = ind[nb];
            if (gid >= 0 && gid < n_blocks) {
                const int32_t lx = gx & (B - 1), ly = gy & (B - 1), lz = gz & (B - 1);
                const int64_t vi = int64_t(gid) * B * B * B + (int64_t(lz) * B + ly) * B + lx;
                val[0] = dens[vi];
#pragma unroll
                for (int c = 0; c < 3; ++c) val[1 + c] = rgb[vi * 3 + c];
#pragma unroll
                for (int c = 0; c < 4; ++c) val[4 + c] = feat[vi * 4 + c];
            }
        }
    }
    T* out = reinterpret_cast<T*>(rec + int64_t(r) * rec_stride + dist_bytes + int64_t(v) * 8 * sizeof(T));
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = val[c];
}

constexpr int kMaxLine = 65;  // B + 1 for B = 64

// Distance pass along x: one thread per (record, cz, cy) line.  Computes
// each cell's activity from its 8 corner densities and the 1D distance to
// the nearest active cell of the line.
template <typename T>
__global__ void k_dist_x(int32_t B, int32_t n_blocks, int64_t rec_stride, int64_t dist_bytes,
                         uint8_t* __restrict__ rec) {
    const int32_t Bc = B + 1, Bp = B + 2;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n_blocks) * Bc * Bc) return;
    const int32_t r = int32_t(t / (Bc * Bc));
    const int32_t yz = int32_t(t - int64_t(r) * Bc * Bc);
    const int32_t cy = yz % Bc, cz = yz / Bc;
    uint8_t* dist = rec + int64_t(r) * rec_stride;
    const T* vox = reinterpret_cast<const T*>(dist + dist_bytes);
    int32_t last = -1000;
    for (int cx = 0; cx < Bc; ++cx) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t v = ((cz + (k >> 2)) * Bp + (cy + ((k >> 1) & 1))) * Bp + (cx + (k & 1));
            any |= vox[int64_t(v) * 8] != T(0);
        }
        if (any) last = cx;
        const int32_t d = cx - last;
        dist[(cz * Bc + cy) * Bc + cx] = uint8_t(d > 255 ? 255 : d);
    }
    last = 1000 + Bc;
    for (int cx = Bc - 1; cx >= 0; --cx) {
        uint8_t* q = &dist[(cz * Bc + cy) * Bc + cx];
        if (*q == 0) last = cx;
        const int32_t d = last - cx;
        if (d < *q) *q = uint8_t(d);
    }
}

// Distance pass along y (axis = 1) or z (axis = 2): one thread per line;
// out[i] = min_j max(|i - j|, in[j]) turns the distance to the nearest active
// cell in the lower dimensions into the Chebyshev distance in one more axis.
__global__ void k_dist_line(int32_t B, int32_t n_blocks, int32_t axis, int64_t rec_stride,
                            uint8_t* __restrict__ rec) {
    const int32_t Bc = B + 1;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n_blocks) * Bc * Bc) return;
    const int32_t r = int32_t(t / (Bc * Bc));
    const int32_t uv = int32_t(t - int64_t(r) * Bc * Bc);
    const int32_t u = uv % Bc, w = uv / Bc;
    uint8_t* dist = rec + int64_t(r) * rec_stride;
    // axis 1: cells (u, i, w) = x u, y i, z w; axis 2: (u, w, i) = x u, y w, z i
    const int32_t stride = axis == 1 ? Bc : Bc * Bc;
    const int32_t base = axis == 1 ? (w * Bc * Bc + u) : (w * Bc + u);
    uint8_t in[kMaxLine];
    for (int i = 0; i < Bc; ++i) in[i] = dist[base + i * stride];
    for (int i = 0; i < Bc; ++i) {
        int32_t best = 255;
        for (int j = 0; j < Bc; ++j) {
            const int32_t dj = i > j ? i - j : j - i;
            const int32_t m = dj > in[j] ? dj : in[j];
            best = m < best ? m : best;
        }
        dist[base + i * stride] = uint8_t(best);
    }
}

static inline unsigned nblk(int64_t n, int t) { return unsigned((n + t - 1) / t); }

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_pack(const PackedLayout& L, int32_t n_blocks, bool f32, const int32_t* ind,
                       const void* dens, const void* rgb, const void* feat, uint8_t* packed, hipStream_t s) {
    uint2* occ = reinterpret_cast<uint2*>(packed + L.off_occ);
    int32_t* rank_lin = reinterpret_cast<int32_t*>(packed + L.off_rank_lin);
    int32_t* rank_id = reinterpret_cast<int32_t*>(packed + L.off_rank_id);
    uint8_t* rec = packed + L.off_rec;
    const int64_t G3 = int64_t(L.G) * L.G * L.G;
    hipError_t e;
    hipLaunchKernelGGL(k_occ_bits, dim3(nblk(L.n_words, 256)), dim3(256), 0, s, ind, G3, n_blocks, L.n_words, occ);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_occ_scan, dim3(1), dim3(1024), 0, s, occ, L.n_words);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_blocks == 0) return hipSuccess;
    if ((e = launch_fill_i32(rank_lin, n_blocks, -1, s)) != hipSuccess) return e;
    if ((e = launch_fill_i32(rank_id, n_blocks, -1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_maps, dim3(nblk(G3, 256)), dim3(256), 0, s, ind, occ, G3, n_blocks, rank_lin,
                       rank_id);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t total = int64_t(n_blocks) * L.Bp * L.Bp * L.Bp;
    const int64_t lines = int64_t(n_blocks) * L.Bc * L.Bc;
    if (f32) {
        hipLaunchKernelGGL(k_pack_vox<float>, dim3(nblk(total, 256)), dim3(256), 0, s, ind, rank_lin,
                           (const float*)dens, (const float*)rgb, (const float*)feat, L.N, L.B, L.logB, n_blocks,
                           total, L.rec_stride, L.dist_bytes, rec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_dist_x<float>, dim3(nblk(lines, 256)), dim3(256), 0, s, L.B, n_blocks, L.rec_stride,
                           L.dist_bytes, rec);
    } else {
        hipLaunchKernelGGL(k_pack_vox<uint8_t>, dim3(nblk(total, 256)), dim3(256), 0, s, ind, rank_lin,
                           (const uint8_t*)dens, (const uint8_t*)rgb, (const uint8_t*)feat, L.N, L.B, L.logB,
                           n_blocks, total, L.rec_stride, L.dist_bytes, rec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_dist_x<uint8_t>, dim3(nblk(lines, 256)), dim3(256), 0, s, L.B, n_blocks,
                           L.rec_stride, L.dist_bytes, rec);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int axis = 1; axis <= 2; ++axis) {
        hipLaunchKernelGGL(k_dist_line, dim3(nblk(lines, 256)), dim3(256), 0, s, L.B, n_blocks, axis,
                           L.rec_stride, rec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace snerg
