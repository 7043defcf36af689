// Packing of a canonical SNeRG atlas into the layout the render kernels read
// (layout described in snerg_dev.h).  Atlas ids outside [0, n_blocks) in the
// indirection grid are treated as empty everywhere, so no kernel can index
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

__global__ void k_pack_lin(const int32_t* __restrict__ ind, int64_t G3, int32_t n_blocks,
                           int32_t* __restrict__ block_lin) {
    int64_t lin = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (lin >= G3) return;
    int32_t id = ind[lin];
    if (id >= 0 && id < n_blocks) block_lin[id] = int32_t(lin);
}

// One thread per padded voxel of every atlas block.
template <typename T>
__global__ void k_pack_vox(const int32_t* __restrict__ ind, const int32_t* __restrict__ block_lin,
                           const T* __restrict__ dens, const T* __restrict__ rgb,
                           const T* __restrict__ feat, int32_t N, int32_t B, int32_t logB,
                           int32_t n_blocks, int64_t total, int64_t vox_stride,
                           uint8_t* __restrict__ vox) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int32_t Bp = B + 2;
    const int64_t per_block = int64_t(Bp) * Bp * Bp;
    const int32_t id = int32_t(t / per_block);
    const int32_t r = int32_t(t - int64_t(id) * per_block);
    const int32_t px = r % Bp, py = (r / Bp) % Bp, pz = r / (Bp * Bp);
    const int32_t G = N >> logB;
    T val[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    const int32_t lin = block_lin[id];
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
    T* out = reinterpret_cast<T*>(vox + int64_t(id) * vox_stride + int64_t(r) * 8 * sizeof(T));
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = val[c];
}

// One thread per mask word.
template <typename T>
__global__ void k_pack_mask(const uint8_t* __restrict__ vox, int32_t B, int32_t n_blocks,
                            int32_t mask_words, int64_t vox_stride, uint32_t* __restrict__ mask) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n_blocks) * mask_words) return;
    const int32_t id = int32_t(t / mask_words);
    const int32_t w = int32_t(t - int64_t(id) * mask_words);
    const int32_t Bp = B + 2, Bc = B + 1;
    const int32_t cells = Bc * Bc * Bc;
    const T* base = reinterpret_cast<const T*>(vox + int64_t(id) * vox_stride);
    uint32_t bits = 0;
    for (int j = 0; j < 32; ++j) {
        const int32_t c = w * 32 + j;
        if (c >= cells) break;
        const int32_t px = c % Bc, py = (c / Bc) % Bc, pz = c / (Bc * Bc);
        bool any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t v = ((pz + (k >> 2)) * Bp + (py + ((k >> 1) & 1))) * Bp + (px + (k & 1));
            any |= base[int64_t(v) * 8] != T(0);
        }
        bits |= uint32_t(any) << j;
    }
    mask[t] = bits;
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
                       const void* dens, const void* rgb, const void* feat, uint8_t* packed,
                       hipStream_t s) {
    int32_t* block_lin = reinterpret_cast<int32_t*>(packed + L.off_lin);
    uint32_t* mask = reinterpret_cast<uint32_t*>(packed + L.off_mask);
    uint8_t* vox = packed + L.off_vox;
    const int64_t G3 = int64_t(L.G) * L.G * L.G;
    hipError_t e = launch_fill_i32(block_lin, n_blocks, -1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack_lin, dim3(nblk(G3, 256)), dim3(256), 0, s, ind, G3, n_blocks, block_lin);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_blocks == 0) return hipSuccess;
    const int64_t total = int64_t(n_blocks) * L.Bp * L.Bp * L.Bp;
    const int64_t words = int64_t(n_blocks) * L.mask_words;
    if (f32) {
        hipLaunchKernelGGL(k_pack_vox<float>, dim3(nblk(total, 256)), dim3(256), 0, s, ind, block_lin,
                           (const float*)dens, (const float*)rgb, (const float*)feat, L.N, L.B, L.logB,
                           n_blocks, total, L.vox_stride, vox);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_pack_mask<float>, dim3(nblk(words, 256)), dim3(256), 0, s, vox, L.B,
                           n_blocks, L.mask_words, L.vox_stride, mask);
    } else {
        hipLaunchKernelGGL(k_pack_vox<uint8_t>, dim3(nblk(total, 256)), dim3(256), 0, s, ind,
                           block_lin, (const uint8_t*)dens, (const uint8_t*)rgb, (const uint8_t*)feat,
                           L.N, L.B, L.logB, n_blocks, total, L.vox_stride, vox);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_pack_mask<uint8_t>, dim3(nblk(words, 256)), dim3(256), 0, s, vox, L.B,
                           n_blocks, L.mask_words, L.vox_stride, mask);
    }
    return hipGetLastError();
}

}  // namespace snerg
