// Forward kernels: march + composite + deferred MLP (Section 5.2, Eq. 5-7),
// and the visit-trace kernel.
#include "march.h"
#include "mlp.h"
#include "snerg_launch.h"

namespace snerg {

struct RayAccum {
    float C[3], V[4], T;
    bool gate;
};

// Composites one active sample (Eq. 2, 5, 6); kx = sigma_scale * delta / value scale.
__device__ __forceinline__ void composite(RayAccum& st, const Sample& smp, float kx, float cs) {
    const float x = smp.sigma_raw * kx;
    const float e = __expf(-x);
    const float alpha = 1.0f - e;
    const float w = st.T * alpha;
    const float wc = w * cs;
    st.C[0] += wc * smp.rgb[0];
    st.C[1] += wc * smp.rgb[1];
    st.C[2] += wc * smp.rgb[2];
    st.V[0] += wc * smp.feat[0];
    st.V[1] += wc * smp.feat[1];
    st.V[2] += wc * smp.feat[2];
    st.V[3] += wc * smp.feat[3];
    st.T *= e;
    st.gate = true;
}

// Per-ray counters of the render's own walk (the counted launch): the
// march's FlatWalk hooks count macroblocks and in-block samples, the sample
// callback the composited samples, their indices and the stop.
struct RayCount {
    int32_t blocks, occupied, in_block, active, stop_k;
    uint32_t k_sum, k_sq;
    __device__ __forceinline__ void block(bool occ) {
        ++blocks;
        occupied += occ ? 1 : 0;
    }
    __device__ __forceinline__ void inblock(int32_t n) { in_block += n; }
};

template <int VT, bool COUNT>
__device__ __forceinline__ void march_composite(const RenderArgs& a, const uint2* occ, const int64_t o[3],
                                                const int32_t s[3], RayAccum& st, RayCount& rc) {
    const GridArgs& g = a.grid;
    const float cs = VT == 0 ? (1.0f / 255.0f) : 1.0f;
    const float kx = g.sigma_scale * cs / float(g.N);
    const float t_stop = a.opts.t_stop;
    const bool early = a.opts.early_stop != 0;
    const bool nn_gate = a.opts.nn_gate != 0;
    // Consecutive samples often fall in the same cell (the step is half a
    // voxel): its corners are then reused instead of loaded again.
    const uint8_t* cached = nullptr;
    Corners8 cn;
    const uint32_t nb = uint32_t(g.Bp), nbb = nb * nb;
    auto on_sample = [&](int64_t k, int32_t, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
            Sample smp;
            if (VT == 0) {
                const uint8_t* cell = vox + (uint64_t(cell_index(p, nb, nbb)) << 3);
                if (cell != cached) {
                    load_corners_u8(cell, g.Bp, cn);
                    cached = cell;
                }
                interp_u8(cn, fr, smp);
                if (nn_gate) smp.active = nearest_nonzero_u8(cn, fr);
            } else {
                gather_f32(vox, g.Bp, p, fr, smp, nn_gate);
            }
            if (!smp.active) return false;
            composite(st, smp, kx, cs);
            const bool stop = early && st.T < t_stop;
            if (COUNT) {
                const uint32_t ku = uint32_t(k);
                ++rc.active;
                rc.k_sum += ku;
                rc.k_sq += ku * ku;
                if (stop) rc.stop_k = int32_t(k);
            }
            return stop;
        };
    if (COUNT) {
        march_ray_flat(g, occ, o, s, on_sample, rc);
    } else {
        march_ray_flat(g, occ, o, s, on_sample);
    }
}

// The wavefront's tile or first ray index is the same in every lane; saying
// so keeps the camera lookup and everything derived from it in scalar
// registers.
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Copies the occupancy table into LDS (all threads of the workgroup call this).
__device__ __forceinline__ const uint2* stage_occupancy(const GridArgs& g) {
    extern __shared__ uint2 s_occ[];
    for (int w = threadIdx.x; w < g.n_words; w += blockDim.x) s_occ[w] = g.occ[w];
    __syncthreads();
    return s_occ;
}

// Pixel of lane `lane` in wavefront tile t; false when the tile overhangs the image.
__device__ __forceinline__ bool tile_pixel(const RenderArgs& a, int64_t t, int lane, int& ci, int& px,
                                           int& py, int64_t& rid) {
    ci = find_camera_by_tile(a.cams, a.n_cams, t);
    const DevCamera& c = a.cams[ci];
    const int64_t tl = t - c.tile_offset;
    const int tx = int(tl % c.tiles_x), ty = int(tl / c.tiles_x);
    px = tx * a.tile_w + (lane % a.tile_w);
    py = ty * a.tile_h + (lane / a.tile_w);
    rid = c.ray_offset + int64_t(py) * c.W + px;
    return px < c.W && py < c.H;
}

template <int VT, int MLP, bool COUNT>
__device__ __forceinline__ void render_ray(const RenderArgs& a, const uint2* occ, bool valid, int ci, int px,
                                           int py, int64_t out_idx) {
    RayAccum st = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, 1.0f, false};
    RayCount rc = {0, 0, 0, 0, -1, 0u, 0u};
    float d[3] = {0.f, 0.f, 1.f};
    if (valid) {
        int64_t o[3];
        int32_t s[3];
        ray_setup(a.cams[ci], a.grid.N, px, py, o, s, d);
        // keep the direction as three floats from here on (left alone, the
        // compiler carries its FP64 form through the march)
        asm volatile("" : "+v"(d[0]), "+v"(d[1]), "+v"(d[2]));
        march_composite<VT, COUNT>(a, occ, o, s, st, rc);
        if (a.opts.unpremultiply) {
            // Eq. 9: saturate alpha above 2/3, keep soft edges below
            const float al = 1.0f - st.T;
            if (al > 0.0f) {
                const float sc = fminf(1.0f, 1.5f * al) / al;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) st.C[ch] *= sc;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) st.V[ch] *= sc;
                st.T = 1.0f - al * sc;
            }
        }
    }
    float R[3] = {0.f, 0.f, 0.f};
    const bool use_mlp = valid && st.gate && a.opts.mlp_on;
    if (MLP == kMlpF32) {
        if (use_mlp) mlp_forward_f32(as_const(a.mlp), st.C, st.V, d, R);
    } else if (MLP == kMlpF16) {
        mlp_forward_f16_wave(as_const(a.mlp), use_mlp, st.C, st.V, d, R);
    }
    if (valid) {
        float4 out;
        out.x = st.C[0] + st.T * a.opts.bg[0] + R[0];
        out.y = st.C[1] + st.T * a.opts.bg[1] + R[1];
        out.z = st.C[2] + st.T * a.opts.bg[2] + R[2];
        out.w = 1.0f - st.T;
        reinterpret_cast<float4*>(a.out)[out_idx] = out;
        if (a.aux) {
            float4* ax = reinterpret_cast<float4*>(a.aux) + 2 * out_idx;
            ax[0] = make_float4(st.C[0], st.C[1], st.C[2], st.V[0]);
            ax[1] = make_float4(st.V[1], st.V[2], st.V[3], st.gate ? st.T : -1.0f);
        }
        if (COUNT) {
            int32_t* c = a.counters + 7 * out_idx;
            c[0] = rc.blocks;
            c[1] = rc.occupied;
            c[2] = rc.in_block;
            c[3] = rc.active;
            c[4] = rc.stop_k;
            c[5] = int32_t(rc.k_sum);
            c[6] = int32_t(rc.k_sq);
        }
    }
}

// PERSIST selects the persistent kernel (a loop over the global tile queue);
// the other kernel serves the one-wavefront-per-tile and ray-list launches.
// They are separate kernels so that each gets its own register allocation.
// COUNT: the counted launch, which also writes each ray's march counters.
template <int VT, int MLP, bool PERSIST, bool COUNT>
__global__ __launch_bounds__(256) void k_render(RenderArgs a) {
    const uint2* occ = stage_occupancy(a.grid);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpg = blockDim.x >> 6;
    // One inlined copy of the per-ray body; the launch modes differ only in
    // how a wavefront obtains its next 64 rays (wave-uniform control flow).
    int64_t t = a.mode == kModeList ? (int64_t(blockIdx.x) * wpg + wave) * a.list_rpw
                                    : int64_t(xcd_grouped(blockIdx.x, gridDim.x)) * wpg + wave;
    for (;;) {
        if (PERSIST) {
            int64_t v = 0;
            if (lane == 0) v = atomicAdd(a.tile_counter, 1);
            t = __shfl(v, 0);
        }
        t = wave_uniform(t);
        bool valid;
        int ci = 0, px = 0, py = 0;
        int64_t out_idx;
        if (a.mode == kModeList) {
            if (t >= a.n_rays) break;  // wave-uniform
            out_idx = t + lane;
            valid = lane < a.list_rpw && out_idx < a.n_rays;
            if (valid) {
                const int64_t r = a.ray_ids[out_idx];
                ci = find_camera_by_ray(a.cams, a.n_cams, r);
                const int64_t local = r - a.cams[ci].ray_offset;
                py = int(local / a.cams[ci].W);
                px = int(local - int64_t(py) * a.cams[ci].W);
            }
        } else {
            if (t >= a.total_tiles) break;  // wave-uniform; every wave reaches it
            valid = tile_pixel(a, a.tile_order ? int64_t(a.tile_order[t]) : t, lane, ci, px, py, out_idx);
        }
        render_ray<VT, MLP, COUNT>(a, occ, valid, ci, px, py, out_idx);
        if (!PERSIST) break;
    }
}

// Visit trace: one lane per listed ray (or per ray id when the list is absent).
template <int VT>
__global__ __launch_bounds__(256) void k_trace(RenderArgs a) {
    const uint2* occ = stage_occupancy(a.grid);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_rays) return;
    const int64_t r = a.ray_ids ? a.ray_ids[i] : i;
    const int ci = find_camera_by_ray(a.cams, a.n_cams, r);
    const DevCamera& c = a.cams[ci];
    const int64_t local = r - c.ray_offset;
    const int py = int(local / c.W), px = int(local - int64_t(py) * c.W);
    int64_t o[3];
    int32_t s[3];
    float d[3];
    ray_setup(c, a.grid.N, px, py, o, s, d);
    const GridArgs& g = a.grid;
    const float cs = VT == 0 ? (1.0f / 255.0f) : 1.0f;
    const float kx = g.sigma_scale * cs / float(g.N);
    RayAccum st = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, 1.0f, false};
    int32_t n_trav = 0, n_occ = 0, n_in = 0, n_act = 0;
    int32_t* vis = a.visits ? a.visits + i * a.max_visits : nullptr;
    const int64_t stop = march_ray(
        g, occ, o, s,
        [&](int32_t lin, bool occ) {
            ++n_trav;
            if (occ) {
                if (vis && n_occ < a.max_visits) vis[n_occ] = lin;
                ++n_occ;
            }
        },
        [&](int32_t n) { n_in += n; },
        [&](int64_t, int32_t, const uint8_t* vox, const int32_t p[3], const int32_t fr[3]) {
            Sample smp;
            if (VT == 0) {
                Corners8 cn;
                load_corners_u8(vox + (uint64_t(cell_index(p, uint32_t(g.Bp), uint32_t(g.Bp * g.Bp))) << 3), g.Bp, cn);
                interp_u8(cn, fr, smp);
                if (a.opts.nn_gate) smp.active = nearest_nonzero_u8(cn, fr);
            } else {
                gather_f32(vox, g.Bp, p, fr, smp, a.opts.nn_gate != 0);
            }
            if (!smp.active) return false;
            ++n_act;
            composite(st, smp, kx, cs);
            return a.opts.early_stop && st.T < a.opts.t_stop;
        });
    a.counts[i] = n_occ;
    if (a.counters) {
        int32_t* cn = a.counters + 5 * i;
        cn[0] = n_trav;
        cn[1] = n_occ;
        cn[2] = n_in;
        cn[3] = n_act;
        cn[4] = int32_t(stop);
    }
}

// Heavy-first tile order.  A frame lasts as long as its slowest wavefronts
// (tiles whose rays graze the surface and composite hundreds of samples);
// issued late, they run on an emptying machine and set the frame time.
// Tiles are therefore sorted by a cost class, the number of the tile's
// centre-ray samples that lie inside occupied macroblocks (before early
// termination, in steps of N/16, capped at 15), and the render takes them
// in decreasing class.  Pass 1: eight lanes per tile walk eighths of its
// centre ray and add their counts into its class; the class histogram.
// Pass 2: each workgroup reserves, per class, a range after all tiles of
// higher classes and writes its tiles there.
constexpr int kCostParts = 8;  // lanes per tile, each walking a part of the centre ray

__global__ __launch_bounds__(256) void k_tile_cost(RenderArgs a, uint8_t* __restrict__ cls,
                                                   int32_t* __restrict__ counts) {
    __shared__ int32_t hist[kCostClasses];
    if (threadIdx.x < kCostClasses) hist[threadIdx.x] = 0;
    const uint2* occ = stage_occupancy(a.grid);  // synchronises
    const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t t = gid / kCostParts;
    const int part = int(gid % kCostParts);
    int32_t k = 0;
    if (t < a.total_tiles) {
        const int ci = find_camera_by_tile(a.cams, a.n_cams, t);
        const DevCamera& c = a.cams[ci];
        const int64_t tl = t - c.tile_offset;
        const int tx = int(tl % c.tiles_x), ty = int(tl / c.tiles_x);
        const int px = min(tx * a.tile_w + a.tile_w / 2, c.W - 1);
        const int py = min(ty * a.tile_h + a.tile_h / 2, c.H - 1);
        int64_t o[3];
        int32_t sd[3];
        float d[3];
        ray_setup(c, a.grid.N, px, py, o, sd, d);
        k = occupied_samples_on_ray(a.grid, occ, o, sd, part, kCostParts);
    }
    // the parts of one tile are adjacent lanes of one wavefront
#pragma unroll
    for (int m = 1; m < kCostParts; m <<= 1) k += __shfl_xor(k, m);
    if (t < a.total_tiles && part == 0) {
        // classes of N/16 samples: a ray crossing the whole grid has up to
        // 2 sqrt(3) N samples, so rays with more than N samples inside
        // occupied blocks share the top class
        k = min(k / max(1, a.grid.N >> 4), kCostClasses - 1);
        cls[t] = uint8_t(k);
        atomicAdd(&hist[k], 1);
    }
    __syncthreads();
    if (threadIdx.x < kCostClasses && hist[threadIdx.x] > 0) atomicAdd(&counts[threadIdx.x], hist[threadIdx.x]);
}

// counts[0..15]: class sizes; counts[16..31]: per-class cursors; counts[32]:
// finished workgroups.  All zero on entry; the last workgroup to finish
// zeroes them again for the next frame (so no clearing launch is needed,
// also inside a replayed graph).
__global__ __launch_bounds__(256) void k_tile_sort(const uint8_t* __restrict__ cls, int32_t* __restrict__ counts,
                                                   int64_t total, int32_t* __restrict__ order) {
    __shared__ int32_t local[kCostClasses], base[kCostClasses];
    __shared__ bool last;
    if (threadIdx.x < kCostClasses) local[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int c = t < total ? int(cls[t]) : -1;
    const int32_t pos = c >= 0 ? atomicAdd(&local[c], 1) : 0;
    __syncthreads();
    if (threadIdx.x < kCostClasses) {
        int32_t off = 0;
        for (int q = kCostClasses - 1; q > int(threadIdx.x); --q) off += counts[q];
        const int32_t mine = local[threadIdx.x];
        base[threadIdx.x] = off + (mine > 0 ? atomicAdd(&counts[kCostClasses + threadIdx.x], mine) : 0);
    }
    __syncthreads();
    if (c >= 0) order[base[c] + pos] = int32_t(t);
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's reads of counts happen before its ticket
        last = atomicAdd(&counts[2 * kCostClasses], 1) == int32_t(gridDim.x) - 1;
    }
    __syncthreads();
    if (last && threadIdx.x <= 2 * kCostClasses) {
        __threadfence();
        atomicExch(&counts[threadIdx.x], 0);
    }
}

hipError_t launch_tile_order(const RenderArgs& a, uint8_t* cls, int32_t* counts, int32_t* order, hipStream_t s) {
    if (a.total_tiles <= 0 || !order) return hipSuccess;
    // kCostParts lanes per tile: the walk is a latency chain, so spread it over many lanes
    const unsigned cblocks = unsigned((a.total_tiles * kCostParts + 255) / 256);
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2);
    hipLaunchKernelGGL(k_tile_cost, dim3(cblocks), dim3(256), lds, s, a, cls, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = unsigned((a.total_tiles + 255) / 256);
    hipLaunchKernelGGL(k_tile_sort, dim3(blocks), dim3(256), 0, s, cls, counts, a.total_tiles, order);
    return hipGetLastError();
}

template <int VT, int MLP>
static hipError_t launch_render_t(const RenderArgs& args, int wpg, int n_groups, hipStream_t s) {
    const int threads = 64 * wpg;
    // A ray list of up to 2^16 rays fills at most one wavefront per SIMD at
    // 64 rays each, and a lone wavefront waits on its own latencies: such
    // lists go 32 (up to 2^16) or 16 (up to 2^15) rays to a wavefront.
    RenderArgs a = args;
    a.list_rpw = a.n_rays <= (int64_t(1) << 15) ? 16 : (a.n_rays <= (int64_t(1) << 16) ? 32 : 64);
    unsigned blocks;
    if (a.mode == kModeList) blocks = unsigned(((a.n_rays + a.list_rpw - 1) / a.list_rpw + wpg - 1) / wpg);
    else if (a.mode == kModeTiles) blocks = unsigned((a.total_tiles + wpg - 1) / wpg);
    else blocks = unsigned(n_groups);
    if (blocks == 0) return hipSuccess;
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2);
    const bool count = a.counters != nullptr;
    if (a.mode == kModePersistent) {
        if (count) hipLaunchKernelGGL((k_render<VT, MLP, true, true>), dim3(blocks), dim3(threads), lds, s, a);
        else hipLaunchKernelGGL((k_render<VT, MLP, true, false>), dim3(blocks), dim3(threads), lds, s, a);
    } else {
        if (count) hipLaunchKernelGGL((k_render<VT, MLP, false, true>), dim3(blocks), dim3(threads), lds, s, a);
        else hipLaunchKernelGGL((k_render<VT, MLP, false, false>), dim3(blocks), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_render(const RenderArgs& a, int vt, int mlp_mode, int wpg, int n_groups,
                         hipStream_t s) {
    if (a.opts.per_sample_mlp) return launch_render_ps(a, vt, mlp_mode == kMlpF16, wpg, n_groups, s);
    if (vt == 0) {
        if (mlp_mode == kMlpF16) return launch_render_t<0, kMlpF16>(a, wpg, n_groups, s);
        if (mlp_mode == kMlpF32) return launch_render_t<0, kMlpF32>(a, wpg, n_groups, s);
        return launch_render_t<0, kMlpOff>(a, wpg, n_groups, s);
    }
    if (mlp_mode == kMlpF16) return launch_render_t<1, kMlpF16>(a, wpg, n_groups, s);
    if (mlp_mode == kMlpF32) return launch_render_t<1, kMlpF32>(a, wpg, n_groups, s);
    return launch_render_t<1, kMlpOff>(a, wpg, n_groups, s);
}

hipError_t launch_trace(const RenderArgs& a, int vt, hipStream_t s) {
    if (a.n_rays <= 0) return hipSuccess;
    const unsigned blocks = unsigned((a.n_rays + 255) / 256);
    const size_t lds = size_t(a.grid.n_words) * sizeof(uint2);
    if (vt == 0) hipLaunchKernelGGL(k_trace<0>, dim3(blocks), dim3(256), lds, s, a);
    else hipLaunchKernelGGL(k_trace<1>, dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace snerg
