// Host-side interface between the C ABI (api.cpp) and the HIP kernels.
#pragma once

#include "snerg_dev.h"

namespace snerg {

enum LaunchMode : int32_t {
    kModeTiles = 0,       // one wavefront per 64-pixel tile, one launch
    kModePersistent = 1,  // resident workgroups pull tiles from a global counter
    kModeList = 2,        // one lane per entry of a ray-id list
};

enum MlpMode : int32_t {
    kMlpOff = 0,
    kMlpF32 = 1,   // FP32 per lane
    kMlpF16 = 2,   // FP16 MFMA tiles, FP32 accumulation
};

struct RenderArgs {
    GridArgs grid;
    RenderOpts opts;
    const float* mlp;
    const DevCamera* cams;
    int32_t n_cams;
    int32_t mode;
    const int64_t* ray_ids;
    int64_t n_rays;
    int64_t total_tiles;
    int32_t tile_w, tile_h;  // tile_w * tile_h == 64
    int32_t list_rpw;        // set by the launch: rays per wavefront of a ray-list launch
    int32_t* tile_counter;   // persistent mode
    const int32_t* tile_order;  // tile of each wavefront slot / queue entry (null: identity)
    float* out;              // [n][4]
    float* aux;              // [n][8] or null
    // visit tracing
    int32_t* visits;
    int32_t max_visits;
    int32_t* counts;
    int32_t* counters;       // trace: [n][5]; counted render: [n][7] (null: the plain render)
};

struct BackwardArgs {
    GridArgs grid;
    RenderOpts opts;
    const float* mlp;
    const DevCamera* cams;
    int32_t n_cams;
    int32_t mlp_mode;
    const int64_t* ray_ids;
    int64_t n_rays;
    const float* aux;
    const float* grad_rgba;
    float* g_mlp_partial;  // [rows][883], rows = backward_partial_rows(n_groups)
    float* gcv;            // [n_rays][8]: g_C (3), g_V (4) per ray from the MLP backward
    float* grad_dens;
    float* grad_rgb;
    float* grad_feat;
    int64_t total_tiles;   // tile_w x tile_h tiles over all cameras (no ray list)
    int32_t tile_w, tile_h;
    int32_t mlp_only;      // MLP gradient only: no re-march
    int32_t patch_rays;    // ray list in groups of 64 neighbouring rays
    int32_t grad_packed;   // grid gradients as grad_dens[voxel][8] (grad_rgb, grad_feat unused)
    int32_t list_rpw;      // set by the launch: rays per wavefront of the list gradient pass
    // short ray lists, two phases (null: one re-march): per list entry
    // kBackwardListCap listed samples, the count and the last listed k
    int4* list;
    int32_t* list_count;
    int64_t* list_klast;
};

// The two-phase backward serves ray lists of at most kBackwardListMaxRays
// rays (few wavefronts, so the slowest one sets the time).
constexpr int kBackwardListCap = 512;
constexpr int64_t kBackwardListMaxRays = int64_t(1) << 18;

// Baking (Section 5.3, 5.4).
struct BakeCullPlan {
    const float* sigma;     // dense [N^3]
    const DevCamera* cams;
    int32_t n_cams;
    int32_t N, logB, G;
    int64_t total_tiles;    // training-ray tiles
    int32_t tile_w, tile_h;
    bool vec4;              // B >= 4 and sigma 16-byte aligned
    double sigma_thr, sum_thr;
    float* bmax;            // scratch [G^3]
    uint64_t* depth_bits;   // scratch [G^3]
    float* block_alpha;     // nullable
    float* block_vis;       // nullable
    int32_t* indirection;
    int32_t* n_blocks_dev;
};

struct BakeQuantPlan {
    const float* sigma;
    const float* rgb;
    const float* feat;
    const int32_t* indirection;
    int32_t n_blocks;
    int32_t N, logB, G;
    bool vec4;              // B >= 4, inputs 16-byte and outputs 4-byte aligned
    float k_sigma;
    int32_t* lin_of;        // scratch [n_blocks]
    uint8_t* dens8;
    uint8_t* rgb8;
    uint8_t* feat8;
};

hipError_t launch_bake_cull(const BakeCullPlan& p, hipStream_t s);
hipError_t launch_bake_quantize(const BakeQuantPlan& p, hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_pack(const PackedLayout& L, int32_t n_blocks, bool f32, const int32_t* ind,
                       const void* dens, const void* rgb, const void* feat, uint8_t* packed,
                       hipStream_t s);

// vt: 0 = uint8 grid, 1 = float32 grid.
hipError_t launch_render(const RenderArgs& a, int vt, int mlp_mode, int waves_per_group,
                         int n_groups, hipStream_t s);
hipError_t launch_trace(const RenderArgs& a, int vt, hipStream_t s);
// Heavy-first tile order for a tiled or persistent render: `cls` [total_tiles]
// and `counts` [33] are scratch (counts zero on entry, left zero on exit),
// `order` [total_tiles] receives the order (null: nothing to do).
constexpr int kCostClasses = 16;
hipError_t launch_tile_order(const RenderArgs& a, uint8_t* cls, int32_t* counts, int32_t* order, hipStream_t s);
hipError_t launch_backward(const BackwardArgs& a, int n_groups, hipStream_t s);
int backward_partial_rows(int n_groups);
// Gradient aggregation in LDS needs int32 voxel keys (fewer than 2^31 voxels).
bool backward_aggregates(const GridArgs& g);
hipError_t launch_render_ps(const RenderArgs& a, int vt, bool f16, int wpg, int n_groups, hipStream_t s);
hipError_t launch_mse(const float* rgba, const float* target, const int64_t* ids, int64_t n, float* grad, float* loss,
                      hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_reduce_mlp(const float* partial, int n_groups, float* out, hipStream_t s);

}  // namespace snerg
