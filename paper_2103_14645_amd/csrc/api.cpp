// C ABI of the gfx950 SNeRG renderer: argument validation (host only, before
// any device work), the handle's small device buffers, launch planning,
// HIP-graph replay of the persistent launch and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "snerg.h"
#include "snerg_launch.h"

using namespace snerg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(SNERG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite3(const double v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }
double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int check_shape(int32_t N, int32_t B, int32_t n_blocks, int32_t dtype) {
    if (dtype != SNERG_U8 && dtype != SNERG_F32) return fail(SNERG_ERR_UNSUPPORTED, "dtype must be SNERG_U8 or SNERG_F32");
    if (!is_pow2(B) || B < 2 || B > 64) return fail(SNERG_ERR_UNSUPPORTED, "B must be a power of two in [2, 64]");
    if (N < 1) return fail(SNERG_ERR_INVALID_ARG, "N must be >= 1");
    if (N % B != 0) return fail(SNERG_ERR_UNSUPPORTED, "N must be a multiple of B");
    if (N > 16384) return fail(SNERG_ERR_RANGE, "N > 16384 overflows the Q16 lattice in int32");
    if (n_blocks < 0) return fail(SNERG_ERR_INVALID_ARG, "n_blocks must be >= 0");
    const int64_t G = N / B;
    if (G > 64) return fail(SNERG_ERR_UNSUPPORTED, "N/B > 64: the macroblock occupancy table must fit in LDS");
    if (n_blocks > G * G * G) return fail(SNERG_ERR_INVALID_ARG, "n_blocks exceeds (N/B)^3");
    return SNERG_OK;
}

int check_grid(const snerg_grid* g) {
    if (!g) return fail(SNERG_ERR_INVALID_ARG, "grid is NULL");
    int rc = check_shape(g->N, g->B, g->n_blocks, g->dtype);
    if (rc) return rc;
    if (!g->indirection) return fail(SNERG_ERR_INVALID_ARG, "grid->indirection is NULL");
    if (!g->packed && g->n_blocks > 0) return fail(SNERG_ERR_INVALID_ARG, "grid->packed is NULL");
    if (!std::isfinite(g->sigma_scale) || g->sigma_scale < 0.0f)
        return fail(SNERG_ERR_INVALID_ARG, "sigma_scale must be finite and >= 0");
    return SNERG_OK;
}

int check_cams(const snerg_camera* cams, int32_t n_cams, int64_t* total) {
    if (!cams) return fail(SNERG_ERR_INVALID_ARG, "cams is NULL");
    if (n_cams < 1) return fail(SNERG_ERR_INVALID_ARG, "n_cams must be >= 1");
    int64_t t = 0;
    for (int32_t c = 0; c < n_cams; ++c) {
        const snerg_camera& k = cams[c];
        char buf[96];
        std::snprintf(buf, sizeof buf, "camera %d: ", c);
        if (k.W < 1 || k.H < 1) return fail(SNERG_ERR_INVALID_ARG, std::string(buf) + "W and H must be >= 1");
        if (int64_t(k.W) * k.H > (int64_t(1) << 31)) return fail(SNERG_ERR_INVALID_ARG, std::string(buf) + "W*H > 2^31");
        if (!std::isfinite(k.focal) || k.focal <= 0.0) return fail(SNERG_ERR_INVALID_ARG, std::string(buf) + "focal must be finite and > 0");
        if (!finite3(k.eye) || !finite3(k.fwd) || !finite3(k.right) || !finite3(k.up))
            return fail(SNERG_ERR_INVALID_ARG, std::string(buf) + "non-finite camera vector");
        const double tol = 1e-6;
        if (std::fabs(dot3(k.fwd, k.fwd) - 1) > tol || std::fabs(dot3(k.right, k.right) - 1) > tol ||
            std::fabs(dot3(k.up, k.up) - 1) > tol || std::fabs(dot3(k.fwd, k.right)) > tol ||
            std::fabs(dot3(k.fwd, k.up)) > tol || std::fabs(dot3(k.right, k.up)) > tol)
            return fail(SNERG_ERR_INVALID_ARG, std::string(buf) + "fwd/right/up must be orthonormal");
        for (int a = 0; a < 3; ++a)
            if (std::fabs(k.eye[a]) > 1000.0) return fail(SNERG_ERR_RANGE, std::string(buf) + "|eye| > 1000");
        t += int64_t(k.W) * k.H;
    }
    *total = t;
    return SNERG_OK;
}

int check_opts(const snerg_opts* o) {
    if (!o) return fail(SNERG_ERR_INVALID_ARG, "opts is NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(o->bg[a])) return fail(SNERG_ERR_INVALID_ARG, "opts->bg must be finite");
    if (!std::isfinite(o->t_stop) || o->t_stop < 0.0f) return fail(SNERG_ERR_INVALID_ARG, "opts->t_stop must be finite and >= 0");
    const uint32_t known = SNERG_FLAG_MLP_FP16 | SNERG_FLAG_PERSISTENT | SNERG_FLAG_GRAPH | SNERG_FLAG_MLP_GRAD_ONLY |
                           SNERG_FLAG_NN_GATE | SNERG_FLAG_UNPREMULTIPLY | SNERG_FLAG_PER_SAMPLE_MLP |
                           SNERG_FLAG_PATCH_RAYS | SNERG_FLAG_ACCUMULATE | SNERG_FLAG_GRAD_PACKED;
    if (o->flags & ~known) return fail(SNERG_ERR_UNSUPPORTED, "unknown opts->flags bits");
    return SNERG_OK;
}

int check_tuning(const snerg_tuning* t) {
    if (!t) return fail(SNERG_ERR_INVALID_ARG, "tuning is NULL");
    if (t->tile_w < 1 || t->tile_h < 1 || t->tile_w * t->tile_h != 64)
        return fail(SNERG_ERR_INVALID_ARG, "tile_w * tile_h must be 64");
    if (t->waves_per_group != 1 && t->waves_per_group != 2 && t->waves_per_group != 4)
        return fail(SNERG_ERR_INVALID_ARG, "waves_per_group must be 1, 2 or 4");
    if (t->groups_per_cu < 1 || t->groups_per_cu > 16) return fail(SNERG_ERR_INVALID_ARG, "groups_per_cu must be in [1, 16]");
    return SNERG_OK;
}

GridArgs grid_args(const snerg_grid* g) {
    const PackedLayout L = make_layout(g->N, g->B, g->n_blocks, g->dtype == SNERG_F32 ? 32 : 8);
    const uint8_t* p = static_cast<const uint8_t*>(g->packed);
    GridArgs a;
    a.ind = g->indirection;
    a.occ = reinterpret_cast<const uint2*>(p + L.off_occ);
    a.rank_lin = reinterpret_cast<const int32_t*>(p + L.off_rank_lin);
    a.rank_id = reinterpret_cast<const int32_t*>(p + L.off_rank_id);
    a.rec = p + L.off_rec;
    a.N = L.N; a.B = L.B; a.logB = L.logB; a.G = L.G; a.Bp = L.Bp; a.Bc = L.Bc;
    a.n_words = L.n_words;
    a.n_blocks = g->n_blocks;
    a.rec_stride = L.rec_stride;
    a.dist_bytes = L.dist_bytes;
    a.sigma_scale = g->sigma_scale;
    return a;
}

RenderOpts render_opts(const snerg_opts* o) {
    RenderOpts r;
    for (int a = 0; a < 3; ++a) r.bg[a] = o->bg[a];
    r.t_stop = o->t_stop;
    r.early_stop = o->early_stop ? 1 : 0;
    r.mlp_on = o->mlp_on ? 1 : 0;
    r.nn_gate = (o->flags & SNERG_FLAG_NN_GATE) ? 1 : 0;
    r.unpremultiply = (o->flags & SNERG_FLAG_UNPREMULTIPLY) ? 1 : 0;
    r.per_sample_mlp = (o->flags & SNERG_FLAG_PER_SAMPLE_MLP) ? 1 : 0;
    return r;
}

}  // namespace

struct snerg_handle {
    int device = 0;
    int n_cu = 256;
    hipStream_t cap_stream = nullptr;
    DevCamera* d_cams = nullptr;
    size_t cams_cap = 0;
    DevCamera* h_cams = nullptr;  // pinned staging
    hipEvent_t cams_copied = nullptr;
    bool cams_pending = false;
    std::vector<DevCamera> last_cams;
    int32_t* d_counter = nullptr;
    float* d_partial = nullptr;
    size_t partial_cap = 0;
    float* d_gcv = nullptr;  // per-ray g_C, g_V of the backward pass
    size_t gcv_cap = 0;
    float* d_list = nullptr;  // two-phase backward of short ray lists: listed samples
    size_t list_cap = 0;
    float* d_list_meta = nullptr;  // and per ray the count (int32) and the last listed k (int64)
    size_t list_meta_cap = 0;
    float* d_tiles = nullptr;  // heavy-first tile order: counters [64], order [tiles] int32, classes [tiles] u8
    size_t tiles_cap = 0;      // in floats
    float* d_bake = nullptr;  // baking scratch: per-block max density, visibility words, atlas map
    size_t bake_cap = 0;      // in floats
    int32_t* h_bake_count = nullptr;  // pinned: kept-block count read back by snerg_bake_cull
    // kernel timing ring (measurement aid): every timing_every-th render
    // call is timed (0: none); timing_now says whether the current one is
    int32_t timing_every = 0;
    int64_t timing_calls = 0;
    bool timing_now = false;
    std::vector<hipEvent_t> t_start, t_stop;
    int64_t t_count = 0;
    snerg_tuning tuning = {8, 8, 4, 8};
    // autotuned launch shapes by workload signature (tuning_signature)
    std::unordered_map<uint64_t, snerg_tuning> tuned;
    // cached graph of {counter reset, persistent render}
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint8_t> graph_key;
};

namespace {

// Camera table for the current call: uploaded only when it changed.
int upload_cams(snerg_handle* h, const snerg_camera* cams, int32_t n_cams, int tile_w, int tile_h,
                hipStream_t s, int64_t* total_tiles) {
    std::vector<DevCamera> t(n_cams);
    int64_t rays = 0, tiles = 0;
    for (int32_t c = 0; c < n_cams; ++c) {
        DevCamera& d = t[c];
        std::memset(&d, 0, sizeof d);
        for (int a = 0; a < 3; ++a) {
            d.eye[a] = cams[c].eye[a];
            d.fwd[a] = cams[c].fwd[a];
            d.right[a] = cams[c].right[a];
            d.up[a] = cams[c].up[a];
        }
        d.focal = cams[c].focal;
        d.W = cams[c].W;
        d.H = cams[c].H;
        d.ray_offset = rays;
        d.tile_offset = tiles;
        d.tiles_x = (cams[c].W + tile_w - 1) / tile_w;
        d.tiles_y = (cams[c].H + tile_h - 1) / tile_h;
        rays += int64_t(cams[c].W) * cams[c].H;
        tiles += int64_t(d.tiles_x) * d.tiles_y;
    }
    *total_tiles = tiles;
    if (h->last_cams.size() == t.size() &&
        std::memcmp(h->last_cams.data(), t.data(), t.size() * sizeof(DevCamera)) == 0)
        return SNERG_OK;
    if (size_t(n_cams) > h->cams_cap) {
        if (h->cams_pending) HIP_TRY(hipEventSynchronize(h->cams_copied));
        h->cams_pending = false;
        if (h->d_cams) HIP_TRY(hipFree(h->d_cams));
        if (h->h_cams) HIP_TRY(hipHostFree(h->h_cams));
        h->d_cams = nullptr;
        h->h_cams = nullptr;
        h->graph_key.clear();
        size_t cap = std::max<size_t>(64, size_t(n_cams));
        HIP_TRY(hipMalloc(&h->d_cams, cap * sizeof(DevCamera)));
        HIP_TRY(hipHostMalloc(&h->h_cams, cap * sizeof(DevCamera), hipHostMallocDefault));
        h->cams_cap = cap;
    }
    if (h->cams_pending) HIP_TRY(hipEventSynchronize(h->cams_copied));  // staging buffer reuse
    std::memcpy(h->h_cams, t.data(), t.size() * sizeof(DevCamera));
    HIP_TRY(hipMemcpyAsync(h->d_cams, h->h_cams, t.size() * sizeof(DevCamera), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(h->cams_copied, s));
    h->cams_pending = true;
    h->last_cams = t;
    return SNERG_OK;
}

// Grows a handle-owned float buffer.  The old buffer may still be read by
// work queued on the handle's stream, so that work is waited for before the
// buffer is freed; growing by half again as much as asked keeps a sequence
// of slowly growing calls from reallocating (and waiting) every time.
int ensure_buffer(float** buf, size_t* cap, size_t need, hipStream_t s) {
    if (need <= *cap) return SNERG_OK;
    if (*buf) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(*buf));
    }
    *buf = nullptr;
    *cap = 0;
    const size_t want = need + need / 2;
    HIP_TRY(hipMalloc(buf, want * sizeof(float)));
    *cap = want;
    return SNERG_OK;
}

// Shared checks; n_rays < 0 means "all rays" (the caller passes no count).
int common_render_checks(const snerg_grid* grid, const float* mlp, bool need_mlp, const snerg_camera* cams,
                         int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                         int64_t* total) {
    int rc;
    if ((rc = check_grid(grid))) return rc;
    if ((rc = check_cams(cams, n_cams, total))) return rc;
    if ((rc = check_opts(opts))) return rc;
    if (need_mlp && opts->mlp_on && !mlp) return fail(SNERG_ERR_INVALID_ARG, "mlp is NULL while opts->mlp_on");
    if (ray_ids && n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    if (!ray_ids && n_rays >= 0 && n_rays != *total)
        return fail(SNERG_ERR_INVALID_ARG, "without ray_ids, n_rays must equal the total pixel count");
    return SNERG_OK;
}

constexpr int kTimingRing = 256;

// Events around the render kernel when timing is enabled (no-ops otherwise).
hipError_t timing_begin(snerg_handle* h, hipStream_t s) {
    h->timing_now = h->timing_every > 0 && h->timing_calls++ % h->timing_every == 0;
    if (!h->timing_now) return hipSuccess;
    return hipEventRecord(h->t_start[size_t(h->t_count % kTimingRing)], s);
}
hipError_t timing_end(snerg_handle* h, hipStream_t s) {
    if (!h->timing_now) return hipSuccess;
    hipError_t e = hipEventRecord(h->t_stop[size_t(h->t_count % kTimingRing)], s);
    ++h->t_count;
    return e;
}

// What a launch shape's speed depends on: the grid's shape and occupancy,
// the image sizes, and the options that select a kernel (FNV-1a over them).
uint64_t tuning_signature(const snerg_grid* g, const snerg_camera* cams, int32_t n_cams, const snerg_opts* o) {
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            x ^= uint64_t(v >> (8 * b)) & 0xFFu;
            x *= 1099511628211ull;
        }
    };
    mix(g->N); mix(g->B); mix(g->n_blocks); mix(g->dtype);
    mix(n_cams);
    for (int32_t c = 0; c < n_cams; ++c) { mix(cams[c].W); mix(cams[c].H); }
    const uint32_t kernel_flags = SNERG_FLAG_MLP_FP16 | SNERG_FLAG_PERSISTENT | SNERG_FLAG_GRAPH | SNERG_FLAG_NN_GATE |
                                  SNERG_FLAG_UNPREMULTIPLY | SNERG_FLAG_PER_SAMPLE_MLP;
    mix(o->flags & kernel_flags); mix(o->mlp_on ? 1 : 0); mix(o->early_stop ? 1 : 0);
    return x;
}

// The launch shape for a render: the autotuned one for this workload if
// there is one, else the handle's.
snerg_tuning tuning_for(const snerg_handle* h, const snerg_grid* g, const snerg_camera* cams, int32_t n_cams,
                        const snerg_opts* o) {
    if (!h->tuned.empty()) {
        auto it = h->tuned.find(tuning_signature(g, cams, n_cams, o));
        if (it != h->tuned.end()) return it->second;
    }
    return h->tuning;
}

int render_impl(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                float* out_rgba, float* aux, hipStream_t s, const snerg_tuning& tu,
                int32_t* counters = nullptr) {
    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    int64_t total_tiles = 0;
    int rc = upload_cams(h, cams, n_cams, tu.tile_w, tu.tile_h, s, &total_tiles);
    if (rc) return rc;
    a.grid = grid_args(grid);
    a.opts = render_opts(opts);
    a.mlp = mlp;
    a.cams = h->d_cams;
    a.n_cams = n_cams;
    a.ray_ids = ray_ids;
    a.n_rays = n_rays;
    a.total_tiles = total_tiles;
    a.tile_w = tu.tile_w;
    a.tile_h = tu.tile_h;
    a.tile_counter = h->d_counter;
    a.out = out_rgba;
    a.aux = aux;
    a.counters = counters;
    const int vt = grid->dtype == SNERG_F32 ? 1 : 0;
    const int mlp_mode = !opts->mlp_on ? kMlpOff : ((opts->flags & SNERG_FLAG_MLP_FP16) ? kMlpF16 : kMlpF32);
    const int wpg = tu.waves_per_group;
    if (ray_ids) {
        a.mode = kModeList;
        HIP_TRY(timing_begin(h, s));
        HIP_TRY(launch_render(a, vt, mlp_mode, wpg, 0, s));
        HIP_TRY(timing_end(h, s));
        return SNERG_OK;
    }
    // heavy-first tile order (scheduling only: every tile's result is unchanged;
    // int32 entries, so frames of more than 2^31 - 1 tiles keep image order)
    // layout: counters [64] (fixed place), order [tiles], classes [tiles] bytes
    int32_t* counts = nullptr;
    int32_t* order = nullptr;
    uint8_t* cls = nullptr;
    if (total_tiles <= int64_t(INT32_MAX)) {
        const size_t order_words = 64 + size_t(total_tiles);
        float* const before = h->d_tiles;
        if ((rc = ensure_buffer(&h->d_tiles, &h->tiles_cap, order_words + (size_t(total_tiles) + 3) / 4, s))) return rc;
        counts = reinterpret_cast<int32_t*>(h->d_tiles);
        order = counts + 64;
        cls = reinterpret_cast<uint8_t*>(h->d_tiles + order_words);
        if (h->d_tiles != before) {
            // the order kernels leave their counters at zero; a new buffer starts at zero
            HIP_TRY(launch_fill_i32(counts, 64, 0, s));
        }
    }
    a.tile_order = order;
    const bool persistent = (opts->flags & SNERG_FLAG_PERSISTENT) != 0;
    a.mode = persistent ? kModePersistent : kModeTiles;
    const int n_groups = persistent ? h->n_cu * tu.groups_per_cu : 0;
    if (!(opts->flags & SNERG_FLAG_GRAPH)) {
        HIP_TRY(launch_tile_order(a, cls, counts, order, s));
        if (persistent) HIP_TRY(launch_fill_i32(h->d_counter, 1, 0, s));
        HIP_TRY(timing_begin(h, s));
        HIP_TRY(launch_render(a, vt, mlp_mode, wpg, n_groups, s));
        HIP_TRY(timing_end(h, s));
        return SNERG_OK;
    }
    // Graph replay: the key is every launch parameter; the camera table's
    // contents live in device memory outside the graph.
    std::vector<uint8_t> key(sizeof a + 3 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof a);
    const int extra[3] = {vt, mlp_mode, wpg * 1000 + n_groups};
    std::memcpy(key.data() + sizeof a, extra, sizeof extra);
    if (!h->graph_exec || key != h->graph_key) {
        if (h->graph_exec) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipGraphExecDestroy(h->graph_exec));
            h->graph_exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = launch_tile_order(a, cls, counts, order, h->cap_stream);
        if (e1 == hipSuccess && persistent) e1 = launch_fill_i32(h->d_counter, 1, 0, h->cap_stream);
        hipError_t e2 = e1 == hipSuccess ? launch_render(a, vt, mlp_mode, wpg, n_groups, h->cap_stream) : e1;
        hipError_t e3 = hipStreamEndCapture(h->cap_stream, &graph);
        if (e2 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return fail(SNERG_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e2));
        }
        HIP_TRY(e3);
        hipError_t e4 = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        HIP_TRY(e4);
        h->graph_key = key;
    }
    HIP_TRY(timing_begin(h, s));
    HIP_TRY(hipGraphLaunch(h->graph_exec, s));
    HIP_TRY(timing_end(h, s));
    return SNERG_OK;
}

// ------------------------------------------------ allocation-free render

// Every scratch buffer of the render path in one fixed device array, for
// callers that cannot allocate (snerg_render_noalloc).  Layout: tile-order
// class counters (64 int32), the persistent launch's tile counter, the
// camera table (kNoAllocMaxCams entries), the tile order (int32 per tile) and
// the tile classes (one byte per tile).  Each GPU holds its own copy; its
// address comes from hipGetSymbolAddress with that GPU current.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int32_t kNoAllocMaxCams = 1024;
constexpr size_t kScrCounts = 0;
constexpr size_t kScrCounter = 256;
constexpr size_t kScrCams = 512;
constexpr size_t kScrOrder = (kScrCams + size_t(kNoAllocMaxCams) * sizeof(DevCamera) + 255) & ~size_t(255);
constexpr int64_t kNoAllocMaxTiles = int64_t((kScratchBytes - kScrOrder) / 5);
static_assert(kNoAllocMaxTiles == 3327488, "the limit stated in snerg.h");
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_on_current_device(uint8_t** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SNERG_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SNERG_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SNERG_OK;
}

// Camera rows go to the device as kernel arguments (no staging buffer).
constexpr int kCamsPerLaunch = 24;
struct CamBatch {
    DevCamera c[kCamsPerLaunch];
    int32_t n, first;
};
static_assert(sizeof(CamBatch) + sizeof(void*) < 4096, "kernel arguments stay below 4 KB");

__global__ void k_put_cams(CamBatch b, DevCamera* dst) {
    const int i = int(threadIdx.x);
    if (i < b.n) dst[b.first + i] = b.c[i];
}

}  // namespace

extern "C" {

const char* snerg_status_string(int status) {
    switch (status) {
    case SNERG_OK: return "ok";
    case SNERG_ERR_INVALID_ARG: return "invalid argument";
    case SNERG_ERR_UNSUPPORTED: return "unsupported configuration";
    case SNERG_ERR_RANGE: return "fixed-point range exceeded";
    case SNERG_ERR_HIP: return "HIP runtime error";
    case SNERG_ERR_WORKSPACE: return "buffer too small";
    default: return "unknown status";
    }
}

const char* snerg_last_error(void) { return g_last_error.c_str(); }

int snerg_create(snerg_handle** out) {
    if (!out) return fail(SNERG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    snerg_handle* h = new (std::nothrow) snerg_handle();
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "out of host memory");
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->cams_copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&h->d_counter, 256);
    if (e != hipSuccess) {
        snerg_destroy(h);
        return fail(SNERG_ERR_HIP, std::string("snerg_create: ") + hipGetErrorString(e));
    }
    // look up this device's scratch array now, so that snerg_render_noalloc
    // finds it ready
    uint8_t* scr = nullptr;
    const int rc = scratch_on_current_device(&scr);
    if (rc) {
        snerg_destroy(h);
        return rc;
    }
    *out = h;
    return SNERG_OK;
}

int snerg_destroy(snerg_handle* h) {
    if (!h) return SNERG_OK;
    if (h->cams_pending) hipEventSynchronize(h->cams_copied);
    if (h->graph_exec) hipGraphExecDestroy(h->graph_exec);
    if (h->d_cams) hipFree(h->d_cams);
    if (h->h_cams) hipHostFree(h->h_cams);
    if (h->d_counter) hipFree(h->d_counter);
    if (h->d_partial) hipFree(h->d_partial);
    if (h->d_gcv) hipFree(h->d_gcv);
    if (h->d_list) hipFree(h->d_list);
    if (h->d_list_meta) hipFree(h->d_list_meta);
    if (h->d_bake) hipFree(h->d_bake);
    if (h->d_tiles) hipFree(h->d_tiles);
    for (hipEvent_t e : h->t_start) hipEventDestroy(e);
    for (hipEvent_t e : h->t_stop) hipEventDestroy(e);
    if (h->h_bake_count) hipHostFree(h->h_bake_count);
    if (h->cams_copied) hipEventDestroy(h->cams_copied);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    delete h;
    return SNERG_OK;
}

int snerg_packed_size(int32_t N, int32_t B, int32_t n_blocks, int32_t dtype, size_t* bytes) {
    if (!bytes) return fail(SNERG_ERR_INVALID_ARG, "bytes is NULL");
    int rc = check_shape(N, B, n_blocks, dtype);
    if (rc) return rc;
    *bytes = size_t(make_layout(N, B, n_blocks, dtype == SNERG_F32 ? 32 : 8).total);
    return SNERG_OK;
}

int snerg_pack_grid(snerg_handle* h, int32_t N, int32_t B, int32_t n_blocks, int32_t dtype,
                    const int32_t* indirection, const void* dens, const void* rgb, const void* feat,
                    void* packed, size_t packed_bytes, void* stream) {
    int rc = check_shape(N, B, n_blocks, dtype);
    if (rc) return rc;
    if (!indirection || !packed) return fail(SNERG_ERR_INVALID_ARG, "indirection/packed is NULL");
    if (n_blocks > 0 && (!dens || !rgb || !feat)) return fail(SNERG_ERR_INVALID_ARG, "dens/rgb/feat is NULL");
    const PackedLayout L = make_layout(N, B, n_blocks, dtype == SNERG_F32 ? 32 : 8);
    if (packed_bytes < size_t(L.total)) return fail(SNERG_ERR_WORKSPACE, "packed buffer smaller than snerg_packed_size()");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    HIP_TRY(launch_pack(L, n_blocks, dtype == SNERG_F32, indirection, dens, rgb, feat,
                        static_cast<uint8_t*>(packed), static_cast<hipStream_t>(stream)));
    return SNERG_OK;
}

int snerg_render(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                 int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                 float* out_rgba, float* aux, void* stream) {
    int64_t total = 0;
    if (n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    int rc = common_render_checks(grid, mlp, true, cams, n_cams, ray_ids, n_rays, opts, &total);
    if (rc) return rc;
    if (!out_rgba) return fail(SNERG_ERR_INVALID_ARG, "out_rgba is NULL");
    if (aux && (opts->flags & SNERG_FLAG_PER_SAMPLE_MLP))
        return fail(SNERG_ERR_UNSUPPORTED, "aux is not produced with SNERG_FLAG_PER_SAMPLE_MLP");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (n_rays == 0) return SNERG_OK;
    return render_impl(h, grid, mlp, cams, n_cams, ray_ids, n_rays, opts, out_rgba, aux,
                       static_cast<hipStream_t>(stream), tuning_for(h, grid, cams, n_cams, opts));
}

int snerg_render_noalloc(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                         int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                         float* out_rgba, float* aux, void* stream) {
    int64_t total = 0;
    if (n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    int rc = common_render_checks(grid, mlp, true, cams, n_cams, ray_ids, n_rays, opts, &total);
    if (rc) return rc;
    if (!out_rgba) return fail(SNERG_ERR_INVALID_ARG, "out_rgba is NULL");
    if (aux && (opts->flags & SNERG_FLAG_PER_SAMPLE_MLP))
        return fail(SNERG_ERR_UNSUPPORTED, "aux is not produced with SNERG_FLAG_PER_SAMPLE_MLP");
    if (opts->flags & SNERG_FLAG_GRAPH)
        return fail(SNERG_ERR_UNSUPPORTED, "snerg_render_noalloc does not build graphs (instantiation allocates)");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (n_cams > kNoAllocMaxCams)
        return fail(SNERG_ERR_WORKSPACE, "snerg_render_noalloc takes at most 1024 cameras");
    const snerg_tuning tu = tuning_for(h, grid, cams, n_cams, opts);
    int64_t tiles = 0;
    for (int32_t c = 0; c < n_cams; ++c)
        tiles += int64_t((cams[c].W + tu.tile_w - 1) / tu.tile_w) * ((cams[c].H + tu.tile_h - 1) / tu.tile_h);
    if (!ray_ids && tiles > kNoAllocMaxTiles)
        return fail(SNERG_ERR_WORKSPACE, "snerg_render_noalloc takes at most " + std::to_string(kNoAllocMaxTiles) +
                                             " tiles of 64 pixels per call");
    uint8_t* base = nullptr;
    if ((rc = scratch_on_current_device(&base))) return rc;
    if (n_rays == 0) return SNERG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevCamera* d_cams = reinterpret_cast<DevCamera*>(base + kScrCams);
    int32_t* counts = reinterpret_cast<int32_t*>(base + kScrCounts);
    int32_t* counter = reinterpret_cast<int32_t*>(base + kScrCounter);
    int32_t* order = reinterpret_cast<int32_t*>(base + kScrOrder);
    uint8_t* cls = base + kScrOrder + size_t(4) * size_t(tiles);
    // camera table, as in upload_cams
    CamBatch b;
    int64_t rays = 0, toff = 0;
    for (int32_t c0 = 0; c0 < n_cams; c0 += kCamsPerLaunch) {
        std::memset(&b, 0, sizeof b);
        b.first = c0;
        b.n = std::min<int32_t>(kCamsPerLaunch, n_cams - c0);
        for (int32_t j = 0; j < b.n; ++j) {
            const snerg_camera& k = cams[c0 + j];
            DevCamera& d = b.c[j];
            for (int a = 0; a < 3; ++a) {
                d.eye[a] = k.eye[a];
                d.fwd[a] = k.fwd[a];
                d.right[a] = k.right[a];
                d.up[a] = k.up[a];
            }
            d.focal = k.focal;
            d.W = k.W;
            d.H = k.H;
            d.ray_offset = rays;
            d.tile_offset = toff;
            d.tiles_x = (k.W + tu.tile_w - 1) / tu.tile_w;
            d.tiles_y = (k.H + tu.tile_h - 1) / tu.tile_h;
            rays += int64_t(k.W) * k.H;
            toff += int64_t(d.tiles_x) * d.tiles_y;
        }
        hipLaunchKernelGGL(k_put_cams, dim3(1), dim3(kCamsPerLaunch), 0, s, b, d_cams);
        HIP_TRY(hipGetLastError());
    }
    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    a.grid = grid_args(grid);
    a.opts = render_opts(opts);
    a.mlp = mlp;
    a.cams = d_cams;
    a.n_cams = n_cams;
    a.ray_ids = ray_ids;
    a.n_rays = n_rays;
    a.total_tiles = tiles;
    a.tile_w = tu.tile_w;
    a.tile_h = tu.tile_h;
    a.tile_counter = counter;
    a.out = out_rgba;
    a.aux = aux;
    const int vt = grid->dtype == SNERG_F32 ? 1 : 0;
    const int mlp_mode = !opts->mlp_on ? kMlpOff : ((opts->flags & SNERG_FLAG_MLP_FP16) ? kMlpF16 : kMlpF32);
    if (ray_ids) {
        a.mode = kModeList;
        HIP_TRY(launch_render(a, vt, mlp_mode, tu.waves_per_group, 0, s));
        return SNERG_OK;
    }
    const bool persistent = (opts->flags & SNERG_FLAG_PERSISTENT) != 0;
    a.mode = persistent ? kModePersistent : kModeTiles;
    a.tile_order = order;
    // the order kernels expect zero counters; the array keeps whatever the
    // last call left, so clear them (a fill kernel, no memset node)
    HIP_TRY(launch_fill_i32(counts, 64, 0, s));
    HIP_TRY(launch_tile_order(a, cls, counts, order, s));
    if (persistent) HIP_TRY(launch_fill_i32(counter, 1, 0, s));
    HIP_TRY(launch_render(a, vt, mlp_mode, tu.waves_per_group, persistent ? h->n_cu * tu.groups_per_cu : 0, s));
    return SNERG_OK;
}

int snerg_render_counted(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                         int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                         float* out_rgba, float* aux, int32_t* counters, void* stream) {
    int64_t total = 0;
    if (n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    int rc = common_render_checks(grid, mlp, true, cams, n_cams, ray_ids, n_rays, opts, &total);
    if (rc) return rc;
    if (!out_rgba || !counters) return fail(SNERG_ERR_INVALID_ARG, "out_rgba/counters is NULL");
    if (opts->flags & SNERG_FLAG_PER_SAMPLE_MLP)
        return fail(SNERG_ERR_UNSUPPORTED, "no counted render with SNERG_FLAG_PER_SAMPLE_MLP");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (n_rays == 0) return SNERG_OK;
    return render_impl(h, grid, mlp, cams, n_cams, ray_ids, n_rays, opts, out_rgba, aux,
                       static_cast<hipStream_t>(stream), tuning_for(h, grid, cams, n_cams, opts), counters);
}

int snerg_trace_visits(snerg_handle* h, const snerg_grid* grid, const snerg_camera* cams, int32_t n_cams,
                       const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts, int32_t max_visits,
                       int32_t* visits, int32_t* counts, int32_t* counters, void* stream) {
    int64_t total = 0;
    if (n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    int rc = common_render_checks(grid, nullptr, false, cams, n_cams, ray_ids, n_rays, opts, &total);
    if (rc) return rc;
    if (max_visits < 0) return fail(SNERG_ERR_INVALID_ARG, "max_visits must be >= 0");
    if (max_visits > 0 && !visits) return fail(SNERG_ERR_INVALID_ARG, "visits is NULL");
    if (!counts) return fail(SNERG_ERR_INVALID_ARG, "counts is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (n_rays == 0) return SNERG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t total_tiles = 0;
    rc = upload_cams(h, cams, n_cams, h->tuning.tile_w, h->tuning.tile_h, s, &total_tiles);
    if (rc) return rc;
    RenderArgs a;
    std::memset(&a, 0, sizeof a);
    a.grid = grid_args(grid);
    a.opts = render_opts(opts);
    a.cams = h->d_cams;
    a.n_cams = n_cams;
    a.ray_ids = ray_ids;
    a.n_rays = n_rays;
    a.visits = visits;
    a.max_visits = max_visits;
    a.counts = counts;
    a.counters = counters;
    HIP_TRY(launch_trace(a, grid->dtype == SNERG_F32 ? 1 : 0, s));
    return SNERG_OK;
}

int snerg_render_backward(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                          int32_t n_cams, const int64_t* ray_ids, int64_t n_rays, const snerg_opts* opts,
                          const float* aux, const float* grad_rgba, float* grad_mlp, float* grad_dens,
                          float* grad_rgb, float* grad_feat, void* stream) {
    int64_t total = 0;
    if (n_rays < 0) return fail(SNERG_ERR_INVALID_ARG, "n_rays must be >= 0");
    int rc = common_render_checks(grid, mlp, true, cams, n_cams, ray_ids, n_rays, opts, &total);
    if (rc) return rc;
    const bool mlp_only = (opts->flags & SNERG_FLAG_MLP_GRAD_ONLY) != 0;
    if (opts->flags & SNERG_FLAG_UNPREMULTIPLY)
        return fail(SNERG_ERR_UNSUPPORTED, "no backward through SNERG_FLAG_UNPREMULTIPLY");
    if (opts->flags & SNERG_FLAG_PER_SAMPLE_MLP)
        return fail(SNERG_ERR_UNSUPPORTED, "no backward through SNERG_FLAG_PER_SAMPLE_MLP");
    if (!mlp_only && grid->dtype != SNERG_F32)
        return fail(SNERG_ERR_UNSUPPORTED, "grid gradients need a SNERG_F32 grid");
    if (!aux || !grad_rgba) return fail(SNERG_ERR_INVALID_ARG, "aux/grad_rgba is NULL");
    if (!grad_mlp) return fail(SNERG_ERR_INVALID_ARG, "grad_mlp is NULL");
    const bool packed = (opts->flags & SNERG_FLAG_GRAD_PACKED) != 0;
    if (!mlp_only && packed && (!grad_dens || grad_rgb || grad_feat))
        return fail(SNERG_ERR_INVALID_ARG, "SNERG_FLAG_GRAD_PACKED takes grad_dens only (grad_rgb, grad_feat NULL)");
    if (!mlp_only && !packed && (!grad_dens || !grad_rgb || !grad_feat))
        return fail(SNERG_ERR_INVALID_ARG, "a grid gradient output is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t B3 = int64_t(grid->B) * grid->B * grid->B;
    const int64_t nv = int64_t(grid->n_blocks) * B3;
    const int64_t want = (n_rays + 127) / 128;
    const int n_groups = int(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(h->n_cu) * 8)));
    const int mlp_mode = !opts->mlp_on ? kMlpOff : ((opts->flags & SNERG_FLAG_MLP_FP16) ? kMlpF16 : kMlpF32);
    const int rows = backward_partial_rows(n_groups);
    if (mlp_mode != kMlpOff) {
        rc = ensure_buffer(&h->d_partial, &h->partial_cap, size_t(rows) * kMlpParams, s);
        if (rc) return rc;
        rc = ensure_buffer(&h->d_gcv, &h->gcv_cap, size_t(std::max<int64_t>(n_rays, 1)) * 8, s);
        if (rc) return rc;
    }
    int64_t total_tiles = 0;
    rc = upload_cams(h, cams, n_cams, h->tuning.tile_w, h->tuning.tile_h, s, &total_tiles);
    if (rc) return rc;
    const bool accumulate = (opts->flags & SNERG_FLAG_ACCUMULATE) != 0;
    if (!mlp_only && !accumulate) {
        if (packed) {
            HIP_TRY(launch_fill_f32(grad_dens, nv * 8, 0.0f, s));
        } else {
            HIP_TRY(launch_fill_f32(grad_dens, nv, 0.0f, s));
            HIP_TRY(launch_fill_f32(grad_rgb, nv * 3, 0.0f, s));
            HIP_TRY(launch_fill_f32(grad_feat, nv * 4, 0.0f, s));
        }
    }
    if (!accumulate) HIP_TRY(launch_fill_f32(grad_mlp, kMlpParams, 0.0f, s));
    if (n_rays == 0) return SNERG_OK;
    BackwardArgs a;
    std::memset(&a, 0, sizeof a);
    a.grid = grid_args(grid);
    a.opts = render_opts(opts);
    a.mlp = mlp;
    a.cams = h->d_cams;
    a.n_cams = n_cams;
    a.mlp_mode = mlp_mode;
    a.ray_ids = ray_ids;
    a.n_rays = n_rays;
    a.aux = aux;
    a.grad_rgba = grad_rgba;
    a.g_mlp_partial = h->d_partial;
    a.gcv = h->d_gcv;
    a.grad_dens = grad_dens;
    a.grad_rgb = grad_rgb;
    a.grad_feat = grad_feat;
    a.total_tiles = total_tiles;
    a.tile_w = h->tuning.tile_w;
    a.tile_h = h->tuning.tile_h;
    a.mlp_only = mlp_only ? 1 : 0;
    a.patch_rays = (opts->flags & SNERG_FLAG_PATCH_RAYS) ? 1 : 0;
    a.grad_packed = packed ? 1 : 0;
    if (ray_ids && !mlp_only && n_rays <= kBackwardListMaxRays && backward_aggregates(a.grid)) {
        rc = ensure_buffer(&h->d_list, &h->list_cap, size_t(n_rays) * kBackwardListCap * 4, s);
        if (rc) return rc;
        rc = ensure_buffer(&h->d_list_meta, &h->list_meta_cap, size_t(n_rays) * 4, s);
        if (rc) return rc;
        a.list = reinterpret_cast<int4*>(h->d_list);
        a.list_klast = reinterpret_cast<int64_t*>(h->d_list_meta);  // [n] int64, then [n] int32
        a.list_count = reinterpret_cast<int32_t*>(h->d_list_meta + 2 * size_t(n_rays));
    }
    HIP_TRY(launch_backward(a, n_groups, s));
    if (mlp_mode != kMlpOff) HIP_TRY(launch_reduce_mlp(h->d_partial, rows, grad_mlp, s));
    return SNERG_OK;
}

int snerg_loss_mse(snerg_handle* h, const float* rgba, const float* target, const int64_t* target_ids, int64_t n,
                   float* grad_rgba, float* loss, void* stream) {
    if (n < 0) return fail(SNERG_ERR_INVALID_ARG, "n must be >= 0");
    if (!loss) return fail(SNERG_ERR_INVALID_ARG, "loss is NULL");
    if (n > 0 && (!rgba || !target || !grad_rgba)) return fail(SNERG_ERR_INVALID_ARG, "rgba/target/grad_rgba is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(launch_mse(rgba, target, target_ids, n, grad_rgba, loss, s));
    return SNERG_OK;
}

int snerg_adam_step(snerg_handle* h, float* param, const float* grad, float* m, float* v, int64_t n,
                    const snerg_adam* cfg, void* stream) {
    if (n < 0) return fail(SNERG_ERR_INVALID_ARG, "n must be >= 0");
    if (!cfg) return fail(SNERG_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->step < 1) return fail(SNERG_ERR_INVALID_ARG, "cfg->step must be >= 1");
    if (!std::isfinite(cfg->lr) || !std::isfinite(cfg->eps) || cfg->eps <= 0.0f)
        return fail(SNERG_ERR_INVALID_ARG, "cfg->lr must be finite and cfg->eps > 0");
    if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f))
        return fail(SNERG_ERR_INVALID_ARG, "cfg->beta1/beta2 must lie in [0, 1)");
    if (n > 0 && (!param || !grad || !m || !v)) return fail(SNERG_ERR_INVALID_ARG, "param/grad/m/v is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    const float c1 = float(1.0 - std::pow(double(cfg->beta1), double(cfg->step)));
    const float c2 = float(1.0 - std::pow(double(cfg->beta2), double(cfg->step)));
    HIP_TRY(launch_adam(param, grad, m, v, n, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2,
                        static_cast<hipStream_t>(stream)));
    return SNERG_OK;
}

namespace {

int check_bake(int32_t N, int32_t B, const snerg_bake_opts* o) {
    if (!o) return fail(SNERG_ERR_INVALID_ARG, "opts is NULL");
    int rc = check_shape(N, B, 0, SNERG_U8);
    if (rc) return rc;
    if (!(o->tau_alpha >= 0.0f && o->tau_alpha < 1.0f)) return fail(SNERG_ERR_INVALID_ARG, "tau_alpha must lie in [0, 1)");
    if (!(o->tau_vis > 0.0f && o->tau_vis <= 1.0f)) return fail(SNERG_ERR_INVALID_ARG, "tau_vis must lie in (0, 1]");
    if (!std::isfinite(o->sigma_scale) || o->sigma_scale <= 0.0f)
        return fail(SNERG_ERR_INVALID_ARG, "sigma_scale must be finite and > 0");
    return SNERG_OK;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Handle-owned baking scratch for G3 macroblocks (grown on demand): the
// per-block largest density (float), visibility words (uint64), the
// kept-block count and the atlas-id map (int32).
struct BakeScratch {
    float* bmax;
    uint64_t* depth_bits;
    int32_t* count;
    int32_t* lin_of;
};

int bake_scratch(snerg_handle* h, int64_t G3, BakeScratch* out) {
    const size_t off_depth = (size_t(G3) + 1) & ~size_t(1);  // in 4-byte words, 8-byte aligned
    const size_t off_count = off_depth + 2 * size_t(G3);
    const size_t off_map = off_count + 2;
    const size_t need = off_map + size_t(G3);
    if (need > h->bake_cap) {
        HIP_TRY(hipDeviceSynchronize());
        if (h->d_bake) HIP_TRY(hipFree(h->d_bake));
        h->d_bake = nullptr;
        h->bake_cap = 0;
        HIP_TRY(hipMalloc(&h->d_bake, need * sizeof(float)));
        h->bake_cap = need;
    }
    out->bmax = h->d_bake;
    out->depth_bits = reinterpret_cast<uint64_t*>(h->d_bake + off_depth);
    out->count = reinterpret_cast<int32_t*>(h->d_bake + off_count);
    out->lin_of = reinterpret_cast<int32_t*>(h->d_bake + off_map);
    return SNERG_OK;
}

}  // namespace

int snerg_bake_cull(snerg_handle* h, int32_t N, int32_t B, const float* sigma, const snerg_camera* cams,
                    int32_t n_cams, const snerg_bake_opts* opts, float* block_alpha, float* block_vis,
                    int32_t* indirection, int32_t* n_blocks, void* stream) {
    int rc = check_bake(N, B, opts);
    if (rc) return rc;
    int64_t total = 0;
    if ((rc = check_cams(cams, n_cams, &total))) return rc;
    if (!sigma || !indirection || !n_blocks) return fail(SNERG_ERR_INVALID_ARG, "sigma/indirection/n_blocks is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t G = N / B, G3 = G * G * G;
    BakeScratch sc;
    if ((rc = bake_scratch(h, G3, &sc))) return rc;
    if (!h->h_bake_count) HIP_TRY(hipHostMalloc(&h->h_bake_count, 256, hipHostMallocDefault));
    int64_t total_tiles = 0;
    rc = upload_cams(h, cams, n_cams, h->tuning.tile_w, h->tuning.tile_h, s, &total_tiles);
    if (rc) return rc;
    BakeCullPlan p;
    p.sigma = sigma;
    p.cams = h->d_cams;
    p.n_cams = n_cams;
    p.N = N;
    p.logB = log2i(B);
    p.G = int32_t(G);
    p.total_tiles = total_tiles;
    p.tile_w = h->tuning.tile_w;
    p.tile_h = h->tuning.tile_h;
    p.vec4 = B >= 4 && aligned(sigma, 16);
    // alpha = 1 - exp(-sigma / N) >= tau_alpha  <=>  sigma >= -N log(1 - tau_alpha)
    p.sigma_thr = -double(N) * std::log1p(-double(opts->tau_alpha));
    // T = exp(-S / N) >= tau_vis  <=>  S <= -N log(tau_vis), S the density prefix sum
    p.sum_thr = -double(N) * std::log(double(opts->tau_vis));
    p.bmax = sc.bmax;
    p.depth_bits = sc.depth_bits;
    p.block_alpha = block_alpha;
    p.block_vis = block_vis;
    p.indirection = indirection;
    p.n_blocks_dev = sc.count;
    HIP_TRY(launch_bake_cull(p, s));
    HIP_TRY(hipMemcpyAsync(h->h_bake_count, p.n_blocks_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_blocks = *h->h_bake_count;
    return SNERG_OK;
}

int snerg_bake_quantize(snerg_handle* h, int32_t N, int32_t B, const float* sigma, const float* rgb, const float* feat,
                        const int32_t* indirection, int32_t n_blocks, const snerg_bake_opts* opts, uint8_t* dens8,
                        uint8_t* rgb8, uint8_t* feat8, void* stream) {
    int rc = check_bake(N, B, opts);
    if (rc) return rc;
    const int64_t G = N / B, G3 = G * G * G;
    if (n_blocks < 0 || n_blocks > G3) return fail(SNERG_ERR_INVALID_ARG, "n_blocks must lie in [0, (N/B)^3]");
    if (n_blocks > 0 && (!sigma || !rgb || !feat || !indirection || !dens8 || !rgb8 || !feat8))
        return fail(SNERG_ERR_INVALID_ARG, "an input or output pointer is NULL");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (n_blocks == 0) return SNERG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    BakeScratch sc;
    if ((rc = bake_scratch(h, G3, &sc))) return rc;
    BakeQuantPlan p;
    p.sigma = sigma;
    p.rgb = rgb;
    p.feat = feat;
    p.indirection = indirection;
    p.n_blocks = n_blocks;
    p.N = N;
    p.logB = log2i(B);
    p.G = int32_t(G);
    p.vec4 = B >= 4 && aligned(sigma, 16) && aligned(rgb, 16) && aligned(feat, 16) && aligned(dens8, 4) &&
             aligned(rgb8, 4) && aligned(feat8, 4);
    p.k_sigma = 255.0f / opts->sigma_scale;
    p.lin_of = sc.lin_of;
    p.dens8 = dens8;
    p.rgb8 = rgb8;
    p.feat8 = feat8;
    HIP_TRY(launch_bake_quantize(p, s));
    return SNERG_OK;
}

int snerg_timing_enable(snerg_handle* h, int32_t on) {
    if (on < 0) return fail(SNERG_ERR_INVALID_ARG, "on must be >= 0 (0 off, n: every n-th render)");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    if (on && h->t_start.empty()) {
        h->t_start.resize(kTimingRing, nullptr);
        h->t_stop.resize(kTimingRing, nullptr);
        for (int i = 0; i < kTimingRing; ++i) {
            HIP_TRY(hipEventCreate(&h->t_start[size_t(i)]));
            HIP_TRY(hipEventCreate(&h->t_stop[size_t(i)]));
        }
    }
    h->timing_every = on;
    h->timing_now = false;
    if (on) {
        h->t_count = 0;
        h->timing_calls = 0;
    }
    return SNERG_OK;
}

int snerg_timing_read(snerg_handle* h, float* ms, int32_t max, int32_t* n) {
    if (!n || max < 0 || (max > 0 && !ms)) return fail(SNERG_ERR_INVALID_ARG, "ms/n is NULL or max < 0");
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    const int64_t have = std::min<int64_t>(h->t_count, kTimingRing);
    const int64_t first = h->t_count - have;
    int32_t w = 0;
    for (int64_t i = first; i < h->t_count && w < max; ++i, ++w) {
        const size_t j = size_t(i % kTimingRing);
        HIP_TRY(hipEventSynchronize(h->t_stop[j]));
        HIP_TRY(hipEventElapsedTime(&ms[w], h->t_start[j], h->t_stop[j]));
    }
    *n = w;
    return SNERG_OK;
}

int snerg_set_tuning(snerg_handle* h, const snerg_tuning* t) {
    int rc = check_tuning(t);
    if (rc) return rc;
    h->tuning = *t;
    return SNERG_OK;
}

int snerg_tuning_lookup(snerg_handle* h, const snerg_grid* grid, const snerg_camera* cams, int32_t n_cams,
                        const snerg_opts* opts, snerg_tuning* t, int32_t* found) {
    if (!h || !grid || !cams || n_cams < 1 || !opts || !t || !found)
        return fail(SNERG_ERR_INVALID_ARG, "a pointer is NULL or n_cams < 1");
    auto it = h->tuned.find(tuning_signature(grid, cams, n_cams, opts));
    *found = it != h->tuned.end() ? 1 : 0;
    *t = *found ? it->second : h->tuning;
    return SNERG_OK;
}

int snerg_tuning_save(snerg_handle* h, const char* path) {
    if (!h || !path) return fail(SNERG_ERR_INVALID_ARG, "handle/path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(SNERG_ERR_INVALID_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "# snerg launch-shape cache: signature tile_w tile_h waves_per_group groups_per_cu\n");
    for (const auto& kv : h->tuned)
        std::fprintf(f, "%016llx %d %d %d %d\n", (unsigned long long)kv.first, kv.second.tile_w, kv.second.tile_h,
                     kv.second.waves_per_group, kv.second.groups_per_cu);
    const bool ok = std::fclose(f) == 0;
    return ok ? SNERG_OK : fail(SNERG_ERR_INVALID_ARG, std::string("cannot write ") + path);
}

int snerg_tuning_load(snerg_handle* h, const char* path) {
    if (!h || !path) return fail(SNERG_ERR_INVALID_ARG, "handle/path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(SNERG_ERR_INVALID_ARG, std::string("cannot read ") + path);
    std::vector<std::pair<uint64_t, snerg_tuning>> got;
    char line[256];
    int rc = SNERG_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        unsigned long long sig = 0;
        snerg_tuning t;
        if (std::sscanf(line, "%llx %d %d %d %d", &sig, &t.tile_w, &t.tile_h, &t.waves_per_group, &t.groups_per_cu) != 5) {
            rc = fail(SNERG_ERR_INVALID_ARG, std::string("malformed line in ") + path);
            break;
        }
        if ((rc = check_tuning(&t))) break;
        got.emplace_back(uint64_t(sig), t);
    }
    std::fclose(f);
    if (rc) return rc;
    for (const auto& kv : got) h->tuned[kv.first] = kv.second;
    return SNERG_OK;
}

int snerg_get_tuning(snerg_handle* h, snerg_tuning* t) {
    if (!h || !t) return fail(SNERG_ERR_INVALID_ARG, "handle/tuning is NULL");
    *t = h->tuning;
    return SNERG_OK;
}

int snerg_autotune(snerg_handle* h, const snerg_grid* grid, const float* mlp, const snerg_camera* cams,
                   int32_t n_cams, const snerg_opts* opts, const snerg_tuning* candidates, int32_t n_candidates,
                   int32_t reps, float* out_rgba, snerg_tuning* best, float* best_ms, void* stream) {
    int64_t total = 0;
    int rc = common_render_checks(grid, mlp, true, cams, n_cams, nullptr, -1, opts, &total);
    if (rc) return rc;
    if (!out_rgba) return fail(SNERG_ERR_INVALID_ARG, "out_rgba is NULL");
    if (reps < 1) return fail(SNERG_ERR_INVALID_ARG, "reps must be >= 1");
    std::vector<snerg_tuning> cand;
    if (candidates) {
        if (n_candidates < 1) return fail(SNERG_ERR_INVALID_ARG, "n_candidates must be >= 1");
        for (int i = 0; i < n_candidates; ++i) {
            if ((rc = check_tuning(&candidates[i]))) return rc;
            cand.push_back(candidates[i]);
        }
    } else {
        const int shapes[4][2] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}};
        const int wpgs[3] = {1, 2, 4};
        const int gpcs[5] = {2, 3, 4, 6, 8};
        const bool persistent = (opts->flags & SNERG_FLAG_PERSISTENT) != 0;
        for (auto& sh : shapes)
            for (int w : wpgs)
                for (int gi = 0; gi < (persistent ? 5 : 1); ++gi)
                    cand.push_back(snerg_tuning{sh[0], sh[1], w, persistent ? gpcs[gi] : 8});
    }
    if (!h) return fail(SNERG_ERR_INVALID_ARG, "handle is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_t = 1e30f;
    snerg_tuning best_c = cand[0];
    for (const snerg_tuning& c : cand) {
        rc = render_impl(h, grid, mlp, cams, n_cams, nullptr, total, opts, out_rgba, nullptr, s, c);
        if (rc) break;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < reps && !rc; ++r)
            rc = render_impl(h, grid, mlp, cams, n_cams, nullptr, total, opts, out_rgba, nullptr, s, c);
        if (rc) break;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms /= float(reps);
        if (ms < best_t) {
            best_t = ms;
            best_c = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    h->tuning = best_c;
    h->tuned[tuning_signature(grid, cams, n_cams, opts)] = best_c;
    if (best) *best = best_c;
    if (best_ms) *best_ms = best_t;
    return render_impl(h, grid, mlp, cams, n_cams, nullptr, total, opts, out_rgba, nullptr, s, best_c);
}

}  // extern "C"
