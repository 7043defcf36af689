// Host-side checks of the march's macroblock walks (built by build(), loaded
// by tests/test_host_walk.py; no GPU involved).  The walks are
// __host__ __device__ code, so the host build runs exactly the arithmetic
// the kernels run.
//
//  * march_ray_flat (the single-loop walk with the incremental macroblock
//    stepping that the render and adjoint kernels use) must hand over the
//    same samples, in the same order and with the same cells and fractions,
//    as march_ray (the nested walk whose visits the GPU tests pin to the
//    oracle), including where on_sample stops the ray;
//  * occupied_samples_on_ray split into parts must add up to the ray's
//    samples inside occupied macroblocks, as march_ray counts them.
#include "march.h"

#include <algorithm>
#include <cstdint>
#include <vector>

using namespace snerg;

namespace {

struct HostGrid {
    GridArgs g{};
    std::vector<uint2> occ;
    std::vector<uint8_t> rec;
};

// Occupancy table from the indirection grid and a pseudo-random distance
// field per occupied block (about 40% active cells): the walks only read the
// distance bytes, so any field exercises them.
void make_grid(HostGrid& h, int N, int B, const int32_t* ind, int n_atlas, uint32_t seed) {
    GridArgs& g = h.g;
    g.N = N;
    g.B = B;
    int lb = 0;
    while ((1 << lb) < B) ++lb;
    g.logB = lb;
    g.G = N / B;
    g.Bp = B + 2;
    g.Bc = B + 1;
    const int64_t G3 = int64_t(g.G) * g.G * g.G;
    g.n_words = int32_t((G3 + 31) / 32);
    h.occ.assign(size_t(g.n_words), make_uint2(0, 0));
    int32_t nb = 0;
    for (int64_t lin = 0; lin < G3; ++lin)
        if (ind[lin] >= 0 && ind[lin] < n_atlas) {
            h.occ[size_t(lin >> 5)].x |= 1u << (lin & 31);
            ++nb;
        }
    int32_t acc = 0;
    for (auto& w : h.occ) {
        w.y = uint32_t(acc);
        acc += __builtin_popcount(w.x);
    }
    g.n_blocks = nb;
    const int64_t cells = int64_t(g.Bc) * g.Bc * g.Bc;
    g.dist_bytes = (cells + 15) & ~int64_t(15);
    g.rec_stride = g.dist_bytes + 16;
    h.rec.assign(size_t(nb) * size_t(g.rec_stride) + 16, 0);
    uint32_t x = seed * 2654435761u + 1u;
    for (int32_t r = 0; r < nb; ++r)
        for (int64_t i = 0; i < cells; ++i) {
            x = x * 1664525u + 1013904223u;
            const uint32_t v = x >> 24;
            h.rec[size_t(r) * size_t(g.rec_stride) + size_t(i)] = uint8_t(v < 102 ? 0 : 1 + (v & 7));
        }
    g.rec = h.rec.data();
}

DevCamera make_camera(const double* cam, int W, int H) {
    DevCamera c{};
    for (int a = 0; a < 3; ++a) {
        c.eye[a] = cam[a];
        c.fwd[a] = cam[3 + a];
        c.right[a] = cam[6 + a];
        c.up[a] = cam[9 + a];
    }
    c.focal = cam[12];
    c.W = W;
    c.H = H;
    return c;
}

struct Visit {
    int64_t k;
    int32_t r, p0, p1, p2, f0, f1, f2;
    bool operator==(const Visit& o) const {
        return k == o.k && r == o.r && p0 == o.p0 && p1 == o.p1 && p2 == o.p2 && f0 == o.f0 && f1 == o.f1 && f2 == o.f2;
    }
};

}  // namespace

// Rays of the camera whose flat walk differs from march_ray; n_samples gets
// the number of samples march_ray handed over (a coverage figure).
extern "C" int64_t walk_flat_vs_nested(int N, int B, const int32_t* ind, int n_atlas, const double* cam, int W,
                                       int H, uint32_t seed, int64_t* n_samples) {
    HostGrid h;
    make_grid(h, N, B, ind, n_atlas, seed);
    const DevCamera c = make_camera(cam, W, H);
    int64_t bad = 0, total = 0;
    std::vector<Visit> a, b;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int64_t o[3];
            int32_t s[3];
            float d[3];
            ray_setup(c, N, px, py, o, s, d);
            // every fifth ray stops after a few samples, as early termination does
            const int stop_at = (px * 7 + py * 13) % 5 == 0 ? 1 + (px + py) % 40 : -1;
            a.clear();
            b.clear();
            march_ray(h.g, h.occ.data(), o, s, [](int32_t, bool) {}, [](int32_t) {},
                      [&](int64_t k, int32_t r, const uint8_t*, const int32_t p[3], const int32_t f[3]) {
                          a.push_back(Visit{k, r, p[0], p[1], p[2], f[0], f[1], f[2]});
                          return int(a.size()) == stop_at;
                      });
            march_ray_flat(h.g, h.occ.data(), o, s,
                           [&](int64_t k, int32_t r, const uint8_t*, const int32_t p[3], const int32_t f[3]) {
                               b.push_back(Visit{k, r, p[0], p[1], p[2], f[0], f[1], f[2]});
                               return int(b.size()) == stop_at;
                           });
            bad += a == b ? 0 : 1;
            total += int64_t(a.size());
        }
    *n_samples = total;
    return bad;
}

// Rays whose eight-part occupied_samples_on_ray sum, or whole-ray count,
// differs from march_ray's count of samples inside occupied macroblocks.
extern "C" int64_t walk_cost_parts(int N, int B, const int32_t* ind, int n_atlas, const double* cam, int W, int H,
                                   int64_t* n_samples) {
    HostGrid h;
    make_grid(h, N, B, ind, n_atlas, 1u);
    // every cell inactive at distance 1: march_ray steps through each sample
    std::fill(h.rec.begin(), h.rec.end(), uint8_t(1));
    const DevCamera c = make_camera(cam, W, H);
    int64_t bad = 0, total = 0;
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            int64_t o[3];
            int32_t s[3];
            float d[3];
            ray_setup(c, N, px, py, o, s, d);
            int32_t in_blocks = 0;
            march_ray(h.g, h.occ.data(), o, s, [](int32_t, bool) {}, [&](int32_t n) { in_blocks += n; },
                      [](int64_t, int32_t, const uint8_t*, const int32_t*, const int32_t*) { return false; });
            int32_t parts = 0;
            for (int p = 0; p < 8; ++p) parts += occupied_samples_on_ray(h.g, h.occ.data(), o, s, p, 8);
            const int32_t whole = occupied_samples_on_ray(h.g, h.occ.data(), o, s, 0, 1);
            bad += (parts != in_blocks || whole != in_blocks) ? 1 : 0;
            total += in_blocks;
        }
    *n_samples = total;
    return bad;
}
