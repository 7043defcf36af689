/*
 * Seeded synthetic SNeRG inputs: a procedural density shell and uniform
 * random colour / feature bytes, laid out as the block-sparse grid of the
 * paper's Section 5.1 (indirection grid over an atlas of B^3 macroblocks).
 *
 * This file generates inputs only.  It contains none of the rendering
 * arithmetic (no ray generation, sampling, interpolation, compositing or
 * MLP); both the FP64 oracle and the GPU library consume what it writes.
 *
 * Shell: the surface radius along unit direction u is
 *     r(u) = r0 + A * sum_{o=0..2} 0.5^o * noise_o(f0 * 2^o * u)
 * where noise_o is lattice value noise in [-1, 1] (hashed lattice values,
 * smoothstep-weighted trilinear blend).  For the voxel centred at world
 * point x (voxel i covers [i, i+1) voxel units, centre at i + 1/2, world
 * box [-1, 1]^3, voxel width v = 2/N) the signed distance in voxels is
 * s = (|x| - r(x/|x|)) / v and the density byte is
 *     max(1, floor(255 * (1 - |s|/3) + 0.5))   if |s| < 3,  else 0
 * (a tent three voxels wide on each side, mimicking the thin opaque
 * shells the paper's sparsity loss produces, Section 4.3).
 *
 * Random numbers: SplitMix64's output function (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied
 * to a counter built from the seed and the lattice/voxel coordinates, so
 * every value is independent of evaluation order and thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix_out(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t hash4(uint64_t seed, uint64_t tag, int64_t a, int64_t b, int64_t c)
{
    uint64_t h = splitmix_out(seed ^ (tag << 56));
    h = splitmix_out(h ^ (uint64_t)a);
    h = splitmix_out(h ^ (uint64_t)b);
    h = splitmix_out(h ^ (uint64_t)c);
    return h;
}

typedef struct {
    int64_t lo;   /* lattice index of table entry 0 on each axis */
    int64_t n;    /* entries per axis */
    double *val;  /* n^3 values in [-1, 1], x fastest */
} noise_table;

#define N_OCT 3

typedef struct {
    int32_t N, B;
    double r0, A, f0;
    uint64_t seed;
    noise_table oct[N_OCT];
} shell_params;

static int tables_init(shell_params *p)
{
    for (int o = 0; o < N_OCT; ++o) {
        double F = p->f0 * (double)(1 << o);
        int64_t lo = (int64_t)floor(-F) - 1;
        int64_t hi = (int64_t)ceil(F) + 2;
        int64_t n = hi - lo + 1;
        double *v = (double *)malloc(sizeof(double) * (size_t)(n * n * n));
        if (!v) return -1;
        for (int64_t z = 0; z < n; ++z)
            for (int64_t y = 0; y < n; ++y)
                for (int64_t x = 0; x < n; ++x) {
                    uint64_t h = hash4(p->seed, 1 + (uint64_t)o, x + lo, y + lo, z + lo);
                    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
                    v[(z * n + y) * n + x] = 2.0 * u - 1.0;
                }
        p->oct[o].lo = lo;
        p->oct[o].n = n;
        p->oct[o].val = v;
    }
    return 0;
}

static void tables_free(shell_params *p)
{
    for (int o = 0; o < N_OCT; ++o) free(p->oct[o].val);
}

static inline double smooth(double t) { return t * t * (3.0 - 2.0 * t); }

static double value_noise(const noise_table *t, double px, double py, double pz)
{
    double fx = floor(px), fy = floor(py), fz = floor(pz);
    int64_t ix = (int64_t)fx - t->lo, iy = (int64_t)fy - t->lo, iz = (int64_t)fz - t->lo;
    double sx = smooth(px - fx), sy = smooth(py - fy), sz = smooth(pz - fz);
    const int64_t n = t->n;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double w = (cx ? sx : 1.0 - sx) * (cy ? sy : 1.0 - sy) * (cz ? sz : 1.0 - sz);
        acc += w * t->val[((iz + cz) * n + (iy + cy)) * n + (ix + cx)];
    }
    return acc;
}

/* Density byte of voxel (gx, gy, gz) of the N^3 grid. */
static uint8_t shell_byte(const shell_params *p, int64_t gx, int64_t gy, int64_t gz)
{
    const double v = 2.0 / (double)p->N;
    double x = ((double)gx + 0.5) * v - 1.0;
    double y = ((double)gy + 0.5) * v - 1.0;
    double z = ((double)gz + 0.5) * v - 1.0;
    double len = sqrt(x * x + y * y + z * z);
    double amp = p->A * 1.75;
    if (len <= 1e-12) return 0;
    if (len < p->r0 - amp - 3.0 * v || len > p->r0 + amp + 3.0 * v) return 0;
    double ux = x / len, uy = y / len, uz = z / len;
    double r = p->r0;
    double wgt = 1.0;
    for (int o = 0; o < N_OCT; ++o) {
        double F = p->f0 * (double)(1 << o);
        r += p->A * wgt * value_noise(&p->oct[o], F * ux, F * uy, F * uz);
        wgt *= 0.5;
    }
    double s = fabs((len - r) / v);
    if (s >= 3.0) return 0;
    double b = floor(255.0 * (1.0 - s / 3.0) + 0.5);
    if (b < 1.0) b = 1.0;
    return (uint8_t)b;
}

/* Smallest and largest distance from the origin over the voxel centres of a block. */
static void block_radius_range(const shell_params *p, int64_t bx, int64_t by, int64_t bz,
                               double *rmin, double *rmax)
{
    const double v = 2.0 / (double)p->N;
    const int64_t B = p->B;
    double lo[3], hi[3];
    int64_t b[3] = {bx, by, bz};
    double mn2 = 0.0, mx2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        lo[a] = ((double)(b[a] * B) + 0.5) * v - 1.0;
        hi[a] = ((double)(b[a] * B + B - 1) + 0.5) * v - 1.0;
        double near = (lo[a] > 0.0) ? lo[a] : ((hi[a] < 0.0) ? hi[a] : 0.0);
        double far = (fabs(lo[a]) > fabs(hi[a])) ? lo[a] : hi[a];
        mn2 += near * near;
        mx2 += far * far;
    }
    *rmin = sqrt(mn2);
    *rmax = sqrt(mx2);
}

static int block_has_shell(const shell_params *p, int64_t bx, int64_t by, int64_t bz)
{
    const double v = 2.0 / (double)p->N;
    double rmin, rmax;
    block_radius_range(p, bx, by, bz, &rmin, &rmax);
    double amp = p->A * 1.75;
    if (rmax < p->r0 - amp - 3.0 * v || rmin > p->r0 + amp + 3.0 * v) return 0;
    const int64_t B = p->B;
    for (int64_t z = 0; z < B; ++z)
        for (int64_t y = 0; y < B; ++y)
            for (int64_t x = 0; x < B; ++x)
                if (shell_byte(p, bx * B + x, by * B + y, bz * B + z)) return 1;
    return 0;
}

/*
 * Marks occupied macroblocks of the shell: occ[(bz*G + by)*G + bx] = 1 when
 * any voxel of the block has a non-zero density byte.  Returns the number
 * of occupied blocks, or -1 on allocation failure.
 */
int64_t shellgen_occupancy(int32_t N, int32_t B, double r0, double A, double f0, uint64_t seed,
                           uint8_t *occ)
{
    shell_params p;
    memset(&p, 0, sizeof p);
    p.N = N; p.B = B; p.r0 = r0; p.A = A; p.f0 = f0; p.seed = seed;
    if (tables_init(&p)) return -1;
    const int64_t G = N / B;
    int64_t count = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : count)
    for (int64_t blk = 0; blk < G * G * G; ++blk) {
        int64_t bx = blk % G, by = (blk / G) % G, bz = blk / (G * G);
        uint8_t o = (uint8_t)block_has_shell(&p, bx, by, bz);
        occ[blk] = o;
        count += o;
    }
    tables_free(&p);
    return count;
}

/*
 * Fills the atlas for the occupied blocks named by `indirection`
 * ((N/B)^3 int32, x fastest, -1 empty, else atlas block id):
 *   dens [n_blocks][B][B][B]     shell density bytes
 *   rgb  [n_blocks][B][B][B][3]  uniform random bytes
 *   feat [n_blocks][B][B][B][4]  uniform random bytes
 * Colour and feature bytes are keyed by global voxel coordinates and
 * `color_seed`.
 */
int shellgen_fill(int32_t N, int32_t B, double r0, double A, double f0, uint64_t seed,
                  uint64_t color_seed, const int32_t *indirection, int32_t n_blocks,
                  uint8_t *dens, uint8_t *rgb, uint8_t *feat)
{
    shell_params p;
    memset(&p, 0, sizeof p);
    p.N = N; p.B = B; p.r0 = r0; p.A = A; p.f0 = f0; p.seed = seed;
    if (tables_init(&p)) return -1;
    const int64_t G = N / B;
    const int64_t B3 = (int64_t)B * B * B;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t blk = 0; blk < G * G * G; ++blk) {
        int32_t id = indirection[blk];
        if (id < 0) continue;
        if (id >= n_blocks) {
#pragma omp atomic write
            err = -2;
            continue;
        }
        int64_t bx = blk % G, by = (blk / G) % G, bz = blk / (G * G);
        for (int64_t z = 0; z < B; ++z)
            for (int64_t y = 0; y < B; ++y)
                for (int64_t x = 0; x < B; ++x) {
                    int64_t gx = bx * B + x, gy = by * B + y, gz = bz * B + z;
                    int64_t li = (z * B + y) * B + x;
                    int64_t vi = (int64_t)id * B3 + li;
                    dens[vi] = shell_byte(&p, gx, gy, gz);
                    uint64_t h = hash4(color_seed, 9, gx, gy, gz);
                    for (int c = 0; c < 3; ++c) rgb[vi * 3 + c] = (uint8_t)(h >> (8 * c));
                    for (int c = 0; c < 4; ++c) feat[vi * 4 + c] = (uint8_t)(h >> (8 * (c + 3)));
                }
    }
    tables_free(&p);
    return err;
}

/*
 * Dense synthetic radiance field for the baking workload (the input of the
 * paper's Section 5.3, which evaluates NeRF densely on the N^3 grid): float
 * density, colour and features for every voxel, x fastest.
 *   sigma = sigma_max * max(0, 1 - |s|/3)      around the shell surface
 *         + sigma_max / 4 inside each of n_blobs balls of radius blob_r whose
 *           centres lie at radius < 0.3 (occluded by the shell)
 *         + haze                                everywhere
 *   rgb, feat = the colour/feature bytes of shellgen_fill / 255.
 */
int shellgen_dense(int32_t N, double r0, double A, double f0, uint64_t seed, uint64_t color_seed,
                   double sigma_max, double haze, int32_t n_blobs, double blob_r, float *sigma, float *rgb,
                   float *feat)
{
    shell_params p;
    memset(&p, 0, sizeof p);
    p.N = N; p.B = 1; p.r0 = r0; p.A = A; p.f0 = f0; p.seed = seed;
    if (tables_init(&p)) return -1;
    double cx[64], cy[64], cz[64];
    if (n_blobs > 64) n_blobs = 64;
    for (int b = 0; b < n_blobs; ++b) {
        uint64_t h = hash4(seed, 77, b, 0, 0);
        double u0 = (double)(h & 0xFFFFF) / 1048576.0, u1 = (double)((h >> 20) & 0xFFFFF) / 1048576.0;
        double u2 = (double)((h >> 40) & 0xFFFFF) / 1048576.0;
        double rr = 0.3 * cbrt(u2), th = acos(1.0 - 2.0 * u0), ph = 6.283185307179586 * u1;
        cx[b] = rr * sin(th) * cos(ph); cy[b] = rr * sin(th) * sin(ph); cz[b] = rr * cos(th);
    }
    const double v = 2.0 / (double)N;
    const double amp = A * 1.75;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t gz = 0; gz < N; ++gz)
        for (int64_t gy = 0; gy < N; ++gy)
            for (int64_t gx = 0; gx < N; ++gx) {
                int64_t vi = (gz * N + gy) * N + gx;
                double x = ((double)gx + 0.5) * v - 1.0, y = ((double)gy + 0.5) * v - 1.0;
                double z = ((double)gz + 0.5) * v - 1.0;
                double len = sqrt(x * x + y * y + z * z);
                double s = haze;
                if (len > 1e-12 && len >= r0 - amp - 3.0 * v && len <= r0 + amp + 3.0 * v) {
                    double ux = x / len, uy = y / len, uz = z / len, r = r0, wgt = 1.0;
                    for (int o = 0; o < N_OCT; ++o) {
                        double F = f0 * (double)(1 << o);
                        r += A * wgt * value_noise(&p.oct[o], F * ux, F * uy, F * uz);
                        wgt *= 0.5;
                    }
                    double d = fabs((len - r) / v);
                    if (d < 3.0) s += sigma_max * (1.0 - d / 3.0);
                }
                for (int b = 0; b < n_blobs; ++b) {
                    double dx = x - cx[b], dy = y - cy[b], dz = z - cz[b];
                    if (dx * dx + dy * dy + dz * dz < blob_r * blob_r) s += 0.25 * sigma_max;
                }
                sigma[vi] = (float)s;
                uint64_t h = hash4(color_seed, 9, gx, gy, gz);
                for (int c = 0; c < 3; ++c) rgb[vi * 3 + c] = (float)((h >> (8 * c)) & 0xFF) / 255.0f;
                for (int c = 0; c < 4; ++c) feat[vi * 4 + c] = (float)((h >> (8 * (c + 3))) & 0xFF) / 255.0f;
            }
    tables_free(&p);
    return 0;
}
