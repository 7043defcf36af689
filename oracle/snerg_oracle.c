/*
 * FP64 CPU oracle for the SNeRG render hot path
 * ("Baking Neural Radiance Fields for Real-Time View Synthesis",
 *  Hedman et al., arXiv 2103.14645).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * library is checked against.  Only the tests, the package smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never
 * calls it.  It shares no code with the GPU library.
 *
 * What it computes, step by step (every sample is visited; nothing is
 * skipped except where the method itself skips):
 *
 *  1. Ray generation (pinhole camera, Appendix B intrinsics).  Pixel (i, j)
 *     has x = (i + 1/2 - W/2)/f, y = (j + 1/2 - H/2)/f and direction
 *     d = D/|D| with D = fwd + x*right - y*up.  The operation order below is
 *     fixed (no contraction) so that any IEEE-754 implementation of the same
 *     basic operations produces the same bits.
 *  2. Sample lattice.  The grid covers the world box [-1, 1]^3 with N^3
 *     voxels; voxel units are u = (x + 1) * N/2.  Samples are half a voxel
 *     apart (step 1/N in world units) and indexed by an integer k >= 0 from
 *     the camera centre, in Q16 fixed point:
 *         o = rint(((eye + 1) * (N/2)) * 2^16),  s = rint(d * 2^15),
 *         P_k = o + k*s.
 *     A sample is inside the grid when 0 <= P_k < N*2^16 on every axis.
 *  3. Macroblock skip (Section 5.1, 5.2; Appendix A).  The sample's
 *     macroblock is floor(P_k / (B*2^16)) per axis; a sample whose
 *     macroblock is marked empty in the indirection grid is skipped.
 *  4. Trilinear interpolation (Section 5.2) of density, diffuse colour and
 *     features over the virtual dense grid: voxel values sit at voxel
 *     centres, a voxel outside the grid or in an empty macroblock reads 0.
 *     The sample is "active" when some corner has non-zero density and
 *     non-zero weight; an inactive sample has sigma = 0 and contributes
 *     nothing (Section 5.2 reads colour and features only where there is
 *     density).
 *  5. Front-to-back compositing (Eq. 2, 5, 6) with a constant step
 *     delta = 1/N: alpha = 1 - exp(-sigma*delta), w = T*alpha,
 *     C_d += w*c_d, V += w*v, T *= (1 - alpha); ray marching ends after the
 *     sample that brings T below t_stop (Section 5.2 ends the march when
 *     the accumulated opacity saturates).
 *  6. Deferred shading (Eq. 7, Section 4.2, Appendix A): once per pixel, if
 *     at least one sample was composited, the MLP with 2 hidden layers of 16
 *     channels maps [C_d, V, d, PE(d)] (PE: sin and cos at octaves 0..3,
 *     NeRF's positional encoding, Section 6) to a residual
 *     R = sigmoid(W3 relu(W2 relu(W1 x + b1) + b2) + b3).
 *  7. Output: rgb = C_d + T*bg + R, alpha = 1 - T.
 *
 * The gradient routine stores each ray's composited samples and runs plain
 * reverse-mode differentiation through steps 4-7.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

#define ORC_U8 0
#define ORC_F32 1
#define ORC_F64 2

#define MLP_IN 34
#define MLP_H 16
#define MLP_OUT 3
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT)

typedef struct {
    int32_t N, B;
    const int32_t *indirection; /* (N/B)^3, x fastest; -1 = empty, else atlas block id */
    int32_t n_blocks;
    int32_t dtype;              /* ORC_U8: stored byte / 255; ORC_F32 / ORC_F64: value as stored */
    const void *dens;           /* [n_blocks][B][B][B] (z, y, x) */
    const void *rgb;            /* [n_blocks][B][B][B][3] */
    const void *feat;           /* [n_blocks][B][B][B][4] */
    double sigma_scale;         /* sigma = sigma_scale * interpolated density value */
} orc_grid;

typedef struct {
    double eye[3], fwd[3], right[3], up[3];
    int32_t W, H;
    double focal;
} orc_camera;

typedef struct {
    double bg[3];
    double t_stop;
    int32_t early_stop;
    int32_t mlp_on;
    int32_t nn_gate;        /* Appendix A: skip a sample whose nearest voxel has zero density */
    int32_t unpremultiply;  /* Eq. 9: scale colour, features and alpha by min(1, 1.5a)/a */
    int32_t per_sample_mlp; /* not deferred: the view MLP's residual added to every composited sample */
} orc_opts;

/* ------------------------------------------------------------------ helpers */

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static double grid_value(const orc_grid *g, const void *base, int64_t idx)
{
    switch (g->dtype) {
    case ORC_U8: return (double)((const uint8_t *)base)[idx] / 255.0;
    case ORC_F32: return (double)((const float *)base)[idx];
    default: return ((const double *)base)[idx];
    }
}

/* Atlas voxel index of dense voxel (x, y, z), or -1 when the voxel lies
 * outside the grid or in an empty macroblock. */
static int64_t voxel_index(const orc_grid *g, int64_t x, int64_t y, int64_t z)
{
    const int64_t N = g->N, B = g->B, G = N / B;
    if (x < 0 || y < 0 || z < 0 || x >= N || y >= N || z >= N) return -1;
    int64_t bx = x / B, by = y / B, bz = z / B;
    int32_t id = g->indirection[(bz * G + by) * G + bx];
    if (id < 0) return -1;
    int64_t lx = x - bx * B, ly = y - by * B, lz = z - bz * B;
    return (int64_t)id * B * B * B + (lz * B + ly) * B + lx;
}

/* ------------------------------------------------------------- step 1: rays */

int orc_ray_setup(const orc_camera *c, int32_t N, int64_t px, int64_t py, int64_t o[3],
                  int64_t s[3], double d[3])
{
    if (!c || N <= 0 || c->focal <= 0.0) return ORC_EINVAL;
    double x = (((double)px + 0.5) - (double)c->W * 0.5) / c->focal;
    double y = (((double)py + 0.5) - (double)c->H * 0.5) / c->focal;
    double D[3];
    for (int a = 0; a < 3; ++a) {
        double t = x * c->right[a];
        t = c->fwd[a] + t;
        double u = y * c->up[a];
        D[a] = t - u;
    }
    double n2 = D[0] * D[0];
    n2 = n2 + D[1] * D[1];
    n2 = n2 + D[2] * D[2];
    double n = sqrt(n2);
    for (int a = 0; a < 3; ++a) {
        d[a] = D[a] / n;
        s[a] = (int64_t)rint(d[a] * 32768.0);
        double e = c->eye[a] + 1.0;
        e = e * (0.5 * (double)N);
        e = e * 65536.0;
        o[a] = (int64_t)rint(e);
    }
    return ORC_OK;
}

/* ---------------------------------------------------- step 4: one sample */

/*
 * Trilinear interpolation at lattice point P (Q16 voxel units).  out[0] =
 * sigma, out[1..3] = diffuse colour, out[4..7] = features.  Returns 1 when
 * the sample is active (a corner with non-zero density and non-zero weight).
 * When `corner_idx` / `corner_w` are given they receive, for the 8 corners
 * (corner c = cx + 2 cy + 4 cz), the atlas voxel index (-1: reads zero) and
 * the weight.
 */
static int sample_point(const orc_grid *g, const int64_t P[3], double out[8],
                        int64_t corner_idx[8], double corner_w[8])
{
    int64_t i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        int64_t Q = P[a] - 32768;
        i0[a] = floor_div(Q, 65536);
        f[a] = (double)(Q - i0[a] * 65536) / 65536.0;
    }
    int active = 0;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double w = (cx ? f[0] : 1.0 - f[0]) * (cy ? f[1] : 1.0 - f[1]) * (cz ? f[2] : 1.0 - f[2]);
        int64_t vi = voxel_index(g, i0[0] + cx, i0[1] + cy, i0[2] + cz);
        if (corner_idx) corner_idx[c] = vi;
        if (corner_w) corner_w[c] = w;
        if (vi < 0) continue;
        double dv = grid_value(g, g->dens, vi);
        if (dv != 0.0 && w != 0.0) active = 1;
        acc[0] += w * dv;
        for (int ch = 0; ch < 3; ++ch) acc[1 + ch] += w * grid_value(g, g->rgb, vi * 3 + ch);
        for (int ch = 0; ch < 4; ++ch) acc[4 + ch] += w * grid_value(g, g->feat, vi * 4 + ch);
    }
    out[0] = g->sigma_scale * acc[0];
    for (int ch = 1; ch < 8; ++ch) out[ch] = acc[ch];
    return active;
}

/* The WebGL renderer's in-block test (Appendix A): the density of the voxel
 * whose centre is nearest to P, i.e. voxel floor(P) in voxel units, is
 * non-zero (empty blocks and the outside read as zero). */
static int nearest_nonzero(const orc_grid *g, const int64_t P[3])
{
    int64_t vi = voxel_index(g, floor_div(P[0], 65536), floor_div(P[1], 65536), floor_div(P[2], 65536));
    return vi >= 0 && grid_value(g, g->dens, vi) != 0.0;
}

int orc_sample(const orc_grid *g, const int64_t P[3], double out[8], int32_t *active)
{
    if (!g || !P || !out) return ORC_EINVAL;
    int a = sample_point(g, P, out, NULL, NULL);
    if (active) *active = a;
    return ORC_OK;
}

/* ------------------------------------------------ step 5: compositing */

typedef struct {
    double C[3], V[4], T;
    int32_t gate;
} comp_state;

static void comp_init(comp_state *st)
{
    memset(st, 0, sizeof *st);
    st->T = 1.0;
}

/* Composites one active sample; returns the weight T*alpha it received. */
static double comp_step(comp_state *st, const double smp[8], double delta)
{
    double alpha = -expm1(-smp[0] * delta);
    double w = st->T * alpha;
    for (int ch = 0; ch < 3; ++ch) st->C[ch] += w * smp[1 + ch];
    for (int ch = 0; ch < 4; ++ch) st->V[ch] += w * smp[4 + ch];
    st->T = st->T * (1.0 - alpha);
    st->gate = 1;
    return w;
}

/*
 * Composites a given list of n samples (rows of 8: sigma, c_d[3], v[4]) with
 * step delta; stops after the sample that brings T below t_stop when
 * early_stop is set.  out: C_d[3], V[4], T.  *n_used = samples composited.
 */
int orc_composite(const double *samples, int64_t n, double delta, double t_stop, int32_t early_stop,
                  double out[8], int64_t *n_used)
{
    if ((!samples && n > 0) || !out) return ORC_EINVAL;
    comp_state st;
    comp_init(&st);
    int64_t k = 0;
    for (; k < n; ++k) {
        comp_step(&st, samples + 8 * k, delta);
        if (early_stop && st.T < t_stop) { ++k; break; }
    }
    for (int ch = 0; ch < 3; ++ch) out[ch] = st.C[ch];
    for (int ch = 0; ch < 4; ++ch) out[3 + ch] = st.V[ch];
    out[7] = st.T;
    if (n_used) *n_used = k;
    return ORC_OK;
}

/* --------------------------------------------------- step 6: deferred MLP */

static const double ORC_PI = 3.14159265358979323846;

/* x = [C_d(3), V(4), d(3), PE(d)(24)], PE octave l: sin(2^l pi d_xyz), cos(2^l pi d_xyz). */
int orc_encode(const double C[3], const double V[4], const double d[3], double x[MLP_IN])
{
    int i = 0;
    for (int a = 0; a < 3; ++a) x[i++] = C[a];
    for (int a = 0; a < 4; ++a) x[i++] = V[a];
    for (int a = 0; a < 3; ++a) x[i++] = d[a];
    for (int l = 0; l < 4; ++l) {
        double fr = (double)(1 << l) * ORC_PI;
        for (int a = 0; a < 3; ++a) x[i++] = sin(fr * d[a]);
        for (int a = 0; a < 3; ++a) x[i++] = cos(fr * d[a]);
    }
    return ORC_OK;
}

/* Parameter blocks inside the 883-float vector. */
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_OUT * MLP_H)

typedef struct {
    double x[MLP_IN], h1[MLP_H], h2[MLP_H], o[MLP_OUT], R[MLP_OUT];
} mlp_acts;

static void mlp_forward(const double *p, const double x[MLP_IN], mlp_acts *a)
{
    memcpy(a->x, x, sizeof a->x);
    for (int j = 0; j < MLP_H; ++j) {
        double s = p[OFF_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) s += p[OFF_W1 + j * MLP_IN + i] * x[i];
        a->h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = p[OFF_B2 + j];
        for (int i = 0; i < MLP_H; ++i) s += p[OFF_W2 + j * MLP_H + i] * a->h1[i];
        a->h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < MLP_OUT; ++j) {
        double s = p[OFF_B3 + j];
        for (int i = 0; i < MLP_H; ++i) s += p[OFF_W3 + j * MLP_H + i] * a->h2[i];
        a->o[j] = s;
        a->R[j] = 1.0 / (1.0 + exp(-s));
    }
}

int orc_mlp(const double *params, const double x[MLP_IN], double R[MLP_OUT])
{
    if (!params || !x || !R) return ORC_EINVAL;
    mlp_acts a;
    mlp_forward(params, x, &a);
    for (int j = 0; j < MLP_OUT; ++j) R[j] = a.R[j];
    return ORC_OK;
}

/* -------------------------------------------------------- one whole ray */

typedef struct {
    int64_t P[3];
    double smp[8];   /* sigma, c_d, v */
    double T_before; /* transmittance before this sample */
} rec_sample;

typedef struct {
    rec_sample *v;
    int64_t n, cap;
} rec_list;

static int rec_push(rec_list *l, const int64_t P[3], const double smp[8], double T_before)
{
    if (l->n == l->cap) {
        int64_t cap = l->cap ? 2 * l->cap : 64;
        rec_sample *nv = (rec_sample *)realloc(l->v, sizeof(rec_sample) * (size_t)cap);
        if (!nv) return ORC_ENOMEM;
        l->v = nv;
        l->cap = cap;
    }
    rec_sample *r = &l->v[l->n++];
    memcpy(r->P, P, sizeof r->P);
    memcpy(r->smp, smp, sizeof r->smp);
    r->T_before = T_before;
    return ORC_OK;
}

typedef struct {
    int32_t blocks_traversed; /* distinct macroblocks holding an inside sample */
    int32_t blocks_occupied;  /* of which occupied */
    int32_t inblock_samples;  /* samples inside occupied macroblocks */
    int32_t active_samples;   /* samples composited */
    int32_t term_k;           /* k of the sample that stopped the ray, -1 if none */
    uint32_t k_sum;           /* sum of the composited samples' k, modulo 2^32 */
    uint32_t k_sq_sum;        /* sum of their k^2, modulo 2^32 */
} ray_counters;

typedef struct {
    double rgba[4];
    double aux[9];  /* C_d[3], V[4], T, gate */
    ray_counters cnt;
    double d[3];
} ray_result;

/*
 * Marches one ray through every lattice index k from the camera centre
 * until the ray has left the grid.  Appends visited occupied macroblocks
 * (linear index into the indirection grid, consecutive repeats collapsed)
 * to `visits` (up to max_visits; *n_visits counts them all) and composited
 * samples to `rec` when given.
 */
static int march_ray(const orc_grid *g, const double *mlp, const orc_camera *cam, int64_t px,
                     int64_t py, const orc_opts *op, ray_result *res, int32_t *visits,
                     int32_t max_visits, int32_t *n_visits, rec_list *rec)
{
    const int64_t N = g->N, B = g->B, G = N / B;
    const int64_t L = N * 65536;
    const double delta = 1.0 / (double)N;
    int64_t o[3], s[3];
    double d[3];
    orc_ray_setup(cam, (int32_t)N, px, py, o, s, d);

    /* Largest k at which the ray can still be inside: along the axis of
     * largest |s| every step moves at least smax. */
    int64_t smax = 0, omax = 0;
    for (int a = 0; a < 3; ++a) {
        if (llabs(s[a]) > smax) smax = llabs(s[a]);
        if (llabs(o[a]) > omax) omax = llabs(o[a]);
    }
    int64_t k_limit = (smax > 0) ? (omax + L) / smax + 2 : 0;

    comp_state st;
    comp_init(&st);
    ray_counters cnt = {0, 0, 0, 0, -1, 0u, 0u};
    int64_t prev_blk = -1, prev_vis = -1;
    int seen_inside = 0;
    int32_t nv = 0;

    for (int64_t k = 0; k <= k_limit; ++k) {
        int64_t P[3];
        int inside = 1;
        for (int a = 0; a < 3; ++a) {
            P[a] = o[a] + k * s[a];
            if (P[a] < 0 || P[a] >= L) inside = 0;
        }
        if (!inside) {
            if (seen_inside) break;
            continue;
        }
        seen_inside = 1;
        int64_t bx = P[0] / (B * 65536), by = P[1] / (B * 65536), bz = P[2] / (B * 65536);
        int64_t blk = (bz * G + by) * G + bx;
        if (blk != prev_blk) {
            cnt.blocks_traversed++;
            prev_blk = blk;
        }
        if (g->indirection[blk] < 0) continue;
        if (blk != prev_vis) {
            if (visits && nv < max_visits) visits[nv] = (int32_t)blk;
            nv++;
            cnt.blocks_occupied++;
            prev_vis = blk;
        }
        cnt.inblock_samples++;
        if (op->nn_gate && !nearest_nonzero(g, P)) continue;
        double smp[8];
        if (!sample_point(g, P, smp, NULL, NULL)) continue;
        cnt.active_samples++;
        cnt.k_sum += (uint32_t)k;
        cnt.k_sq_sum += (uint32_t)k * (uint32_t)k;
        if (op->per_sample_mlp && op->mlp_on && mlp) {
            /* the network of Eq. 7 on this sample's own colour and features
             * (as NeRF queries its MLP at every sample), its residual added
             * to the sample's colour before compositing */
            double x[MLP_IN], Rk[3];
            orc_encode(&smp[1], &smp[4], d, x);
            orc_mlp(mlp, x, Rk);
            for (int ch = 0; ch < 3; ++ch) smp[1 + ch] += Rk[ch];
        }
        if (rec && rec_push(rec, P, smp, st.T)) return ORC_ENOMEM;
        comp_step(&st, smp, delta);
        if (op->early_stop && st.T < op->t_stop) {
            cnt.term_k = (int32_t)k;
            break;
        }
    }
    if (n_visits) *n_visits = nv;
    if (op->unpremultiply) {
        /* Eq. 9, after compositing and before the deferred network */
        double alpha = 1.0 - st.T;
        if (alpha > 0.0) {
            double sc = (1.5 * alpha < 1.0 ? 1.5 * alpha : 1.0) / alpha;
            for (int ch = 0; ch < 3; ++ch) st.C[ch] *= sc;
            for (int ch = 0; ch < 4; ++ch) st.V[ch] *= sc;
            st.T = 1.0 - alpha * sc;
        }
    }

    double R[3] = {0.0, 0.0, 0.0};
    if (st.gate && op->mlp_on && mlp && !op->per_sample_mlp) {
        double x[MLP_IN];
        orc_encode(st.C, st.V, d, x);
        orc_mlp(mlp, x, R);
    }
    for (int ch = 0; ch < 3; ++ch) res->rgba[ch] = st.C[ch] + st.T * op->bg[ch] + R[ch];
    res->rgba[3] = 1.0 - st.T;
    for (int ch = 0; ch < 3; ++ch) res->aux[ch] = st.C[ch];
    for (int ch = 0; ch < 4; ++ch) res->aux[3 + ch] = st.V[ch];
    res->aux[7] = st.T;
    res->aux[8] = (double)st.gate;
    res->cnt = cnt;
    memcpy(res->d, d, sizeof res->d);
    return ORC_OK;
}

/* ------------------------------------------------------- ray addressing */

static int check_grid(const orc_grid *g)
{
    if (!g || !g->indirection || !g->dens || !g->rgb || !g->feat) return ORC_EINVAL;
    if (g->N <= 0 || g->B <= 0 || g->N % g->B != 0) return ORC_EINVAL;
    if (g->dtype < ORC_U8 || g->dtype > ORC_F64) return ORC_EINVAL;
    return ORC_OK;
}

/* Camera index and pixel of global ray id r (cameras in order, rows from the
 * top, columns left to right). */
static int locate_ray(const orc_camera *cams, int32_t n_cams, int64_t r, int32_t *ci, int64_t *px,
                      int64_t *py)
{
    if (r < 0) return ORC_EINVAL;
    for (int32_t c = 0; c < n_cams; ++c) {
        int64_t n = (int64_t)cams[c].W * cams[c].H;
        if (r < n) {
            *ci = c;
            *py = r / cams[c].W;
            *px = r % cams[c].W;
            return ORC_OK;
        }
        r -= n;
    }
    return ORC_EINVAL;
}

static int set_threads(int32_t n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
    return omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

/*
 * Renders rays ray_ids[0..n_rays) (all rays of all cameras when ray_ids is
 * NULL; then n_rays must equal their total).  rgba [n][4]; aux (nullable)
 * [n][9] = C_d, V, T, gate; counters (nullable) [n][7] = macroblocks
 * traversed, occupied macroblocks visited, samples inside occupied
 * macroblocks, composited samples, stopping k (-1 if none), and the sums of
 * the composited samples' k and k^2 modulo 2^32 (stored as int32 bits),
 * which name the set of composited samples, not just its size.
 */
int orc_render(const orc_grid *g, const double *mlp, const orc_camera *cams, int32_t n_cams,
               const int64_t *ray_ids, int64_t n_rays, const orc_opts *op, double *rgba, double *aux,
               int32_t *counters, int32_t n_threads)
{
    if (check_grid(g) || !cams || n_cams <= 0 || !op || !rgba || n_rays < 0) return ORC_EINVAL;
    set_threads(n_threads);
    int err = ORC_OK;
#pragma omp parallel for schedule(static, 64)
    for (int64_t i = 0; i < n_rays; ++i) {
        int64_t r = ray_ids ? ray_ids[i] : i;
        int32_t ci;
        int64_t px, py;
        if (locate_ray(cams, n_cams, r, &ci, &px, &py)) {
#pragma omp atomic write
            err = ORC_EINVAL;
            continue;
        }
        ray_result res;
        if (march_ray(g, mlp, &cams[ci], px, py, op, &res, NULL, 0, NULL, NULL)) {
#pragma omp atomic write
            err = ORC_ENOMEM;
            continue;
        }
        memcpy(rgba + 4 * i, res.rgba, sizeof res.rgba);
        if (aux) memcpy(aux + 9 * i, res.aux, sizeof res.aux);
        if (counters) {
            int32_t *c = counters + 7 * i;
            c[0] = res.cnt.blocks_traversed;
            c[1] = res.cnt.blocks_occupied;
            c[2] = res.cnt.inblock_samples;
            c[3] = res.cnt.active_samples;
            c[4] = res.cnt.term_k;
            c[5] = (int32_t)res.cnt.k_sum;
            c[6] = (int32_t)res.cnt.k_sq_sum;
        }
    }
    return err;
}

/* Occupied macroblocks visited by each ray, in order: visits [n][max_visits]
 * (linear indirection-grid index), counts [n] (may exceed max_visits). */
int orc_trace_visits(const orc_grid *g, const orc_camera *cams, int32_t n_cams,
                     const int64_t *ray_ids, int64_t n_rays, const orc_opts *op, int32_t max_visits,
                     int32_t *visits, int32_t *counts, int32_t n_threads)
{
    if (check_grid(g) || !cams || n_cams <= 0 || !op || !counts || max_visits < 0) return ORC_EINVAL;
    if (max_visits > 0 && !visits) return ORC_EINVAL;
    set_threads(n_threads);
    int err = ORC_OK;
#pragma omp parallel for schedule(static, 64)
    for (int64_t i = 0; i < n_rays; ++i) {
        int64_t r = ray_ids ? ray_ids[i] : i;
        int32_t ci;
        int64_t px, py;
        if (locate_ray(cams, n_cams, r, &ci, &px, &py)) {
#pragma omp atomic write
            err = ORC_EINVAL;
            continue;
        }
        ray_result res;
        orc_opts o2 = *op;
        o2.mlp_on = 0;
        march_ray(g, NULL, &cams[ci], px, py, &o2, &res, visits ? visits + (int64_t)max_visits * i : NULL,
                  max_visits, &counts[i], NULL);
    }
    return err;
}

/* ------------------------------------------------------------ gradients */

/*
 * Gradient of L = sum_r g_rgba[r] . rgba[r] with respect to the MLP
 * parameters (883, same order as the parameter vector) and the grid values
 * (shapes of dens / rgb / feat; ORC_F32 or ORC_F64 grids only), accumulated
 * into the zero-initialised outputs.  The set of composited samples and the
 * stopping sample are held fixed (the render is piecewise smooth in them).
 * Plain reverse-mode: each ray's composited samples are stored during the
 * forward march, then the MLP, the compositing recurrence and the
 * trilinear weights are differentiated in reverse order.  Single threaded.
 * With g_cv (nullable, [n][7]) the MLP is not differentiated: its rows give
 * each ray's dL/dC_d (3) and dL/dV (4) directly (to check a reduced
 * precision MLP backward against this FP64 march backward).
 */
int orc_render_grad(const orc_grid *g, const double *mlp, const orc_camera *cams, int32_t n_cams,
                    const int64_t *ray_ids, int64_t n_rays, const orc_opts *op,
                    const double *g_rgba, double *g_mlp, double *g_dens, double *g_rgb,
                    double *g_feat, const double *g_cv)
{
    if (check_grid(g) || g->dtype == ORC_U8 || !cams || n_cams <= 0 || !op || !g_rgba) return ORC_EINVAL;
    if (!g_mlp || !g_dens || !g_rgb || !g_feat || (!mlp && op->mlp_on)) return ORC_EINVAL;
    if (op->unpremultiply || op->per_sample_mlp) return ORC_EINVAL; /* forward-only variants */
    const double delta = 1.0 / (double)g->N;
    rec_list rec = {NULL, 0, 0};
    for (int64_t i = 0; i < n_rays; ++i) {
        int64_t r = ray_ids ? ray_ids[i] : i;
        int32_t ci;
        int64_t px, py;
        if (locate_ray(cams, n_cams, r, &ci, &px, &py)) {
            free(rec.v);
            return ORC_EINVAL;
        }
        rec.n = 0;
        ray_result res;
        if (march_ray(g, mlp, &cams[ci], px, py, op, &res, NULL, 0, NULL, &rec)) {
            free(rec.v);
            return ORC_ENOMEM;
        }
        const double *gr = g_rgba + 4 * i;
        double gC[3], gV[4] = {0, 0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) gC[ch] = gr[ch];
        /* rgb = C + T bg + R, alpha = 1 - T */
        double gT = gr[0] * op->bg[0] + gr[1] * op->bg[1] + gr[2] * op->bg[2] - gr[3];

        if (g_cv) {
            for (int ch = 0; ch < 3; ++ch) gC[ch] = g_cv[7 * i + ch];
            for (int ch = 0; ch < 4; ++ch) gV[ch] = g_cv[7 * i + 3 + ch];
        } else if (res.aux[8] != 0.0 && op->mlp_on && mlp) {
            double x[MLP_IN];
            orc_encode(res.aux, res.aux + 3, res.d, x);
            mlp_acts a;
            mlp_forward(mlp, x, &a);
            double go[MLP_OUT], gh2[MLP_H], gh1[MLP_H];
            for (int j = 0; j < MLP_OUT; ++j) go[j] = gr[j] * a.R[j] * (1.0 - a.R[j]);
            for (int i2 = 0; i2 < MLP_H; ++i2) gh2[i2] = 0.0;
            for (int j = 0; j < MLP_OUT; ++j) {
                g_mlp[OFF_B3 + j] += go[j];
                for (int i2 = 0; i2 < MLP_H; ++i2) {
                    g_mlp[OFF_W3 + j * MLP_H + i2] += go[j] * a.h2[i2];
                    gh2[i2] += mlp[OFF_W3 + j * MLP_H + i2] * go[j];
                }
            }
            for (int i2 = 0; i2 < MLP_H; ++i2) gh2[i2] = (a.h2[i2] > 0.0) ? gh2[i2] : 0.0;
            for (int i2 = 0; i2 < MLP_H; ++i2) gh1[i2] = 0.0;
            for (int j = 0; j < MLP_H; ++j) {
                g_mlp[OFF_B2 + j] += gh2[j];
                for (int i2 = 0; i2 < MLP_H; ++i2) {
                    g_mlp[OFF_W2 + j * MLP_H + i2] += gh2[j] * a.h1[i2];
                    gh1[i2] += mlp[OFF_W2 + j * MLP_H + i2] * gh2[j];
                }
            }
            for (int i2 = 0; i2 < MLP_H; ++i2) gh1[i2] = (a.h1[i2] > 0.0) ? gh1[i2] : 0.0;
            double gx[MLP_IN];
            for (int i2 = 0; i2 < MLP_IN; ++i2) gx[i2] = 0.0;
            for (int j = 0; j < MLP_H; ++j) {
                g_mlp[OFF_B1 + j] += gh1[j];
                for (int i2 = 0; i2 < MLP_IN; ++i2) {
                    g_mlp[OFF_W1 + j * MLP_IN + i2] += gh1[j] * a.x[i2];
                    gx[i2] += mlp[OFF_W1 + j * MLP_IN + i2] * gh1[j];
                }
            }
            for (int ch = 0; ch < 3; ++ch) gC[ch] += gx[ch];
            for (int ch = 0; ch < 4; ++ch) gV[ch] += gx[3 + ch];
        }

        /* Reverse through the compositing recurrence
         *   w_k = T_{k-1} a_k, T_k = T_{k-1} (1 - a_k), a_k = 1 - exp(-sigma_k delta). */
        double aT = gT; /* adjoint of T after the current sample */
        for (int64_t k = rec.n - 1; k >= 0; --k) {
            const rec_sample *rs = &rec.v[k];
            double alpha = -expm1(-rs->smp[0] * delta);
            double Tb = rs->T_before;
            double w = Tb * alpha;
            double gw = 0.0;
            double gc[3], gv[4];
            for (int ch = 0; ch < 3; ++ch) {
                gc[ch] = w * gC[ch];
                gw += gC[ch] * rs->smp[1 + ch];
            }
            for (int ch = 0; ch < 4; ++ch) {
                gv[ch] = w * gV[ch];
                gw += gV[ch] * rs->smp[4 + ch];
            }
            double g_alpha = gw * Tb - aT * Tb;
            double aT_prev = gw * alpha + aT * (1.0 - alpha);
            double g_sigma = g_alpha * delta * (1.0 - alpha); /* d alpha / d sigma = delta exp(-sigma delta) */
            aT = aT_prev;

            int64_t cidx[8];
            double cw[8], tmp[8];
            sample_point(g, rs->P, tmp, cidx, cw);
            for (int c = 0; c < 8; ++c) {
                if (cidx[c] < 0) continue;
                g_dens[cidx[c]] += g->sigma_scale * cw[c] * g_sigma;
                for (int ch = 0; ch < 3; ++ch) g_rgb[cidx[c] * 3 + ch] += cw[c] * gc[ch];
                for (int ch = 0; ch < 4; ++ch) g_feat[cidx[c] * 4 + ch] += cw[c] * gv[ch];
            }
        }
    }
    free(rec.v);
    return ORC_OK;
}

int orc_mlp_nparams(void) { return MLP_NPARAM; }

/* ------------------------------------------------------------- baking */

/*
 * Voxel visibility from training views (Section 5.3): the largest
 * transmittance between each voxel and any training camera.  sigma is a
 * densely evaluated field, float64 [N^3] (x fastest), density per unit
 * length of the world box.  Every ray of every camera is marched over the
 * whole sample lattice of step 1 (no early stop, no skipping); sample k lies
 * in voxel floor(P_k / 2^16), reads that voxel's density, and sees
 *     T_k = exp(-delta * sum_{j < k} sigma_j),  delta = 1/N,
 * the sum running over the ray's earlier samples inside the grid.
 * vis [N^3] receives max over all samples in the voxel of T_k (0 when no
 * sample falls in it); depth [N^3] (nullable) the smallest prefix sum
 * sum_{j<k} sigma_j of those samples (+inf when none), whose exponent gives
 * vis.  Rays are split over threads; each thread keeps its own copy of
 * the outputs, merged at the end.
 */
int orc_bake_visibility(int32_t N, const double *sigma, const orc_camera *cams, int32_t n_cams, double *vis,
                        double *depth, int32_t n_threads)
{
    if (N <= 0 || !sigma || !cams || n_cams <= 0 || !vis) return ORC_EINVAL;
    const int64_t nv = (int64_t)N * N * N;
    const int64_t L = (int64_t)N * 65536;
    const double delta = 1.0 / (double)N;
    int64_t total = 0;
    for (int32_t c = 0; c < n_cams; ++c) total += (int64_t)cams[c].W * cams[c].H;
    const int nt = set_threads(n_threads);
    double *buf = (double *)malloc(sizeof(double) * (size_t)nv * (size_t)nt);
    if (!buf) return ORC_ENOMEM;
    for (int64_t i = 0; i < nv * nt; ++i) buf[i] = INFINITY;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = buf + (size_t)nv * (size_t)tid;
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < total; ++r) {
            int32_t ci;
            int64_t px, py;
            locate_ray(cams, n_cams, r, &ci, &px, &py);
            int64_t o[3], s[3];
            double d[3];
            orc_ray_setup(&cams[ci], N, px, py, o, s, d);
            int64_t smax = 0, omax = 0;
            for (int a = 0; a < 3; ++a) {
                if (llabs(s[a]) > smax) smax = llabs(s[a]);
                if (llabs(o[a]) > omax) omax = llabs(o[a]);
            }
            const int64_t k_limit = (smax > 0) ? (omax + L) / smax + 2 : 0;
            double sum = 0.0;
            int seen_inside = 0;
            for (int64_t k = 0; k <= k_limit; ++k) {
                int64_t P[3];
                int inside = 1;
                for (int a = 0; a < 3; ++a) {
                    P[a] = o[a] + k * s[a];
                    if (P[a] < 0 || P[a] >= L) inside = 0;
                }
                if (!inside) {
                    if (seen_inside) break;
                    continue;
                }
                seen_inside = 1;
                const int64_t v = ((P[2] >> 16) * N + (P[1] >> 16)) * N + (P[0] >> 16);
                if (sum < mine[v]) mine[v] = sum;
                sum = sum + sigma[v];
            }
        }
    }
    for (int64_t v = 0; v < nv; ++v) {
        double m = INFINITY;
        for (int t = 0; t < nt; ++t)
            if (buf[(size_t)nv * t + v] < m) m = buf[(size_t)nv * t + v];
        vis[v] = isinf(m) ? 0.0 : exp(-delta * m);
        if (depth) depth[v] = m;
    }
    free(buf);
    return ORC_OK;
}
