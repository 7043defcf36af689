"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a
hand-derived closed form, an invariant, a special case that reduces to a
textbook result, or an independent brute-force computation.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import brute_marcher

Q16 = 65536


def axis_camera(eye, fwd, right, up, W_=1, H_=1, focal=1.0):
    return W.Camera(np.array(eye, float), np.array(fwd, float), np.array(right, float),
                    np.array(up, float), W_, H_, focal)


def world_of_voxel_coord(u, N):
    """World coordinate of voxel-unit coordinate u (grid box [-1, 1])."""
    return u * 2.0 / N - 1.0


# ----------------------------------------------------------------- ray setup

def test_ray_setup_hand_case():
    # 2x2 image, focal 1, looking +z with right +x and up +y: the top-left
    # pixel (0, 0) has x = y = -1/2, so D = (-1/2, 1/2, 1), |D| = sqrt(3/2).
    cam = axis_camera((0.0, 0.0, -2.0), (0, 0, 1), (1, 0, 0), (0, 1, 0), 2, 2, 1.0)
    o, s, d = O.ray_setup(cam, 64, 0, 0)
    r = math.sqrt(1.5)
    assert np.allclose(d, [-0.5 / r, 0.5 / r, 1.0 / r], atol=1e-15)
    # 32768 * 0.5 / sqrt(1.5) = 13377.31..., 32768 / sqrt(1.5) = 26754.62...
    assert list(s) == [-13377, 13377, 26755]
    # eye + 1 = (1, 1, -1) voxel-units * 32 * 65536
    assert list(o) == [32 * Q16, 32 * Q16, -32 * Q16]


def test_ray_setup_origin_fixed_point():
    cam = axis_camera((-2.0, 0.5, 0.25), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    o, s, _ = O.ray_setup(cam, 64, 0, 0)
    assert list(o) == [-1 * 32 * Q16, int(1.5 * 32 * Q16), int(1.25 * 32 * Q16)]
    assert list(s) == [32768, 0, 0]


def test_ray_setup_geometry_of_look_at_camera():
    cam = W.look_at((1.2, -1.1, 0.9), 33, 21, 39.0)
    _, _, d_tl = O.ray_setup(cam, 64, 0, 0)
    assert np.dot(d_tl, cam.up) > 0 and np.dot(d_tl, cam.right) < 0   # top-left looks up-left
    _, _, d_c = O.ray_setup(cam, 64, 16, 10)                            # odd sizes: exact centre
    assert np.allclose(d_c, cam.fwd / np.linalg.norm(cam.fwd), atol=1e-16)
    for (i, j) in [(0, 0), (5, 17), (32, 20)]:
        _, _, d1 = O.ray_setup(cam, 64, i, j)
        _, _, d2 = O.ray_setup(cam, 64, cam.W - 1 - i, j)               # mirror about the up-fwd plane
        assert abs(np.linalg.norm(d1) - 1.0) < 1e-15
        assert abs(np.dot(d1, cam.right) + np.dot(d2, cam.right)) < 1e-15
        assert abs(np.dot(d1, cam.up) - np.dot(d2, cam.up)) < 1e-15
    # the last column's centre lies half a pixel inside the horizontal field of view
    _, _, d_r = O.ray_setup(cam, 64, cam.W - 1, 10)
    ang = math.atan2(np.dot(d_r, cam.right), np.dot(d_r, cam.fwd))
    assert abs(ang - math.atan((cam.W / 2 - 0.5) / cam.focal)) < 1e-14
    assert abs(math.atan(cam.W / 2 / cam.focal) - math.radians(19.5)) < 1e-14


# -------------------------------------------------------- lattice and visits

def grid_with_blocks(N, B, occupied_xyz, fill=200, seed=5):
    """Block-sparse grid whose occupied macroblocks (bx, by, bz) have every
    density byte equal to `fill` and random colours/features."""
    G = N // B
    rng = np.random.default_rng(seed)
    ind = np.full(G ** 3, -1, np.int32)
    perm = rng.permutation(len(occupied_xyz))
    for n, (bx, by, bz) in enumerate(occupied_xyz):
        ind[(bz * G + by) * G + bx] = perm[n]
    nb = len(occupied_xyz)
    dens = np.full((nb, B, B, B), fill, np.uint8)
    rgb = rng.integers(0, 256, (nb, B, B, B, 3), dtype=np.uint8)
    feat = rng.integers(0, 256, (nb, B, B, B, 4), dtype=np.uint8)
    return W.Grid(N, B, ind, dens, rgb, feat)


def test_visits_axis_aligned_rays():
    N, B = 64, 8
    G = N // B
    occ = [(1, 3, 4), (4, 3, 4), (5, 3, 4), (7, 3, 4), (2, 3, 5), (3, 2, 4)]
    g = grid_with_blocks(N, B, occ)
    og = O.OracleGrid(g, sigma_scale=0.0)  # no opacity: nothing stops the ray
    # world y, z at voxel-unit coordinates 3*8 + 2.5 and 4*8 + 5.5
    y = world_of_voxel_coord(3 * B + 2.5, N)
    z = world_of_voxel_coord(4 * B + 5.5, N)
    plus_x = axis_camera((-2.0, y, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    minus_x = axis_camera((2.0, y, z), (-1, 0, 0), (0, 1, 0), (0, 0, 1))
    row = [(bx, 3, 4) for bx in range(G)]
    expect = [(bz * G + by) * G + bx for (bx, by, bz) in row if (bx, by, bz) in occ]
    vis, cnt = O.trace_visits(og, [plus_x])
    assert list(vis[0, :cnt[0]]) == expect
    vis, cnt = O.trace_visits(og, [minus_x])
    assert list(vis[0, :cnt[0]]) == expect[::-1]


def test_visits_half_open_faces():
    N, B = 64, 8
    G = N // B
    occ = [(2, 3, 4), (2, 4, 4)]
    g = grid_with_blocks(N, B, occ)
    og = O.OracleGrid(g, sigma_scale=0.0)
    z = world_of_voxel_coord(4 * B + 1.5, N)
    # y exactly on the face between block rows 3 and 4: belongs to row 4
    y_face = world_of_voxel_coord(4 * B, N)
    cam = axis_camera((-2.0, y_face, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    o, s, _ = O.ray_setup(cam, N, 0, 0)
    assert o[1] == 4 * B * Q16
    vis, cnt = O.trace_visits(og, [cam])
    assert list(vis[0, :cnt[0]]) == [(4 * G + 4) * G + 2]
    # y = +1 is outside (half-open grid), y = -1 is inside.  Block (2, 0, 5)
    # is occupied so that a closed upper bound (y block row G, which aliases
    # row 0 of the next z slab in x-fastest order) would report a visit.
    g_top = grid_with_blocks(N, B, occ + [(2, 0, 5)])
    top = axis_camera((-2.0, 1.0, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    _, cnt = O.trace_visits(O.OracleGrid(g_top, sigma_scale=0.0), [top])
    assert cnt[0] == 0
    g2 = grid_with_blocks(N, B, [(3, 0, 4)])
    og2 = O.OracleGrid(g2, sigma_scale=0.0)
    bottom = axis_camera((-2.0, -1.0, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    vis, cnt = O.trace_visits(og2, [bottom])
    assert list(vis[0, :cnt[0]]) == [(4 * G + 0) * G + 3]


def test_visits_diagonal_through_block_corners():
    N, B = 64, 8
    G = N // B
    occ = [(b, b, b) for b in (0, 2, 3, 6)] + [(1, 2, 3)]
    g = grid_with_blocks(N, B, occ)
    og = O.OracleGrid(g, sigma_scale=0.0)
    r3 = 1.0 / math.sqrt(3.0)
    # right and up only need to be orthogonal to fwd for the 1x1 image
    cam = axis_camera((-1.5, -1.5, -1.5), (r3, r3, r3), (r3, -r3, 0.0), (0.0, 0.0, 1.0))
    o, s, _ = O.ray_setup(cam, N, 0, 0)
    assert list(s) == [18919, 18919, 18919]   # rint(32768 / sqrt 3) = rint(18918.6)
    vis, cnt = O.trace_visits(og, [cam])
    assert list(vis[0, :cnt[0]]) == [(b * G + b) * G + b for b in (0, 2, 3, 6)]


def test_ray_missing_grid_returns_background():
    g = W.tiny_grid()
    og = O.OracleGrid(g)
    cam = axis_camera((0.0, 0.0, 3.0), (0, 0, 1), (1, 0, 0), (0, 1, 0))  # looks away
    bg = (0.2, 0.4, 0.7)
    r = O.render(og, W.mlp_weights(), [cam], bg=bg)
    assert np.array_equal(r["rgba"][0], np.array([0.2, 0.4, 0.7, 0.0]))
    assert r["aux"][0, 8] == 0 and r["counters"][0, 0] == 0


def test_empty_grid_returns_background_everywhere():
    g = W.tiny_grid()
    g.indirection[:] = -1
    og = O.OracleGrid(g)
    r = O.render(og, W.mlp_weights(), [W.orbit_camera(16, 16)], bg=(0.1, 0.5, 0.9))
    assert np.all(r["rgba"] == np.array([0.1, 0.5, 0.9, 0.0]))
    assert np.all(r["aux"][:, 8] == 0) and np.all(r["counters"][:, 1:4] == 0)
    assert np.any(r["counters"][:, 0] > 0)


# ----------------------------------------------------------------- trilinear

def test_sample_at_voxel_centre_returns_voxel_value():
    g = W.tiny_grid(n_occupied=64, seed=3)
    og = O.OracleGrid(g)
    G, B = g.G, g.B
    rng = np.random.default_rng(0)
    occ_lin = np.nonzero(g.indirection >= 0)[0]
    for _ in range(200):
        lin = int(rng.choice(occ_lin))
        bid = g.indirection[lin]
        bx, by, bz = lin % G, (lin // G) % G, lin // (G * G)
        lx, ly, lz = rng.integers(0, B, 3)
        P = [(bx * B + lx) * Q16 + 32768, (by * B + ly) * Q16 + 32768, (bz * B + lz) * Q16 + 32768]
        out, act = O.sample(og, P)
        byte = g.dens[bid, lz, ly, lx]
        assert out[0] == pytest.approx(50.0 * byte / 255.0, abs=1e-13)
        assert np.allclose(out[1:4], g.rgb[bid, lz, ly, lx] / 255.0, atol=1e-15)
        assert np.allclose(out[4:8], g.feat[bid, lz, ly, lx] / 255.0, atol=1e-15)
        assert act == (byte != 0)


def dense_float_grid(N, B, fn):
    """Fully occupied grid whose values come from fn(x, y, z) at voxel indices."""
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    vals = fn(x.astype(float), y.astype(float), z.astype(float))  # [N,N,N,8]
    dummy = np.ones((N, N, N), np.uint8)
    g = W.grid_from_dense(dummy, np.zeros((N, N, N, 3), np.uint8), np.zeros((N, N, N, 4), np.uint8), B,
                          permute_seed=7)
    G = N // B
    d = np.zeros((g.n_blocks, B, B, B)); r = np.zeros((g.n_blocks, B, B, B, 3))
    f = np.zeros((g.n_blocks, B, B, B, 4))
    for lin in range(G ** 3):
        bid = g.indirection[lin]
        bx, by, bz = lin % G, (lin // G) % G, lin // (G * G)
        sl = (slice(bz * B, bz * B + B), slice(by * B, by * B + B), slice(bx * B, bx * B + B))
        d[bid] = vals[sl][..., 0]
        r[bid] = vals[sl][..., 1:4]
        f[bid] = vals[sl][..., 4:8]
    return g, (d, r, f)


def test_trilinear_reproduces_affine_fields():
    N, B = 16, 4
    coef = np.random.default_rng(1).normal(size=(8, 4))

    def fn(x, y, z):
        return np.stack([c[0] + c[1] * x + c[2] * y + c[3] * z + 40.0 for c in coef], axis=-1)

    g, vals = dense_float_grid(N, B, fn)
    og = O.OracleGrid(g, values=vals, sigma_scale=2.0)
    rng = np.random.default_rng(2)
    for _ in range(300):
        P = rng.integers(32768, (N - 1) * Q16 + 32768, size=3)   # all corners inside
        out, act = O.sample(og, P)
        u = (P - 32768) / Q16                                      # continuous voxel index
        exact = fn(u[0], u[1], u[2])
        assert act
        assert out[0] == pytest.approx(2.0 * exact[0], rel=1e-13)
        assert np.allclose(out[1:8], exact[1:8], rtol=1e-13)


def test_trilinear_weights_and_outside_corners():
    N, B = 16, 4
    g, vals = dense_float_grid(N, B, lambda x, y, z: np.stack([np.ones_like(x)] * 8, axis=-1))
    og = O.OracleGrid(g, values=vals, sigma_scale=1.0)
    # a fully occupied constant field: weights sum to one wherever all corners are inside
    out, _ = O.sample(og, [5 * Q16 + 1234, 7 * Q16 + 40000, 3 * Q16 + 7])
    assert np.allclose(out, 1.0, atol=1e-15)
    # grid corner P = 0: i0 = -1, f = 1/2 -> only voxel (0,0,0) is inside, weight 1/8
    out, act = O.sample(og, [0, 0, 0])
    assert np.allclose(out, 0.125, atol=1e-16) and act
    # on the face x = 0 (P_x = 0) with y, z at voxel centres: weight 1/2
    out, _ = O.sample(og, [0, 3 * Q16 + 32768, 3 * Q16 + 32768])
    assert np.allclose(out, 0.5, atol=1e-16)


def test_neighbour_blocks_read_through_indirection():
    N, B = 16, 4
    g = grid_with_blocks(N, B, [(1, 1, 1), (2, 1, 1)], fill=100, seed=9)
    og = O.OracleGrid(g)
    # P on the face x = 8 between blocks 1 and 2, y, z at voxel centres inside row 1
    P = [8 * Q16, 5 * Q16 + 32768, 6 * Q16 + 32768]
    out, act = O.sample(og, P)
    G = N // B
    ida = g.indirection[(1 * G + 1) * G + 1]
    idb = g.indirection[(1 * G + 1) * G + 2]
    # corners x = 7 (block 1, local 3) and x = 8 (block 2, local 0), weight 1/2 each
    rgb = 0.5 * (g.rgb[ida, 2, 1, 3].astype(float) + g.rgb[idb, 2, 1, 0]) / 255.0
    assert np.allclose(out[1:4], rgb, atol=1e-15) and act
    # the same face against an empty neighbour block reads zero there
    P2 = [4 * Q16, 5 * Q16 + 32768, 6 * Q16 + 32768]
    out2, _ = O.sample(og, P2)
    assert np.allclose(out2[1:4], 0.5 * g.rgb[ida, 2, 1, 0] / 255.0, atol=1e-15)
    assert out2[0] == pytest.approx(0.5 * 50.0 * 100 / 255.0, rel=1e-14)


def test_active_predicate_needs_nonzero_weight():
    N, B = 16, 4
    g = grid_with_blocks(N, B, [(1, 1, 1)], fill=0, seed=2)
    G = N // B
    bid = g.indirection[(1 * G + 1) * G + 1]
    g.dens[bid, 1, 1, 2] = 77                          # voxel (6, 5, 5)
    og = O.OracleGrid(g)
    # centre of voxel (5,5,5): f = 0 on every axis, the (6,5,5) corner has weight 0
    _, act = O.sample(og, [5 * Q16 + 32768, 5 * Q16 + 32768, 5 * Q16 + 32768])
    assert not act
    out, act = O.sample(og, [5 * Q16 + 32768 + 1, 5 * Q16 + 32768, 5 * Q16 + 32768])
    assert act and out[0] > 0


# --------------------------------------------------------------- compositing

def test_composite_single_sample_closed_form():
    sigma, delta = 37.0, 1.0 / 64
    c = np.array([0.2, 0.5, 0.9]); v = np.array([0.1, 0.3, 0.6, 1.0])
    C, V, T, n = O.composite(np.concatenate([[sigma], c, v]), delta)
    a = 1.0 - math.exp(-sigma * delta)
    assert np.allclose(C, a * c, rtol=1e-15) and np.allclose(V, a * v, rtol=1e-15)
    assert T == pytest.approx(1.0 - a, rel=1e-15) and n == 1


def test_composite_constant_slab_closed_form():
    sigma, delta, n = 3.0, 1.0 / 512, 40
    c = np.array([0.7, 0.1, 0.4]); v = np.array([0.3, 0.3, 0.8, 0.05])
    rows = np.tile(np.concatenate([[sigma], c, v]), (n, 1))
    C, V, T, used = O.composite(rows, delta, early_stop=False)
    Texp = math.exp(-n * sigma * delta)
    assert T == pytest.approx(Texp, rel=1e-14)
    assert np.allclose(C, c * (1 - Texp), rtol=1e-13) and np.allclose(V, v * (1 - Texp), rtol=1e-13)


def test_composite_invariants_and_stop_rule():
    rng = np.random.default_rng(4)
    rows = np.concatenate([rng.uniform(0, 60, (300, 1)), rng.uniform(0, 1, (300, 7))], axis=1)
    delta = 1.0 / 64
    Ts = [O.composite(rows[:m], delta, early_stop=False)[2] for m in range(1, 60)]
    assert all(b <= a for a, b in zip(Ts, Ts[1:]))                      # T non-increasing
    # sum of weights telescopes to 1 - T: use unit colour in every channel
    ones = rows.copy(); ones[:, 1:] = 1.0
    C, V, T, _ = O.composite(ones[:50], delta, early_stop=False)
    assert np.allclose(C, 1.0 - T, atol=1e-15) and np.allclose(V, 1.0 - T, atol=1e-15)
    # early stop: ends right after the first sample with T < t_stop
    C, V, T, n = O.composite(rows, delta, t_stop=1e-3, early_stop=True)
    Tall = np.cumprod(np.exp(-rows[:, 0] * delta))
    first = int(np.argmax(Tall < 1e-3))
    assert n == first + 1 and T == pytest.approx(Tall[first], rel=1e-12) and T < 1e-3
    assert Tall[first - 1] >= 1e-3


def test_render_constant_slab_along_axis():
    # density only in voxel columns x in [20, 30) of the row the ray follows;
    # the ray runs along +x through voxel centres in y and z.
    N, B = 64, 8
    dens = np.zeros((N, N, N), np.uint8)
    rgb = np.zeros((N, N, N, 3), np.uint8); feat = np.zeros((N, N, N, 4), np.uint8)
    jy, jz = 29, 35
    dens[jz, jy, 20:30] = 51                                   # sigma = 10
    rgb[jz, jy, 20:30] = (255, 102, 0); feat[jz, jy, 20:30] = (0, 51, 102, 255)
    g = W.grid_from_dense(dens, rgb, feat, B, permute_seed=1)
    og = O.OracleGrid(g)
    y = world_of_voxel_coord(jy + 0.5, N); z = world_of_voxel_coord(jz + 0.5, N)
    cam = axis_camera((-2.0, y, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    bg = np.array([0.25, 0.5, 0.75])
    r = O.render(og, None, [cam], bg=bg, mlp_on=False, early_stop=False)
    # Samples sit at voxel units 20, 20.5, ..., 30.  The end faces 20 and 30
    # see half the slab voxel (sigma/2 and colour c/2, the outside voxel
    # reads zero); the 19 samples in between see full sigma and colour c.
    sig, dl = 10.0, 1.0 / N
    Th, Tf = math.exp(-0.5 * sig * dl), math.exp(-sig * dl)
    T = Th * Tf ** 19 * Th
    # first face: (1 - Th) c/2; middle: Th (1 - Tf^19) c; last face: Th Tf^19 (1 - Th) c/2
    k = 0.5 * (1 - Th) + Th * (1 - Tf ** 19) + Th * Tf ** 19 * 0.5 * (1 - Th)
    c = np.array([1.0, 0.4, 0.0]); v = np.array([0.0, 0.2, 0.4, 1.0])
    assert r["counters"][0, 3] == 21
    assert r["rgba"][0, 3] == pytest.approx(1 - T, rel=1e-13)
    assert np.allclose(r["rgba"][0, :3], k * c + T * bg, rtol=1e-13)
    assert np.allclose(r["aux"][0, 3:7], k * v, rtol=1e-13)


# -------------------------------------------------------------- MLP and PE

def test_encode_values_and_order():
    x = O.encode([0.1, 0.2, 0.3], [0.4, 0.5, 0.6, 0.7], [0.5, 0.25, 1.0 / 6.0])
    assert np.allclose(x[:10], [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.5, 0.25, 1.0 / 6.0])
    s2 = math.sqrt(2) / 2
    # octave 0: sin(pi d), cos(pi d); octave 1: sin(2 pi d), cos(2 pi d)
    assert np.allclose(x[10:16], [1.0, s2, 0.5, 0.0, s2, math.sqrt(3) / 2], atol=1e-15)
    assert np.allclose(x[16:22], [0.0, 1.0, math.sqrt(3) / 2, -1.0, 0.0, 0.5], atol=1e-15)
    x = O.encode([0, 0, 0], [0, 0, 0, 0], [1.0, 0.0, 0.0])
    for l in range(4):
        sin_part, cos_part = x[10 + 6 * l: 13 + 6 * l], x[13 + 6 * l: 16 + 6 * l]
        assert np.all(np.abs(sin_part) < 1e-14)
        assert cos_part[0] == pytest.approx(-1.0 if l == 0 else 1.0, abs=1e-15)
        assert cos_part[1] == 1.0 and cos_part[2] == 1.0


def test_mlp_zero_weights_give_half():
    R = O.mlp_eval(np.zeros(883), np.random.default_rng(0).normal(size=34))
    assert np.all(R == 0.5)


def test_mlp_single_path_catches_transposition():
    p = W.MLP(np.zeros((16, 34)), np.zeros(16), np.zeros((16, 16)), np.zeros(16), np.zeros((3, 16)),
              np.zeros(3))
    p.W1[2, 5] = 1.5          # hidden unit 2 reads input 5
    p.W2[7, 2] = -2.0         # hidden unit 7 of layer 2 reads unit 2
    p.W3[1, 7] = -0.5         # green reads unit 7
    p.b3[:] = [0.3, 0.0, -0.2]
    x = np.zeros(34); x[5] = 0.8
    R = O.mlp_eval(p, x)
    # layer 2 pre-activation is -2 * 1.2 < 0: relu kills it
    assert np.allclose(R, [1 / (1 + math.exp(-0.3)), 0.5, 1 / (1 + math.exp(0.2))], atol=1e-16)
    p.W2[7, 2] = 2.0
    R = O.mlp_eval(p, x)
    assert R[1] == pytest.approx(1.0 / (1.0 + math.exp(0.5 * 2.0 * 1.2)), rel=1e-15)
    x2 = np.zeros(34); x2[2] = 0.8          # a transposed W1 would read input 2 for unit 5
    assert O.mlp_eval(p, x2)[1] == 0.5
    p.b1[2] = -2.0                          # relu on the first layer
    assert O.mlp_eval(p, x)[1] == 0.5


# --------------------------------------------------------------- end to end

@pytest.mark.parametrize("seed,n_occ,early", [(0, 8, True), (1, 64, True), (2, 200, False), (3, 200, True)])
def test_oracle_matches_brute_force_dense_marcher(seed, n_occ, early):
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    mlp = W.mlp_weights(seed + 10)
    cam = W.orbit_camera(24, 20, seed=seed + 1)
    og = O.OracleGrid(g)
    bg = (0.3, 0.6, 0.9)
    r = O.render(og, mlp, [cam], bg=bg, early_stop=early)
    lat = [O.ray_setup(cam, g.N, i, j) for j in range(cam.H) for i in range(cam.W)]
    lat = tuple(np.array(a) for a in zip(*lat))
    b = brute_marcher.march(g, lat, mlp, bg=bg, early_stop=early)
    assert np.max(np.abs(r["rgba"] - b["rgba"])) < 1e-12
    assert np.array_equal(r["aux"][:, 8] != 0, b["gate"])
    assert np.array_equal(r["counters"][:, 3], b["n_used"])
    # every counter, including the set of composited sample indices
    assert np.array_equal(r["counters"].astype(np.int64), b["counters"])
    vis, cnt = O.trace_visits(og, [cam], early_stop=early)
    for i in range(cam.n_rays):
        assert list(vis[i, :cnt[i]]) == b["visits"][i]
    if early and n_occ >= 64:
        assert np.any(r["counters"][:, 4] >= 0)   # the stop rule was exercised


def test_oracle_ray_ids_select_rays():
    g = W.tiny_grid(n_occupied=64, seed=1)
    cams = [W.orbit_camera(9, 7, seed=4), W.orbit_camera(5, 6, seed=5)]
    og = O.OracleGrid(g)
    mlp = W.mlp_weights()
    full = O.render(og, mlp, cams)
    ids = np.array([0, 62, 63, 92, 70, 5])
    part = O.render(og, mlp, cams, ray_ids=ids)
    assert np.array_equal(full["rgba"][ids], part["rgba"])
    with pytest.raises(RuntimeError):
        O.render(og, mlp, cams, ray_ids=np.array([93]))


# ------------------------------------------------- render variants (flags)

@pytest.mark.parametrize("seed,n_occ,early", [(0, 64, True), (2, 200, False), (5, 120, True)])
def test_variants_match_brute_force(seed, n_occ, early):
    # the nearest-voxel gate of the WebGL renderer (Appendix A) and the
    # partial un-premultiply of Eq. 9, each against the dense marcher
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    mlp = W.mlp_weights(seed + 10)
    cam = W.orbit_camera(24, 20, seed=seed + 1)
    og = O.OracleGrid(g)
    lat = [O.ray_setup(cam, g.N, i, j) for j in range(cam.H) for i in range(cam.W)]
    lat = tuple(np.array(a) for a in zip(*lat))
    for kw in (dict(nn_gate=True), dict(unpremultiply=True), dict(nn_gate=True, unpremultiply=True)):
        r = O.render(og, mlp, [cam], bg=(0.3, 0.6, 0.9), early_stop=early, **kw)
        b = brute_marcher.march(g, lat, mlp, bg=(0.3, 0.6, 0.9), early_stop=early, **kw)
        assert np.max(np.abs(r["rgba"] - b["rgba"])) < 1e-12, kw
        assert np.array_equal(r["counters"][:, 3], b["n_used"]), kw
        assert np.array_equal(r["counters"].astype(np.int64), b["counters"]), kw
    exact = O.render(og, mlp, [cam], early_stop=False)["counters"][:, 3]
    gated = O.render(og, mlp, [cam], early_stop=False, nn_gate=True)["counters"][:, 3]
    assert np.all(gated <= exact) and np.any(gated < exact)   # a strict subset of the samples


def _single_voxel_ray(sig_byte, c_bytes):
    # one voxel (x = 20, y = 29, z = 35) of a 64^3 grid; a ray along +x through
    # its centre line, samples at voxel units 0, 0.5, 1, ... in x
    N, B = 64, 8
    dens = np.zeros((N, N, N), np.uint8)
    rgb = np.zeros((N, N, N, 3), np.uint8); feat = np.zeros((N, N, N, 4), np.uint8)
    dens[35, 29, 20] = sig_byte
    rgb[35, 29, 20] = c_bytes
    g = W.grid_from_dense(dens, rgb, feat, B, permute_seed=2)
    y = world_of_voxel_coord(29.5, N); z = world_of_voxel_coord(35.5, N)
    cam = axis_camera((-2.0, y, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    return O.OracleGrid(g), cam, N


def test_nn_gate_single_voxel_closed_form():
    # Exact predicate: samples at x = 20 (weight 1/2), 20.5 (weight 1) and 21
    # (weight 1/2) are composited.  Nearest-voxel gate: only x in [20, 21),
    # i.e. the samples at 20 and 20.5.
    og, cam, N = _single_voxel_ray(102, (255, 0, 51))
    sig, dl = 50.0 * 102 / 255, 1.0 / N
    c = np.array([1.0, 0.0, 0.2])
    Th, Tf = math.exp(-0.5 * sig * dl), math.exp(-sig * dl)
    r = O.render(og, None, [cam], mlp_on=False, early_stop=False, bg=(0, 0, 0))
    assert r["counters"][0, 3] == 3
    assert r["rgba"][0, 3] == pytest.approx(1 - Th * Tf * Th, rel=1e-13)
    rn = O.render(og, None, [cam], mlp_on=False, early_stop=False, bg=(0, 0, 0), nn_gate=True)
    assert rn["counters"][0, 3] == 2
    assert rn["rgba"][0, 3] == pytest.approx(1 - Th * Tf, rel=1e-13)
    assert np.allclose(rn["rgba"][0, :3], (1 - Th) * c / 2 + Th * (1 - Tf) * c, rtol=1e-13)


def test_unpremultiply_closed_form():
    # Eq. 9 on a composited alpha a: colour, features and alpha scale by
    # min(1, 1.5 a) / a, so a >= 2/3 saturates to 1 and the background vanishes.
    for byte in (40, 255):
        og, cam, N = _single_voxel_ray(byte, (255, 128, 0))
        bg = np.array([0.2, 0.4, 0.6])
        r = O.render(og, None, [cam], mlp_on=False, early_stop=False, bg=bg)
        u = O.render(og, None, [cam], mlp_on=False, early_stop=False, bg=bg, unpremultiply=True)
        a = r["rgba"][0, 3]
        sc = min(1.0, 1.5 * a) / a
        C = r["aux"][0, :3]
        assert u["rgba"][0, 3] == pytest.approx(min(1.0, 1.5 * a), rel=1e-14)
        assert np.allclose(u["rgba"][0, :3], C * sc + (1 - min(1.0, 1.5 * a)) * bg, rtol=1e-13, atol=1e-15)
    # a ray that composites nothing is left alone
    e = O.render(og, None, [W.orbit_camera(4, 4, seed=1)], mlp_on=False, unpremultiply=True, bg=bg)
    assert np.allclose(e["rgba"][e["aux"][:, 8] == 0], np.concatenate([bg, [0.0]]))


def test_per_sample_mlp_zero_network_closed_form():
    # A zero network outputs sigmoid(0) = 1/2 at every sample, so the
    # non-deferred render adds (1/2) sum_k w_k = (1 - T)/2 to the deferred
    # render's diffuse colour, and runs no per-pixel network.
    g = W.tiny_grid(n_occupied=64, seed=1)
    cam = W.orbit_camera(16, 12, seed=2)
    og = O.OracleGrid(g)
    bg = np.array([0.1, 0.2, 0.3])
    zero = np.zeros(883)
    d = O.render(og, zero, [cam], bg=bg, mlp_on=False)
    p = O.render(og, zero, [cam], bg=bg, per_sample_mlp=True)
    T = 1.0 - d["rgba"][:, 3]
    np.testing.assert_allclose(p["rgba"][:, :3], d["rgba"][:, :3] + 0.5 * (1.0 - T)[:, None], rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(p["counters"], d["counters"])


@pytest.mark.parametrize("seed,early,gate", [(0, True, False), (2, False, False), (3, True, True)])
def test_per_sample_mlp_matches_brute_force(seed, early, gate):
    g = W.tiny_grid(n_occupied=120, seed=seed)
    mlp = W.mlp_weights(seed + 20)
    cam = W.orbit_camera(20, 16, seed=seed + 3)
    og = O.OracleGrid(g)
    lat = [O.ray_setup(cam, g.N, i, j) for j in range(cam.H) for i in range(cam.W)]
    lat = tuple(np.array(a) for a in zip(*lat))
    r = O.render(og, mlp, [cam], bg=(0.3, 0.6, 0.9), early_stop=early, per_sample_mlp=True, nn_gate=gate)
    b = brute_marcher.march(g, lat, mlp, bg=(0.3, 0.6, 0.9), early_stop=early, per_sample_mlp=True, nn_gate=gate)
    assert np.max(np.abs(r["rgba"] - b["rgba"])) < 1e-12
    deferred = O.render(og, mlp, [cam], bg=(0.3, 0.6, 0.9), early_stop=early, nn_gate=gate)["rgba"]
    assert np.max(np.abs(r["rgba"] - deferred)) > 1e-3   # a different image, same samples
