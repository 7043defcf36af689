"""Pins of the FP64 baking reference (Section 5.3 culls, Section 5.4 8-bit
quantisation) in oracle/bake.py and orc_bake_visibility: transmittance along
an axis-aligned ray in closed form, the maximum over cameras on opposite
sides, an empty field, an opaque slab hiding what lies behind it, the
empty-space threshold on both sides of its closed form, and the
quantisation as the exact inverse of the renderer's dequantisation."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bake as K


def axis_camera(N, direction, yv, zv, dist=3.0):
    """1x1 camera on the x axis looking along +x (direction=+1) or -x, its
    single ray through the centres of voxel row (y = yv, z = zv)."""
    y = (yv + 0.5) * 2.0 / N - 1.0
    z = (zv + 0.5) * 2.0 / N - 1.0
    fwd = np.array([float(direction), 0.0, 0.0])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    return W.Camera(np.array([-direction * dist, y, z]), fwd, right, up, 1, 1, 1.0)


def test_axis_ray_transmittance_closed_form():
    # The ray's samples are half a voxel apart, the first at the grid face:
    # voxel x is entered at sample 2x, after 2x samples of density s0, so
    # its visibility is exp(-2 x s0 / N) and every other voxel has none.
    N, s0, yv, zv = 16, 0.75, 5, 9
    sigma = np.full((N, N, N), s0)
    vis, depth = K.voxel_visibility(sigma, [axis_camera(N, +1, yv, zv)])
    x = np.arange(N)
    np.testing.assert_array_equal(depth[zv, yv, :], 2 * x * s0)
    np.testing.assert_allclose(vis[zv, yv, :], np.exp(-2 * x * s0 / N), rtol=1e-15)
    mask = np.ones_like(vis, bool)
    mask[zv, yv, :] = False
    assert np.all(vis[mask] == 0.0) and np.all(np.isinf(depth[mask]))


def test_camera_inside_the_grid_sees_from_its_own_voxel():
    # eye on the face between voxels 2 and 3 along x, looking +x: sample k sits
    # at x = 3 + k/2 voxels (k = 0 included), so voxel x >= 3 is entered after
    # 2 (x - 3) samples and the voxels behind the eye see nothing
    N, s0, yv, zv = 16, 0.25, 7, 4
    sigma = np.full((N, N, N), s0)
    cam = axis_camera(N, +1, yv, zv)
    cam.eye = np.array([3.0 * 2.0 / N - 1.0, cam.eye[1], cam.eye[2]])
    vis, depth = K.voxel_visibility(sigma, [cam])
    x = np.arange(3, N)
    np.testing.assert_array_equal(depth[zv, yv, 3:], 2 * (x - 3) * s0)
    assert np.all(vis[zv, yv, :3] == 0.0) and vis[zv, yv, 3] == 1.0


def test_visibility_is_the_maximum_over_cameras():
    # From the -x side voxel x is entered after 30 - 2x samples (the ray's
    # first sample sits in the upper half of voxel N - 1).
    N, s0, yv, zv = 16, 0.5, 3, 12
    sigma = np.full((N, N, N), s0)
    cams = [axis_camera(N, +1, yv, zv), axis_camera(N, -1, yv, zv)]
    vis, depth = K.voxel_visibility(sigma, cams)
    x = np.arange(N)
    np.testing.assert_array_equal(depth[zv, yv, :], np.minimum(2 * x, 2 * N - 2 - 2 * x) * s0)
    vis_back, _ = K.voxel_visibility(sigma, cams[1:])
    np.testing.assert_allclose(vis_back[zv, yv, :], np.exp(-(2 * N - 2 - 2 * x) * s0 / N), rtol=1e-15)


def test_empty_field_is_fully_visible_and_fully_culled():
    N, B = 32, 8
    sigma = np.zeros((N, N, N), np.float32)
    cams = W.sphere_cameras([(24, 24, 60.0)] * 6, seed=1)
    c = K.cull(sigma, B, cams)
    seen = c.vis > 0
    assert seen.sum() > 0.9 * seen.size
    assert np.all(c.vis[seen] == 1.0) and np.all(c.depth[seen] == 0.0)
    assert np.all(c.alpha == 0.0) and c.n_blocks == 0
    # tau_alpha = 0 keeps every macroblock some training sample reaches
    c0 = K.cull(sigma, B, cams, tau_alpha=0.0)
    np.testing.assert_array_equal(c0.keep, seen)
    np.testing.assert_array_equal(c0.indirection[seen], np.arange(int(seen.sum())))


def test_opaque_slab_hides_what_lies_behind_it():
    # Slab over voxels x in [12, 16), density 400: every ray that gets past it
    # crosses at least 8 samples of it, transmittance <= exp(-100).  A dense
    # ball behind it has a high alpha but no visibility; the slab's own
    # macroblocks (x in [8, 16)) are seen with T = 1 at their front face.
    N, B = 32, 8
    sigma = np.zeros((N, N, N), np.float32)
    sigma[:, :, 12:16] = 400.0
    sigma[14:18, 14:18, 26:30] = 900.0
    cams = [W.look_at((-3.0, 0.1 * i, 0.05 * i), 40, 40, 30.0, target=(0.0, 0.1 * i, 0.05 * i)) for i in range(3)]
    c = K.cull(sigma, B, cams)
    G = N // B
    bx = np.arange(G ** 3) % G
    assert np.all(c.vis[bx >= 2] < 1e-40)
    hit = c.vis > 0
    assert np.all(c.vis[(bx <= 1) & hit] == 1.0) and hit[bx == 1].sum() >= 8
    assert np.all(c.alpha[bx == 1] == pytest.approx(1.0 - math.exp(-400.0 / N)))
    ball = (np.arange(G ** 3) // (G * G) == 1) & ((np.arange(G ** 3) // G) % G == 1) & (bx == 3)
    assert c.alpha[ball].item() > 0.99 and not c.keep[ball].item()
    np.testing.assert_array_equal(c.keep, (bx == 1) & hit)


@pytest.mark.parametrize("rel,kept", [(1.0 + 1e-6, True), (1.0 - 1e-6, False), (0.6, False)])
def test_empty_space_threshold_closed_form(rel, kept):
    # alpha = 1 - exp(-sigma / N) >= 0.005  <=>  sigma >= -N log(0.995); a
    # voxel width of 2/N (or a sign slip) would move the threshold.
    N, B = 32, 8
    s_t = -N * math.log(1.0 - K.TAU_ALPHA)
    sigma = np.zeros((N, N, N))
    sigma[20, 5, 9] = s_t * rel
    cams = W.sphere_cameras([(24, 24, 60.0)] * 6, seed=1)
    c = K.cull(sigma, B, cams)
    lin = (20 // B * (N // B) + 5 // B) * (N // B) + 9 // B
    assert c.vis[lin] == 1.0
    assert c.alpha[lin] == pytest.approx(1.0 - math.exp(-s_t * rel / N), rel=1e-15)
    assert bool(c.keep[lin]) is kept and c.n_blocks == int(kept)


def test_quantisation_inverts_the_render_dequantisation():
    b = np.arange(256)
    np.testing.assert_array_equal(K.quantize((b / 255.0).astype(np.float32)), b)
    np.testing.assert_array_equal(K.quantize((b * (50.0 / 255.0)).astype(np.float32), 50.0), b)
    x = np.array([-0.3, 0.0, 1.0, 1.7, np.nan, np.inf, -np.inf], np.float32)
    np.testing.assert_array_equal(K.quantize(x), [0, 0, 255, 255, 0, 255, 0])
    # half-way cases round to even: 0.5 * 255 = 127.5 exactly in float32
    assert K.quantize(np.float32([0.5]))[0] == 128
    assert K.quantize(np.float32([1.5 / 255.0]))[0] == round(float(np.float32(1.5 / 255.0) * np.float32(255.0)))


def test_bake_of_a_dequantised_grid_returns_its_bytes():
    # A sparse grid turned into a dense field (sigma = 50 b / 255, c = b / 255)
    # and baked again: with every block in view, the kept blocks are exactly
    # the occupied blocks whose largest density clears the alpha threshold,
    # and their bytes come back unchanged.
    g = W.tiny_grid(N=32, B=8, n_occupied=20, seed=5)
    N, B, G = g.N, g.B, g.G
    sigma = np.zeros((N, N, N), np.float32)
    rgb = np.zeros((N, N, N, 3), np.float32)
    feat = np.zeros((N, N, N, 4), np.float32)
    for lin in np.nonzero(g.indirection >= 0)[0]:
        bid = g.indirection[lin]
        bz, by, bx = lin // (G * G), (lin // G) % G, lin % G
        sl = (slice(bz * B, bz * B + B), slice(by * B, by * B + B), slice(bx * B, bx * B + B))
        sigma[sl] = (g.dens[bid] * (50.0 / 255.0)).astype(np.float32)
        rgb[sl] = (g.rgb[bid] / 255.0).astype(np.float32)
        feat[sl] = (g.feat[bid] / 255.0).astype(np.float32)
    cams = W.sphere_cameras([(24, 24, 60.0)] * 8, seed=2)
    c = K.cull(sigma, B, cams, tau_vis=1e-30)
    occ = g.indirection >= 0
    assert np.all(c.vis[occ] > 0)
    np.testing.assert_array_equal(c.keep, occ & (K.block_max(sigma.astype(np.float64), B) >= -N * math.log(0.995)))
    d8, r8, f8 = K.pack_atlas(sigma, rgb, feat, B, c.indirection, 50.0)
    for lin in np.nonzero(c.keep)[0]:
        np.testing.assert_array_equal(d8[c.indirection[lin]], g.dens[g.indirection[lin]])
        np.testing.assert_array_equal(r8[c.indirection[lin]], g.rgb[g.indirection[lin]])
        np.testing.assert_array_equal(f8[c.indirection[lin]], g.feat[g.indirection[lin]])
