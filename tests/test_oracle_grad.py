"""Pins of the oracle's analytic gradient: central finite differences of the
oracle's forward render, and closed forms."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.test_oracle import axis_camera, world_of_voxel_coord


def shadow_of(g, rng=None, jitter=0.0):
    d = g.dens.astype(np.float64) / 255.0
    r = g.rgb.astype(np.float64) / 255.0
    f = g.feat.astype(np.float64) / 255.0
    if rng is not None and jitter:
        nz = d != 0
        d = np.where(nz, d + jitter * rng.uniform(-1, 1, d.shape), 0.0)
        r = r + jitter * rng.uniform(-1, 1, r.shape)
        f = f + jitter * rng.uniform(-1, 1, f.shape)
    return d, r, f


def loss(og, mlp, cams, g_rgba, **kw):
    return float(np.sum(O.render(og, mlp, cams, **kw)["rgba"] * g_rgba))


@pytest.mark.parametrize("early", [False, True])
def test_oracle_gradient_matches_central_differences(early):
    rng = np.random.default_rng(11)
    g = W.tiny_grid(n_occupied=96, seed=4)
    vals = shadow_of(g, rng, 0.01)
    mlp = W.mlp_weights(5)
    cams = [W.orbit_camera(10, 9, seed=6)]
    n = cams[0].n_rays
    g_rgba = rng.normal(size=(n, 4))
    og = O.OracleGrid(g, values=vals)
    gm, gd, gr, gf = O.render_grad(og, mlp, cams, g_rgba, early_stop=early)
    base_cnt = O.render(og, mlp, cams, early_stop=early)["counters"]
    assert np.abs(gd).max() > 0 and np.abs(gm).max() > 0

    def fd(set_value, theta):
        h = 1e-6 * max(1.0, abs(theta))
        l0 = loss(og_p[0], mlp_p[0], cams, g_rgba, early_stop=early)
        set_value(theta + h)
        lp = loss(og_p[0], mlp_p[0], cams, g_rgba, early_stop=early)
        cp = O.render(og_p[0], mlp_p[0], cams, early_stop=early)["counters"]
        set_value(theta - h)
        lm = loss(og_p[0], mlp_p[0], cams, g_rgba, early_stop=early)
        cm = O.render(og_p[0], mlp_p[0], cams, early_stop=early)["counters"]
        set_value(theta)
        if not (np.array_equal(cp, base_cnt) and np.array_equal(cm, base_cnt)):
            return None   # the step flipped a stop decision: not a smooth probe
        fwd, bwd = (lp - l0) / h, (l0 - lm) / h
        if abs(fwd - bwd) > 1e-4 * (abs(fwd) + abs(bwd)) + 1e-6:
            return None   # one-sided slopes differ: the step crosses a ReLU kink
        return (lp - lm) / (2 * h)

    flat = mlp.flat().astype(np.float64)
    mlp_p = [W.MLP.from_flat(flat)]
    og_p = [og]
    checked = 0
    for idx in rng.choice(883, 24, replace=False):
        def set_mlp(v, idx=idx):
            f2 = flat.copy(); f2[idx] = v
            mlp_p[0] = f2            # float64 parameter vector: no float32 rounding of the step
        got = fd(set_mlp, flat[idx])
        if got is None:
            continue
        assert gm[idx] == pytest.approx(got, rel=2e-5, abs=1e-7)
        checked += 1
    mlp_p[0] = mlp
    # grid values touched by composited samples, density only where non-zero
    d, r, f = (a.copy() for a in vals)
    og_p[0] = O.OracleGrid(g, values=(d, r, f))
    for arr, grad, nz_only in ((d, gd, True), (r, gr, False), (f, gf, False)):
        cand = np.flatnonzero((grad != 0) & ((arr != 0) if nz_only else True))
        for idx in rng.choice(cand, min(12, cand.size), replace=False):
            def set_grid(v, arr=arr, idx=idx):
                arr.reshape(-1)[idx] = v
            got = fd(set_grid, arr.reshape(-1)[idx])
            if got is None:
                continue
            assert grad.reshape(-1)[idx] == pytest.approx(got, rel=2e-5, abs=1e-7)
            checked += 1
    assert checked >= 50


def test_gradient_of_alpha_through_constant_slab_closed_form():
    # Same slab as the forward closed form: optical depth tau = 20 sigma delta
    # with sigma = 50 s for every slab voxel value s, so d(alpha)/ds summed
    # over the slab voxels is 20 * 50 * delta * exp(-tau).
    N, B = 64, 8
    dens = np.zeros((N, N, N), np.uint8)
    rgb = np.zeros((N, N, N, 3), np.uint8); feat = np.zeros((N, N, N, 4), np.uint8)
    jy, jz = 29, 35
    dens[jz, jy, 20:30] = 51
    g = W.grid_from_dense(dens, rgb, feat, B, permute_seed=1)
    vals = shadow_of(g)
    og = O.OracleGrid(g, values=vals)
    y = world_of_voxel_coord(jy + 0.5, N); z = world_of_voxel_coord(jz + 0.5, N)
    cam = axis_camera((-2.0, y, z), (1, 0, 0), (0, -1, 0), (0, 0, 1))
    _, gd, _, _ = O.render_grad(og, None, [cam], np.array([[0.0, 0.0, 0.0, 1.0]]), mlp_on=False,
                                early_stop=False)
    s = 51 / 255.0
    delta = 1.0 / N
    tau = 20 * 50.0 * s * delta
    slab = vals[0] != 0            # the zero voxels at x = 19, 30 also get gradient: excluded
    assert gd[slab].sum() == pytest.approx(20 * 50.0 * delta * math.exp(-tau), rel=1e-12)
    # and d(red)/ds through the background term: rgb_red = C_red + T bg_red, C = 0 here
    _, gd2, _, _ = O.render_grad(og, None, [cam], np.array([[1.0, 0.0, 0.0, 0.0]]), mlp_on=False,
                                 early_stop=False, bg=(0.8, 0.0, 0.0))
    assert gd2[slab].sum() == pytest.approx(-0.8 * 20 * 50.0 * delta * math.exp(-tau), rel=1e-12)


def test_mlp_bias_gradient_for_zero_network():
    # With every weight zero the residual is sigmoid(b3) = 1/2 for gated rays,
    # so dL/db3 = sum over gated rays of g * 1/4 and all weight gradients vanish.
    g = W.tiny_grid(n_occupied=96, seed=4)
    og = O.OracleGrid(g, values=shadow_of(g))
    cams = [W.orbit_camera(8, 8, seed=6)]
    rng = np.random.default_rng(0)
    g_rgba = rng.normal(size=(64, 4))
    zero = W.MLP.from_flat(np.zeros(883))
    gm, _, _, _ = O.render_grad(og, zero, cams, g_rgba)
    gate = O.render(og, zero, cams)["aux"][:, 8] != 0
    assert gate.any()
    assert np.allclose(gm[-3:], 0.25 * g_rgba[gate, :3].sum(axis=0), rtol=1e-13)
    assert np.all(gm[:-3] == 0.0)


def test_gcv_override_matches_mlp_backward():
    # Supplying each ray's dL/dC_d, dL/dV computed by an independent NumPy
    # chain must reproduce the grid gradients of the oracle's own MLP backward.
    from tests import fp16_reference as F
    g = W.tiny_grid(n_occupied=96, seed=4)
    og = O.OracleGrid(g, values=shadow_of(g))
    mlp = W.mlp_weights(5)
    cams = [W.orbit_camera(9, 8, seed=6)]
    rng = np.random.default_rng(1)
    g_rgba = rng.normal(size=(72, 4))
    aux = O.render(og, mlp, cams)["aux"]
    dW, gcv = F.mlp_backward_fp16(mlp, aux, F.directions(cams, g.N), g_rgba, round_operands=False)
    gm, gd, gr, gf = O.render_grad(og, mlp, cams, g_rgba)
    _, gd2, gr2, gf2 = O.render_grad(og, mlp, cams, g_rgba, g_cv=gcv)
    assert np.allclose(dW, gm, rtol=1e-10, atol=1e-14)
    for a_, b_ in ((gd, gd2), (gr, gr2), (gf, gf2)):
        assert np.allclose(a_, b_, rtol=1e-10, atol=1e-14)
