"""GPU parity of the render variants against the FP64 oracle: the
nearest-voxel in-block gate of the WebGL renderer (Appendix A) and the
partial un-premultiply of Eq. 9.  Bars as for the plain render: counters
bit-exact, FP32 RGBA within 1e-4, gradients within 1e-4 of their scale."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2103_14645_amd import snerg as S
from tests.gpu_helpers import device_grid, gpu_render, handle, oracle_variants, parity_error, say
from tests.test_gpu_backward import compare, run_backward, shadow_values

pytestmark = pytest.mark.gpu

VARIANTS = [dict(nn_gate=True), dict(unpremultiply=True), dict(nn_gate=True, unpremultiply=True)]


def _case(n_occ, seed):
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    cams = [W.orbit_camera(64, 48, seed=seed + 1), W.orbit_camera(37, 23, seed=seed + 2)]
    return g, cams, W.mlp_weights(seed + 2)


def _oracle(og, mlp, cams, ids=None, **kw):
    return [O.render(og, mlp, cams, ray_ids=ids, t_stop=1e-3 * f, **kw)["rgba"] for f in (1.0, 1 - 1e-5, 1 + 1e-5)]


@pytest.mark.parametrize("kw", VARIANTS)
@pytest.mark.parametrize("n_occ,seed", [(64, 1), (200, 2)])
def test_variant_render_matches_oracle(kw, n_occ, seed):
    say(f"variant {kw} n_occ={n_occ} seed={seed}")
    g, cams, mlp = _case(n_occ, seed)
    dg = device_grid(g)
    flags = S.make_opts(**kw).flags
    og = O.OracleGrid(g)
    for fp16 in (False, True):
        opts = S.make_opts(fp16=fp16, **kw)
        n = sum(c.n_rays for c in cams)
        out = torch.empty((n, 4), device="cuda")
        S.snerg_render(handle(), dg.struct(), S.mlp_tensor(mlp), S.make_cameras(cams), None, n, opts, out)
        torch.cuda.synchronize()
        err, flagged = parity_error(out.cpu().numpy(), _oracle(og, mlp, cams, **kw))
        say(f"  fp16={fp16} flags={flags} max_err={err.max():.3e} near_threshold={flagged}")
        assert err.max() <= (2e-3 if fp16 else 1e-4)


@pytest.mark.parametrize("seed", [1, 5])
def test_nn_gate_counters_bit_exact(seed):
    say(f"nn gate counters seed={seed}")
    g, cams, _ = _case(200, seed)
    dg = device_grid(g)
    for early in (False, True):
        vis, cnt, ctr = S.trace_visits(handle(), dg, cams, opts=S.make_opts(early_stop=early, mlp_on=False, nn_gate=True),
                                       max_visits=64)
        torch.cuda.synchronize()
        og = O.OracleGrid(g)
        octr = O.render(og, None, cams, early_stop=early, mlp_on=False, nn_gate=True)["counters"][:, :5]
        ovis, ocnt = O.trace_visits(og, cams, early_stop=early, max_visits=64, nn_gate=True)
        same = np.ones(len(octr), bool)
        if early:
            alt = [O.render(og, None, cams, early_stop=True, mlp_on=False, nn_gate=True, t_stop=1e-3 * f)["counters"][:, :5]
                   for f in (1 - 1e-5, 1 + 1e-5)]
            same = np.all(octr == alt[0], axis=1) & np.all(octr == alt[1], axis=1)
        ctr, cnt, vis = ctr.cpu().numpy(), cnt.cpu().numpy(), vis.cpu().numpy()
        say(f"  early={early} rays={len(same)} near_threshold={int((~same).sum())}")
        assert np.array_equal(ctr[same], octr[same]) and np.array_equal(cnt[same], ocnt[same])
        assert np.array_equal(vis[same], ovis[same])


def test_nn_gate_backward_matches_oracle_gradient():
    say("nn gate backward vs oracle gradient")
    g = W.tiny_grid(n_occupied=200, seed=2)
    vals = shadow_values(g, 2)
    mlp = W.mlp_weights(3)
    cams = [W.orbit_camera(48, 40, seed=4), W.orbit_camera(21, 35, seed=5)]
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(2)
    g_rgba = rng.normal(size=(n, 4)) / n
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, nn_gate=True)
    og = O.OracleGrid(g, values=vals)
    alt = [O.render(og, mlp, cams, nn_gate=True, t_stop=1e-3 * f)["counters"] for f in (1 - 1e-5, 1 + 1e-5)]
    assert np.array_equal(alt[0], alt[1])
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, nn_gate=True)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)
    assert np.abs(out - O.render(og, mlp, cams, nn_gate=True)["rgba"]).max() <= 1e-4


def test_variants_on_plain512_sampled_rays():
    say("plain512 with both variants: 6000 sampled rays")
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    dg = device_grid(g)
    kw = dict(nn_gate=True, unpremultiply=True)
    frame = gpu_render(dg, mlp, cams, **kw)
    ids = np.sort(np.random.default_rng(8).choice(frame.shape[0], 6000, replace=False))
    err, flagged = parity_error(frame[ids], _oracle(O.OracleGrid(g), mlp, cams, ids=ids, **kw))
    say(f"  max_err={err.max():.3e} near_threshold={flagged}")
    assert err.max() <= 1e-4


@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("n_occ,seed,gate", [(64, 1, False), (200, 2, False), (200, 3, True)])
def test_per_sample_mlp_matches_oracle(fp16, n_occ, seed, gate):
    say(f"per-sample mlp fp16={fp16} n_occ={n_occ} seed={seed} gate={gate}")
    g, cams, mlp = _case(n_occ, seed)
    dg = device_grid(g)
    n = sum(c.n_rays for c in cams)
    opts = S.make_opts(fp16=fp16, per_sample_mlp=True, nn_gate=gate)
    out = torch.empty((n, 4), device="cuda")
    S.snerg_render(handle(), dg.struct(), S.mlp_tensor(mlp), S.make_cameras(cams), None, n, opts, out)
    torch.cuda.synchronize()
    err, flagged = parity_error(out.cpu().numpy(), _oracle(O.OracleGrid(g), mlp, cams, per_sample_mlp=True, nn_gate=gate))
    say(f"  max_err={err.max():.3e} near_threshold={flagged}")
    assert err.max() <= (2e-3 if fp16 else 1e-4)


def test_per_sample_mlp_launch_modes_agree_bitwise():
    g, cams, mlp = _case(200, 2)
    dg = device_grid(g)
    for fp16 in (False, True):
        base = gpu_render(dg, mlp, cams, fp16=fp16, per_sample_mlp=True)
        for kw in (dict(persistent=True), dict(persistent=True, graph=True)):
            say(f"per-sample fp16={fp16} {kw}")
            assert np.array_equal(gpu_render(dg, mlp, cams, fp16=fp16, per_sample_mlp=True, **kw), base)
        ids = np.random.default_rng(0).permutation(base.shape[0])[:1000]
        assert np.array_equal(gpu_render(dg, mlp, cams, ids=ids, fp16=fp16, per_sample_mlp=True), base[ids])


def test_per_sample_mlp_on_plain512_sampled_rays():
    say("plain512, per-sample FP16 network: 4000 sampled rays")
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    frame = gpu_render(device_grid(g), mlp, cams, fp16=True, per_sample_mlp=True)
    ids = np.sort(np.random.default_rng(9).choice(frame.shape[0], 4000, replace=False))
    err, flagged = parity_error(frame[ids], _oracle(O.OracleGrid(g), mlp, cams, ids=ids, per_sample_mlp=True))
    say(f"  max_err={err.max():.3e} near_threshold={flagged}")
    assert err.max() <= 2e-3
