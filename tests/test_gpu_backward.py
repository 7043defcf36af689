"""GPU adjoint against the FP64 oracle's gradient (which is itself pinned to
central differences).  Bar: |g_gpu - g_oracle| <= 1e-4 * max|g_oracle| + 1e-7
per element, for the MLP parameters and every grid value."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2103_14645_amd import autograd as A
from paper_2103_14645_amd import finetune as F
from paper_2103_14645_amd import snerg as S
from tests.gpu_helpers import handle, say

pytestmark = pytest.mark.gpu


def shadow_values(g, seed):
    rng = np.random.default_rng(seed)
    d = g.dens / 255.0
    return (np.where(d > 0, d + 0.01 * rng.uniform(-1, 1, d.shape), 0.0).astype(np.float32),
            (g.rgb / 255.0 + 0.01 * rng.uniform(-1, 1, g.rgb.shape)).astype(np.float32),
            (g.feat / 255.0 + 0.01 * rng.uniform(-1, 1, g.feat.shape)).astype(np.float32))


def run_backward(g, vals, mlp, cams, g_rgba, ids=None, **kw):
    h = handle()
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals)
    m = S.mlp_tensor(mlp)
    cams_c = S.make_cameras(cams)
    opts = S.make_opts(**kw)
    idt = torch.from_numpy(np.asarray(ids, np.int64)).cuda() if ids is not None else None
    dens.requires_grad_(True); rgb.requires_grad_(True); feat.requires_grad_(True); m.requires_grad_(True)
    out = A.render_shadow(r, dens, rgb, feat, m, cams_c, idt, opts)
    out.backward(torch.from_numpy(g_rgba.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return (m.grad.cpu().numpy().astype(np.float64), dens.grad.cpu().numpy(), rgb.grad.cpu().numpy(),
            feat.grad.cpu().numpy(), out.detach().cpu().numpy())


def stable_ids(og, mlp, cams, ids):
    """Drop rays whose early-stop decision lies within a relative 1e-5 of
    t_stop (either branch would be a correct render, with another gradient)."""
    alt = [O.render(og, mlp, cams, ray_ids=ids, t_stop=1e-3 * f)["counters"] for f in (1 - 1e-5, 1 + 1e-5)]
    keep = np.all(alt[0] == alt[1], axis=1)
    say(f"  dropped {int((~keep).sum())} near-threshold rays of {len(ids)}")
    return ids[keep]


def compare(name, gpu, ref, rel=1e-4):
    scale = float(np.abs(ref).max())
    err = float(np.abs(gpu - ref).max())
    say(f"  {name}: max|ref|={scale:.3e} max_err={err:.3e}")
    assert err <= rel * scale + 1e-7, name


@pytest.mark.parametrize("n_occ,seed,early,mlp_on,subset", [(96, 4, False, True, False), (200, 2, True, True, False),
                                                           (120, 5, True, False, False), (200, 7, True, True, True)])
def test_backward_matches_oracle_gradient(n_occ, seed, early, mlp_on, subset):
    say(f"backward n_occ={n_occ} seed={seed} early={early} mlp={mlp_on} subset={subset}")
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(48, 40, seed=seed + 2), W.orbit_camera(21, 35, seed=seed + 3)]
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(n, n // 2, replace=False)) if subset else None
    m = len(ids) if subset else n
    g_rgba = rng.normal(size=(m, 4)) / m
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, early_stop=early, mlp_on=mlp_on)
    og = O.OracleGrid(g, values=vals)
    # near-threshold stops could pick a different branch: require none here
    alt = [O.render(og, mlp, cams, ray_ids=ids, early_stop=early, mlp_on=mlp_on, t_stop=1e-3 * f)["counters"]
           for f in (1 - 1e-5, 1 + 1e-5)]
    assert np.array_equal(alt[0], alt[1])
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids, early_stop=early, mlp_on=mlp_on)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)
    ref = O.render(og, mlp, cams, ray_ids=ids, early_stop=early, mlp_on=mlp_on)["rgba"]
    assert np.abs(out - ref).max() <= 1e-4


@pytest.mark.parametrize("layout,patch", [("patches", True), ("scattered", True), ("scattered", False),
                                          ("patches", False)])
def test_patch_ray_lists_match_oracle_gradient(layout, patch):
    # ray lists with SNERG_FLAG_PATCH_RAYS (gradients summed per wavefront in
    # LDS) or without (an LDS log): exact up to summation order for any list,
    # patch-shaped (as the fine-tuning patch sampler draws them, ragged
    # patches included) or not
    say(f"backward of a {layout} list, SNERG_FLAG_PATCH_RAYS={patch}")
    seed = 8
    g = W.tiny_grid(n_occupied=200, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(48, 40, seed=seed + 2), W.orbit_camera(21, 35, seed=seed + 3)]
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(seed)
    if layout == "patches":
        class _C:
            cam_list, mlp = cams, torch.zeros(1)
        gen = torch.Generator()
        gen.manual_seed(seed)
        ids = F.MlpFineTuner.patch_order(_C(), gen).numpy()[: n // 2]
    else:
        ids = rng.permutation(n)[: n // 2]
    og = O.OracleGrid(g, values=vals)
    ids = stable_ids(og, mlp, cams, ids)
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, patch_rays=patch)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)


@pytest.mark.parametrize("patch", [False, True])
def test_long_rays_past_the_sample_list(patch):
    # A ray list's backward lists up to 512 samples per ray before its
    # gradient pass; longer rays walk on from their start past the listed
    # ones.  Rays along a fully occupied column of 16 macroblocks (512
    # voxels, about 1,024 samples each) take that path; the whole frame and a
    # list of its rays against the oracle, early stop off.
    N, B = 512, 32
    G = N // B
    ind = np.full(G ** 3, -1, np.int32)
    for bx in range(G):
        ind[(8 * G + 8) * G + bx] = bx
    rng = np.random.default_rng(12)
    dens = rng.integers(3, 9, (G, B, B, B), dtype=np.uint8)  # nowhere zero (also after the shadow's +-0.01)
    rgb = rng.integers(0, 256, (G, B, B, B, 3), dtype=np.uint8)
    feat = rng.integers(0, 256, (G, B, B, B, 4), dtype=np.uint8)
    g = W.Grid(N, B, ind, dens, rgb, feat)
    fwd, up = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    y, z = (8 * B + 16.25) * 2.0 / N - 1.0, (8 * B + 15.75) * 2.0 / N - 1.0
    cams = [W.Camera(np.array([-2.5, y, z]), fwd, np.cross(fwd, up), up, 12, 10, 3000.0)]
    vals = shadow_values(g, 12)
    mlp = W.mlp_weights(13)
    og = O.OracleGrid(g, values=vals)
    n = cams[0].n_rays
    cnt = O.render(og, mlp, cams, early_stop=False)["counters"]
    say(f"long rays: composited samples per ray {int(cnt[:, 3].min())}..{int(cnt[:, 3].max())}")
    assert cnt[:, 3].min() > 600  # every ray overflows the 512-sample list
    ids = np.random.default_rng(3).permutation(n)[: n - 7]
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    gm, gd, gr, gf, _ = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, early_stop=False, patch_rays=patch)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids, early_stop=False)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)


@pytest.mark.parametrize("patch", [False, True])
def test_long_ray_list_single_remarch(patch):
    # Lists longer than 2^18 rays take the single re-march (one lane per
    # ray, gradients summed in the LDS table), not the two phases.
    seed = 14
    g = W.tiny_grid(n_occupied=120, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(640, 480, seed=seed + 2)]
    n = cams[0].n_rays
    rng = np.random.default_rng(seed)
    og = O.OracleGrid(g, values=vals)
    ids = stable_ids(og, mlp, cams, rng.permutation(n)[: (1 << 18) + 4097])
    assert len(ids) > (1 << 18)
    say(f"backward of a {len(ids)}-ray list, SNERG_FLAG_PATCH_RAYS={patch}")
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    gm, gd, gr, gf, _ = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, patch_rays=patch)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)


@pytest.mark.parametrize("patch", [False, True])
def test_small_and_empty_ray_lists(patch):
    # A one-ray list, a list of rays that miss the grid or composite nothing
    # (their gradients are zero), a ragged 65-ray list, and a zero-ray call
    # (it clears the outputs, or leaves them with SNERG_FLAG_ACCUMULATE).
    seed = 15
    g = W.tiny_grid(n_occupied=64, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(32, 24, seed=seed + 2)]
    og = O.OracleGrid(g, values=vals)
    base = O.render(og, mlp, cams)
    composited = base["counters"][:, 3]
    hit = np.flatnonzero(composited > 0)
    miss = np.flatnonzero(composited == 0)
    assert len(hit) > 65 and len(miss) > 8
    rng = np.random.default_rng(seed)
    for name, ids in (("one ray", hit[:1]), ("nothing composited", miss[:40]),
                      ("65 rays", rng.permutation(hit)[:65])):
        ids = stable_ids(og, mlp, cams, np.asarray(ids))
        say(f"  list of {len(ids)} rays ({name}), SNERG_FLAG_PATCH_RAYS={patch}")
        g_rgba = rng.normal(size=(len(ids), 4)) / max(len(ids), 1)
        gm, gd, gr, gf, _ = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, patch_rays=patch)
        om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
        if name == "nothing composited":
            assert not (gd.any() or gr.any() or gf.any())
        compare("mlp", gm, om)
        compare("dens", gd, od)
        compare("rgb", gr, orr)
        compare("feat", gf, of)
    # zero rays
    h = handle()
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals)
    r.pack(dens, rgb, feat)
    carr = S.make_cameras(cams)
    idt = torch.zeros(1, dtype=torch.int64, device="cuda")
    empty4 = torch.zeros((1, 4), device="cuda")
    aux = torch.zeros((1, 8), device="cuda")
    for acc in (False, True):
        gm = torch.full((883,), 7.0, device="cuda")
        gd, gr, gf = (torch.full_like(x, 7.0) for x in (dens, rgb, feat))
        S.snerg_render_backward(h, r.struct(), S.mlp_tensor(mlp), carr, idt, 0,
                                S.make_opts(accumulate=acc, patch_rays=patch), aux, empty4, gm, gd, gr, gf)
        torch.cuda.synchronize()
        want = 7.0 if acc else 0.0
        assert all(bool((x == want).all()) for x in (gm, gd, gr, gf)), acc


def test_mse_step_reduces_loss():
    say("autograd: one SGD step on an MSE against perturbed targets lowers the loss")
    g = W.tiny_grid(n_occupied=96, seed=4)
    vals = shadow_values(g, 4)
    mlp = W.mlp_weights(5)
    cams = [W.orbit_camera(32, 32, seed=6)]
    target_mlp, _ = W.perturbed(mlp, g, seed=3)
    h = handle()
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals)
    cams_c = S.make_cameras(cams)
    with torch.no_grad():
        target = A.render_shadow(r, dens, rgb, feat, S.mlp_tensor(target_mlp), cams_c)
    m = S.mlp_tensor(mlp).requires_grad_(True)
    losses = []
    for _ in range(3):
        out = A.render_shadow(r, dens, rgb, feat, m, cams_c)
        loss = ((out[:, :3] - target[:, :3]) ** 2).mean()
        losses.append(float(loss))
        m.grad = None
        loss.backward()
        with torch.no_grad():
            m -= 0.5 * m.grad / (m.grad.norm() + 1e-12) * 0.05
    say(f"  losses {losses}")
    assert losses[-1] < losses[0]


def test_fp16_mlp_backward_matches_oracle_gradient():
    # Two bars.  Tight: against the same arithmetic with FP16 operands
    # emulated in NumPy on the oracle's per-ray state (tests/fp16_reference.py),
    # grid gradients from the FP64 oracle march fed the emulated dL/dC_d,
    # dL/dV; the remaining differences are FP32 versus FP64 sums.  Loose:
    # against the exact FP64 gradient; FP16 operand rounding (u = 2^-11) in a
    # ReLU chain with cancelling sums measures about 2% of max|g| here.
    from tests import fp16_reference as F
    say("fp16 mlp backward vs FP16-emulated and exact oracle gradients")
    seed = 2
    g = W.tiny_grid(n_occupied=200, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(48, 40, seed=seed + 2), W.orbit_camera(21, 35, seed=seed + 3)]
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(seed)
    g_rgba = rng.normal(size=(n, 4)) / n
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, fp16=True)
    og = O.OracleGrid(g, values=vals)
    aux = O.render(og, mlp, cams)["aux"]
    dW16, gcv16 = F.mlp_backward_fp16(mlp, aux, F.directions(cams, g.N), g_rgba)
    _, ed, er, ef = O.render_grad(og, mlp, cams, g_rgba, g_cv=gcv16)
    compare("mlp vs fp16 emulation", gm, dW16, rel=1e-3)
    compare("dens vs fp16 emulation", gd, ed, rel=1e-3)
    compare("rgb vs fp16 emulation", gr, er, rel=1e-3)
    compare("feat vs fp16 emulation", gf, ef, rel=1e-3)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba)
    for name, a_, b_ in (("mlp", gm, om), ("dens", gd, od), ("rgb", gr, orr), ("feat", gf, of)):
        compare(name + " vs exact", a_, b_, rel=5e-2)
    ref = O.render(og, mlp, cams)["rgba"]
    assert np.abs(out - ref).max() <= 2e-3


def test_adjoint512_minibatch_full_size():
    # The 512^3 adjoint grid at full size: a random minibatch of rays over 8
    # 800x800 views, every grid value's gradient against the oracle's.
    cfg = W.config("adjoint512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    n = sum(c.n_rays for c in cams)
    vals = (g.dens / np.float32(255.0), g.rgb / np.float32(255.0), g.feat / np.float32(255.0))
    vals = tuple(np.ascontiguousarray(v, np.float32) for v in vals)
    og = O.OracleGrid(g, values=vals)
    ids = stable_ids(og, mlp, cams, np.sort(np.random.default_rng(3).choice(n, 4096, replace=False)))
    rng = np.random.default_rng(5)
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    say(f"adjoint512 minibatch: {len(ids)} rays of {n}, {g.n_blocks} blocks")
    gm, gd, gr, gf, _ = run_backward(g, vals, mlp, cams, g_rgba, ids=ids)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)


def test_large1024_fp16_minibatch_full_size():
    # The 1024^3 (8% occupied) grid with the FP16 MLP forward and backward on a
    # random minibatch over the 64 1080p views, against the FP16 emulation
    # (tight) and the exact gradient (loose), as in the 64^3 FP16 test.
    from tests import fp16_reference as F
    cfg = W.config("large1024")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    n = sum(c.n_rays for c in cams)
    vals = tuple(np.ascontiguousarray(v / np.float32(255.0), np.float32) for v in (g.dens, g.rgb, g.feat))
    og = O.OracleGrid(g, values=vals)
    ids = stable_ids(og, mlp, cams, np.sort(np.random.default_rng(3).choice(n, 2048, replace=False)))
    rng = np.random.default_rng(6)
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    say(f"large1024 fp16 minibatch: {len(ids)} rays of {n}, {g.n_blocks} blocks")
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, ids=ids, fp16=True)
    orc = O.render(og, mlp, cams, ray_ids=ids)
    dirs = F.directions_of(cams, g.N, ids)
    dW16, gcv16 = F.mlp_backward_fp16(mlp, orc["aux"], dirs, g_rgba)
    _, ed, er, ef = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids, g_cv=gcv16)
    compare("mlp vs fp16 emulation", gm, dW16, rel=1e-3)
    compare("dens vs fp16 emulation", gd, ed, rel=1e-3)
    compare("rgb vs fp16 emulation", gr, er, rel=1e-3)
    compare("feat vs fp16 emulation", gf, ef, rel=1e-3)
    # and against the exact FP64 gradient.  The bar is the one the FP16
    # arithmetic itself sets: 5% of max|g| (half-precision operands three
    # layers deep, about 2% on the 64^3 case), or 1.5 times the distance of
    # the FP16 emulation from the exact gradient where that is larger (the
    # feature gradient reaches the grid only through the network's input
    # gradient, a sum over 16 hidden units whose terms cancel, so the FP16
    # operand rounding is a larger share of it); and the forward at the FP16
    # render bar
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    _, ed16, er16, ef16 = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids, g_cv=gcv16)
    for name, a_, b_, e_ in (("mlp", gm, om, dW16), ("dens", gd, od, ed16), ("rgb", gr, orr, er16),
                             ("feat", gf, of, ef16)):
        scale = float(np.abs(b_).max())
        fp16_own = float(np.abs(e_ - b_).max())
        err = float(np.abs(a_ - b_).max())
        bar = max(5e-2 * scale, 1.5 * fp16_own) + 1e-7
        say(f"  {name} vs exact: max|ref|={scale:.3e} max_err={err:.3e} fp16 emulation's own {fp16_own:.3e}")
        assert err <= bar, name
    assert np.abs(out - orc["rgba"]).max() <= 2e-3


@pytest.mark.parametrize("patch", [False, True])
def test_accumulate_flag_adds_minibatch_gradients(patch):
    # SNERG_FLAG_ACCUMULATE: two minibatches added into the same arrays give
    # the sum of the two overwriting calls (up to float summation order), and
    # the sum matches the oracle's gradient of both minibatches together
    say(f"backward with SNERG_FLAG_ACCUMULATE, patch lists={patch}")
    seed = 9
    g = W.tiny_grid(n_occupied=160, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(40, 32, seed=seed + 2)]
    n = cams[0].n_rays
    og = O.OracleGrid(g, values=vals)
    ids = stable_ids(og, mlp, cams, np.random.default_rng(seed).permutation(n)[: (n // 128) * 128])
    ids = ids[: (len(ids) // 128) * 128]
    halves = (ids[: len(ids) // 2], ids[len(ids) // 2:])
    rng = np.random.default_rng(seed + 5)
    g_rgba = rng.normal(size=(len(ids), 4)) / len(ids)
    h = handle()
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals)
    r.pack(dens, rgb, feat)
    m = S.mlp_tensor(mlp)
    carr = S.make_cameras(cams)
    outs = {}
    for acc in (False, True):
        gm = torch.zeros(883, device="cuda")
        gd, gr, gf = torch.zeros_like(dens), torch.zeros_like(rgb), torch.zeros_like(feat)
        total = [np.zeros(883), np.zeros(vals[0].shape), np.zeros(vals[1].shape), np.zeros(vals[2].shape)]
        for k, part in enumerate(halves):
            idt = torch.from_numpy(part.astype(np.int64)).cuda()
            gpart = torch.from_numpy(g_rgba[k * len(halves[0]):(k + 1) * len(halves[0])].astype(np.float32)).cuda()
            opts = S.make_opts(accumulate=acc, patch_rays=patch)
            out = torch.empty((len(part), 4), device="cuda")
            aux = torch.empty((len(part), 8), device="cuda")
            S.snerg_render(h, r.struct(), m, carr, idt, len(part), opts, out, aux)
            S.snerg_render_backward(h, r.struct(), m, carr, idt, len(part), opts, aux, gpart, gm, gd, gr, gf)
            torch.cuda.synchronize()
            if not acc:
                for t_, x in zip(total, (gm, gd, gr, gf)):
                    t_ += x.cpu().numpy()
        outs[acc] = total if not acc else [x.cpu().numpy().astype(np.float64) for x in (gm, gd, gr, gf)]
    ref = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    for name, a_, b_, o_ in zip(("mlp", "dens", "rgb", "feat"), outs[True], outs[False], ref):
        compare(name + " accumulated vs summed", a_, b_)
        compare(name + " accumulated vs oracle", a_, o_)


@pytest.mark.parametrize("layout,patch,mlp_on", [("views", False, True), ("scattered", False, True),
                                                 ("patches", True, True), ("scattered", False, False)])
def test_packed_grid_gradients(layout, patch, mlp_on):
    # SNERG_FLAG_GRAD_PACKED: the grid gradients as one [voxel][8] array
    # (density, RGB, features 0..3) hold the oracle's gradient as the three
    # separate arrays do; a second, accumulating call over the same rays
    # doubles them.  Whole views (summing table), scattered lists (log),
    # patch lists (table), and no view network (four channels handed over).
    say(f"packed grid gradients: {layout}, SNERG_FLAG_PATCH_RAYS={patch}, mlp_on={mlp_on}")
    seed = 10
    g = W.tiny_grid(n_occupied=180, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(48, 40, seed=seed + 2), W.orbit_camera(24, 32, seed=seed + 3)]
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(seed)
    og = O.OracleGrid(g, values=vals)
    if layout == "views":
        ids = None
        alt = [O.render(og, mlp, cams, mlp_on=mlp_on, t_stop=1e-3 * f)["counters"] for f in (1 - 1e-5, 1 + 1e-5)]
        assert np.array_equal(alt[0], alt[1])
        m = n
    else:
        if layout == "patches":
            class _C:
                cam_list, mlp = cams, torch.zeros(1)
            gen = torch.Generator()
            gen.manual_seed(seed)
            ids = F.MlpFineTuner.patch_order(_C(), gen).numpy()[: n // 2]
        else:
            ids = rng.permutation(n)[: n // 2]
        ids = stable_ids(og, mlp, cams, ids)
        m = len(ids)
    g_rgba = rng.normal(size=(m, 4)) / m
    h = handle()
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals)
    r.pack(dens, rgb, feat)
    mt = S.mlp_tensor(mlp)
    carr = S.make_cameras(cams)
    idt = torch.from_numpy(ids.astype(np.int64)).cuda() if ids is not None else None
    opts = S.make_opts(patch_rays=patch, mlp_on=mlp_on, grad_packed=True)
    out = torch.empty((m, 4), device="cuda")
    aux = torch.empty((m, 8), device="cuda")
    S.snerg_render(h, r.struct(), mt, carr, idt, m, opts, out, aux)
    gout = torch.from_numpy(g_rgba.astype(np.float32)).cuda()
    nv = dens.numel()
    gm = torch.empty(883, device="cuda")
    gp = torch.full((nv, 8), float("nan"), device="cuda")  # overwritten (cleared) by the call
    S.snerg_render_backward(h, r.struct(), mt, carr, idt, m, opts, aux, gout, gm, gp, None, None)
    torch.cuda.synchronize()
    once = gp.cpu().numpy().astype(np.float64)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids, mlp_on=mlp_on)
    compare("mlp", gm.cpu().numpy().astype(np.float64), om)
    compare("dens", once[:, 0], od.reshape(-1))
    compare("rgb", once[:, 1:4], orr.reshape(-1, 3))
    compare("feat", once[:, 4:], of.reshape(-1, 4))
    acc = S.make_opts(patch_rays=patch, mlp_on=mlp_on, grad_packed=True, accumulate=True)
    S.snerg_render_backward(h, r.struct(), mt, carr, idt, m, acc, aux, gout, gm, gp, None, None)
    torch.cuda.synchronize()
    compare("accumulated twice", gp.cpu().numpy().astype(np.float64), 2 * once)


@pytest.mark.parametrize("n_list", [32768, 65536, 65537 + 4000])
def test_scattered_lists_either_side_of_the_wavefront_split(n_list):
    # Scattered lists run the list gradient pass (and the ray-list render)
    # with 16 rays per wavefront up to 2^15 rays, 32 up to 2^16 and 64
    # above: gradients and the rendered colours against the oracle.
    say(f"scattered list of {n_list} rays")
    seed = 16
    g = W.tiny_grid(n_occupied=120, seed=seed)
    vals = shadow_values(g, seed)
    mlp = W.mlp_weights(seed + 1)
    cams = [W.orbit_camera(320, 240, seed=seed + 2)]
    og = O.OracleGrid(g, values=vals)
    rng = np.random.default_rng(seed)
    ids = stable_ids(og, mlp, cams, rng.permutation(cams[0].n_rays)[:n_list + 64])[:n_list]
    assert len(ids) == n_list
    g_rgba = rng.normal(size=(n_list, 4)) / n_list
    gm, gd, gr, gf, out = run_backward(g, vals, mlp, cams, g_rgba, ids=ids)
    om, od, orr, of = O.render_grad(og, mlp, cams, g_rgba, ray_ids=ids)
    compare("mlp", gm, om)
    compare("dens", gd, od)
    compare("rgb", gr, orr)
    compare("feat", gf, of)
    assert np.abs(out - O.render(og, mlp, cams, ray_ids=ids)["rgba"]).max() <= 1e-4
