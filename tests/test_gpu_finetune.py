"""GPU fine-tuning of the deferred network (Section 5.5) against the FP64
reference in oracle/train.py: the squared-error kernel, the Adam kernel,
the MLP-only backward on the uint8 grid, and a multi-step trajectory."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from oracle import train as T
from paper_2103_14645_amd import finetune as F
from paper_2103_14645_amd import snerg as S
from tests.gpu_helpers import device_grid, handle, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,with_ids", [(1, False), (257, True), (4096, False), (0, False)])
def test_mse_kernel(n, with_ids):
    say(f"mse n={n} ids={with_ids}")
    rng = np.random.default_rng(n)
    rgba = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    rows = 3 * n + 5
    tgt = rng.uniform(0, 1, (rows, 4)).astype(np.float32)
    ids = rng.choice(rows, n, replace=False) if with_ids else np.arange(n)
    g = torch.full((max(n, 1), 4), 9.0, device="cuda")
    loss = torch.full((1,), 7.0, device="cuda")
    S.snerg_loss_mse(handle(), torch.from_numpy(rgba).cuda(), torch.from_numpy(tgt).cuda(), n, g, loss,
                     target_ids=torch.from_numpy(ids.astype(np.int64)).cuda() if with_ids else None)
    torch.cuda.synchronize()
    ref_loss, ref_g = T.mse(rgba, tgt[ids])
    assert float(loss.item()) == pytest.approx(ref_loss, rel=1e-5, abs=1e-12)
    if n:
        assert np.abs(g.cpu().numpy()[:n] - ref_g).max() <= 1e-6 * max(1.0, np.abs(ref_g).max())


def test_adam_kernel_five_steps():
    say("adam: five steps on 10,001 parameters")
    rng = np.random.default_rng(1)
    n = 10001
    p0 = rng.normal(size=n).astype(np.float32)
    p = torch.from_numpy(p0.copy()).cuda()
    m, v = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    opt = T.Adam(n, lr=1e-2)
    ref = p0.astype(np.float64)
    for t in range(1, 6):
        g = (rng.normal(size=n) * np.where(rng.uniform(size=n) < 0.1, 0.0, 1.0)).astype(np.float32)
        S.snerg_adam_step(handle(), p, torch.from_numpy(g).cuda(), m, v, n, 1e-2, t)
        ref = opt.step(ref, g)
    torch.cuda.synchronize()
    assert np.abs(p.cpu().numpy() - ref).max() <= 1e-5


def _case(seed=4):
    g = W.tiny_grid(n_occupied=96, seed=seed)
    cams = [W.orbit_camera(40, 32, seed=seed + 1), W.orbit_camera(24, 36, seed=seed + 2)]
    mlp = W.mlp_weights(seed + 2)
    start, _ = W.perturbed(mlp, g, seed=seed + 3, rel=0.3)
    return g, cams, mlp, start


@pytest.mark.parametrize("fp16", [False, True])
def test_mlp_only_backward_on_uint8_grid(fp16):
    say(f"mlp-only backward, uint8 grid, fp16={fp16}")
    g, cams, mlp, start = _case()
    n = sum(c.n_rays for c in cams)
    dg = device_grid(g)
    ids = np.sort(np.random.default_rng(0).choice(n, n // 2, replace=False))
    idt = torch.from_numpy(ids).cuda()
    m = S.mlp_tensor(start)
    out = torch.empty((len(ids), 4), device="cuda")
    aux = torch.empty((len(ids), 8), device="cuda")
    S.snerg_render(handle(), dg.struct(), m, S.make_cameras(cams), idt, len(ids), S.make_opts(fp16=fp16), out, aux)
    grng = np.random.default_rng(2)
    g_rgba = (grng.normal(size=(len(ids), 4)) / len(ids)).astype(np.float32)
    gm = torch.empty(883, device="cuda")
    S.snerg_render_backward(handle(), dg.struct(), m, S.make_cameras(cams), idt, len(ids),
                            S.make_opts(fp16=fp16, mlp_grad_only=True), aux, torch.from_numpy(g_rgba).cuda(),
                            gm, None, None, None)
    torch.cuda.synchronize()
    og = O.OracleGrid(g, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (g.dens, g.rgb, g.feat)))
    ref = O.render_grad(og, start, cams, g_rgba.astype(np.float64), ray_ids=ids)[0]
    err = np.abs(gm.cpu().numpy() - ref).max()
    scale = np.abs(ref).max()
    say(f"  max|ref|={scale:.3e} max_err={err:.3e}")
    assert err <= (5e-2 if fp16 else 1e-4) * scale + 1e-7


def test_finetuning_trajectory_matches_oracle():
    say("fine-tuning: 6 Adam steps on 256-ray minibatches vs the FP64 reference")
    g, cams, mlp, start = _case()
    n = sum(c.n_rays for c in cams)
    og = O.OracleGrid(g, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (g.dens, g.rgb, g.feat)))
    target = O.render(og, mlp, cams)["rgba"]
    rng = np.random.default_rng(3)
    batches = [np.sort(rng.choice(n, 256, replace=False)) for _ in range(6)]
    lr = 1e-3
    ref_w, ref_loss = T.finetune(g, start.flat(), cams, target, batches, lr=lr)
    dg = device_grid(g)
    w = S.mlp_tensor(start)
    ft = F.MlpFineTuner(handle(), dg.struct(), w, cams, torch.from_numpy(target.astype(np.float32)).cuda(), lr=lr,
                        max_batch=256)
    for k, b in enumerate(batches):
        loss = float(ft.step(torch.from_numpy(b).cuda()).item())
        err = np.abs(w.cpu().numpy() - ref_w[k]).max()
        say(f"  step {k}: loss {loss:.6f} (oracle {ref_loss[k]:.6f}), max weight diff {err:.2e}")
        assert loss == pytest.approx(ref_loss[k], rel=1e-4, abs=1e-9)
        # each Adam step moves a weight by at most ~lr; FP32 gradients may flip
        # only near-zero components, bounded by a fraction of one step
        assert err <= 0.05 * lr * (k + 1)


def test_finetuning_lowers_the_loss_on_the_gpu():
    say("fine-tuning: two epochs of 512-ray minibatches lower the loss")
    g, cams, mlp, start = _case(seed=9)
    og = O.OracleGrid(g, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (g.dens, g.rgb, g.feat)))
    target = torch.from_numpy(O.render(og, mlp, cams)["rgba"].astype(np.float32)).cuda()
    dg = device_grid(g)
    w = S.mlp_tensor(start)
    ft = F.MlpFineTuner(handle(), dg.struct(), w, cams, target, lr=3e-3, max_batch=512)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    losses = []
    for _ in range(6):
        losses += [float(x.item()) for x in ft.epoch(512, gen)]
    say(f"  first {np.mean(losses[:3]):.5f} last {np.mean(losses[-3:]):.5f} over {len(losses)} steps")
    assert np.mean(losses[-3:]) < 0.7 * np.mean(losses[:3])


def test_finetuning_with_patch_minibatches_lowers_the_loss():
    say("fine-tuning: six epochs of 512-ray minibatches of whole 8x8 patches")
    g, cams, mlp, start = _case(seed=9)
    og = O.OracleGrid(g, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (g.dens, g.rgb, g.feat)))
    target = torch.from_numpy(O.render(og, mlp, cams)["rgba"].astype(np.float32)).cuda()
    dg = device_grid(g)
    w = S.mlp_tensor(start)
    ft = F.MlpFineTuner(handle(), dg.struct(), w, cams, target, lr=3e-3, max_batch=512)
    gen = torch.Generator()
    gen.manual_seed(3)
    losses = []
    for _ in range(6):
        losses += [float(x.item()) for x in ft.epoch(512, gen, patches=True)]
    say(f"  first {np.mean(losses[:3]):.5f} last {np.mean(losses[-3:]):.5f} over {len(losses)} steps")
    assert np.mean(losses[-3:]) < 0.7 * np.mean(losses[:3])
