"""The adjoint at full size (the 512^3 fine-tuning workload) against central
finite differences of the FP64 oracle.

Workload: the 512^3 grid (B = 32, 433 occupied macroblocks) as a float32
shadow, 8 views at 800x800, the squared-error loss of Eq. 3 against targets
rendered from the seeded perturbation (features x (1 + 0.05 U[-1, 1]),
weights + 0.05 std N(0, 1)).  A minibatch of 8,192 rays drawn over the 8
views is rendered on the GPU with the per-ray state, its loss gradient
g = dL/dRGBA comes from snerg_loss_mse, and snerg_render_backward gives
dL/dtheta.  For 64 sampled parameters (16 network weights, 16 densities
with rho > 0, 16 colours, 16 features, each with a non-zero gradient) the
FP64 oracle re-renders the minibatch at theta +- h and differentiates
L'(theta) = sum_r g_r . rgba_r(theta), whose gradient is dL/dtheta by the
chain rule (each ray's output is differenced before the sum over rays).
Probes whose step flips a stopping decision or an active sample (the
counters change) or crosses a ReLU kink (the one-sided slopes disagree)
are replaced by others.  Bar: |g_gpu - g_fd| <= 1e-3 |g_fd| +
1e-5 max|g_fd| per probe, the maximum over the probes of the same kind;
colour and feature probes add the rounding the backward's LDS tables are
built to: their fixed point rounds each hand-over of a voxel to within
2^-24 M (M: the wavefront's largest |dL/dC_d|, |dL/dV|, at most the largest
over the minibatch, which the FP64 network backward of the oracle's per-ray
state gives here), and each of the H rays whose output the probe moves
hands the voxel over at most once per sample it takes in the voxel's eight
cells (at half-voxel steps a straight ray's path there is at most 2 sqrt(3)
voxels long: seven samples), allowing 8 H 2^-24 M.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2103_14645_amd import autograd as A
from paper_2103_14645_amd import snerg as S
from tests import fp16_reference as F
from tests.gpu_helpers import handle, say

pytestmark = pytest.mark.gpu

N_RAYS = 8192


def test_adjoint512_gradient_matches_finite_differences():
    cfg = W.config("adjoint512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    n = sum(c.n_rays for c in cams)
    vals32 = tuple(np.ascontiguousarray(a / np.float32(255.0), np.float32) for a in (g.dens, g.rgb, g.feat))
    vals64 = tuple(a.astype(np.float64) for a in vals32)
    og = O.OracleGrid(g, values=vals64)
    flat = mlp.flat().astype(np.float64)
    rng = np.random.default_rng(3)
    ids = np.sort(rng.choice(n, N_RAYS, replace=False))
    # rays whose stopping decision lies within 1e-5 of t_stop could take either branch
    alt = [O.render(og, flat, cams, ray_ids=ids, t_stop=1e-3 * f)["counters"] for f in (1 - 1e-5, 1 + 1e-5)]
    ids = ids[np.all(alt[0] == alt[1], axis=1)]
    m = len(ids)
    say(f"adjoint512 FD: {m} rays of {n}, {g.n_blocks} blocks")

    # GPU: targets from the perturbed copy, forward, loss gradient, backward
    h = handle()
    dens, rgb, feat = (torch.from_numpy(v).cuda() for v in vals32)
    pmlp, pfeat = W.perturbed(mlp, g)
    carr = S.make_cameras(cams)
    idt = torch.from_numpy(ids.astype(np.int64)).cuda()
    opts = S.make_opts()
    rt = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    rt.pack(dens, rgb, torch.from_numpy(pfeat).cuda())
    target = torch.empty((m, 4), device="cuda")
    S.snerg_render(h, rt.struct(), S.mlp_tensor(pmlp), carr, idt, m, opts, target)
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    r.pack(dens, rgb, feat)
    mt = S.mlp_tensor(mlp)
    out = torch.empty((m, 4), device="cuda")
    aux = torch.empty((m, 8), device="cuda")
    S.snerg_render(h, r.struct(), mt, carr, idt, m, opts, out, aux)
    gout = torch.empty((m, 4), device="cuda")
    loss = torch.empty(1, device="cuda")
    S.snerg_loss_mse(h, out, target, m, gout, loss)
    gm = torch.empty(883, device="cuda")
    gd, gr, gf = torch.empty_like(dens), torch.empty_like(rgb), torch.empty_like(feat)
    S.snerg_render_backward(h, r.struct(), mt, carr, idt, m, opts, aux, gout, gm, gd, gr, gf)
    torch.cuda.synchronize()
    g_rgba = gout.cpu().numpy().astype(np.float64)
    grads = [gm.cpu().numpy(), gd.cpu().numpy(), gr.cpu().numpy(), gf.cpu().numpy()]
    say(f"  loss {float(loss.item()):.6e}; max|dL/dW| {np.abs(grads[0]).max():.3e}, "
        f"max|dL/ddens| {np.abs(grads[1]).max():.3e}")

    base = O.render(og, flat, cams, ray_ids=ids)
    base_cnt = base["counters"]
    rgba0 = base["rgba"]
    # largest per-ray |dL/dC_d|, |dL/dV| (FP64 network backward, no rounding)
    _, gcv = F.mlp_backward_fp16(mlp, base["aux"], F.directions_of(cams, g.N, ids), g_rgba, round_operands=False)
    m_cv = float(np.abs(gcv).max())

    def rerender(params):
        res = O.render(og, params, cams, ray_ids=ids)
        return res["rgba"], res["counters"]

    def fd(set_value, theta):
        # Each ray's output is differenced before the sum over rays: summing
        # L' first would leave a rounding noise of about eps |L'| / h in the
        # quotient, as large as the smallest gradients probed here.
        hstep = 1e-6 * max(1.0, abs(theta))
        set_value(theta + hstep)
        rp, cp = rerender(params_now[0])
        set_value(theta - hstep)
        rm, cm = rerender(params_now[0])
        set_value(theta)
        if not (np.array_equal(cp, base_cnt) and np.array_equal(cm, base_cnt)):
            return None  # the step flipped a stop or an active sample
        fwd = float(np.sum((rp - rgba0) * g_rgba)) / hstep
        bwd = float(np.sum((rgba0 - rm) * g_rgba)) / hstep
        if abs(fwd - bwd) > 1e-4 * (abs(fwd) + abs(bwd)) + 1e-12:
            return None  # the step crosses a ReLU kink
        moved = int(np.count_nonzero(np.any(rp != rm, axis=1)))
        return float(np.sum((rp - rm) * g_rgba)) / (2 * hstep), moved

    params_now = [flat]
    checked = []

    def probe(kind, cand, grad, set_value, get_value, want):
        got = 0
        for idx in rng.permutation(cand):
            if got == want:
                break
            v = fd(lambda x, idx=idx: set_value(idx, x), get_value(idx))
            if v is None:
                continue
            q = 8 * v[1] * 2.0 ** -24 * m_cv if kind in ("rgb", "feat") else 0.0
            checked.append((kind, int(idx), float(grad.flat[idx]), v[0], q))
            got += 1
        assert got == want, f"too few smooth probes for {kind}"

    # network weights
    gmv = grads[0]
    cand = np.flatnonzero(np.abs(gmv) > 1e-3 * np.abs(gmv).max())

    def set_w(idx, x):
        f2 = flat.copy()
        f2[idx] = x
        params_now[0] = f2

    probe("mlp", cand, gmv, set_w, lambda idx: flat[idx], 16)
    params_now[0] = flat
    # grid values: densities only where non-zero
    for arr_i, kind, nz in ((0, "dens", True), (1, "rgb", False), (2, "feat", False)):
        arr = og.arrays[arr_i]
        grad = grads[arr_i + 1]
        sel = np.abs(grad.reshape(-1)) > 1e-3 * np.abs(grad).max()
        if nz:
            sel &= arr.reshape(-1) != 0
        cand = np.flatnonzero(sel)

        def set_g(idx, x, arr=arr):
            arr.reshape(-1)[idx] = x

        probe(kind, cand, grad, set_g, lambda idx, arr=arr: float(arr.reshape(-1)[idx]), 16)
    worst = 0.0
    for kind, idx, got, want, q in checked:
        scale = max(abs(c[3]) for c in checked if c[0] == kind)  # the floor is per kind of parameter
        err = abs(got - want)
        bar = 1e-3 * abs(want) + 1e-5 * scale + q
        worst = max(worst, err / bar)
        assert err <= bar, (kind, idx, got, want, q)
    say(f"  {len(checked)} probes, worst error / bar = {worst:.3e}; largest |dL/dC_d|, |dL/dV| {m_cv:.3e}")
