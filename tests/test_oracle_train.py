"""Pins of the FP64 fine-tuning reference (Section 5.5; Adam as in Kingma
and Ba, Algorithm 1): closed forms of Adam's first steps, the loss gradient
against central differences, the weight gradient of the squared error
against central differences through the oracle renderer, and a decreasing
loss over a short fine-tuning run."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import train as T


def test_mse_value_and_gradient_by_differences():
    rng = np.random.default_rng(0)
    rgba, tgt = rng.uniform(0, 1, (7, 4)), rng.uniform(0, 1, (7, 4))
    loss, g = T.mse(rgba, tgt)
    assert loss == pytest.approx(((rgba[:, :3] - tgt[:, :3]) ** 2).mean())
    assert np.all(g[:, 3] == 0.0)
    h = 1e-6
    for (i, c) in [(0, 0), (3, 2), (6, 1)]:
        p, m = rgba.copy(), rgba.copy()
        p[i, c] += h
        m[i, c] -= h
        fd = (T.mse(p, tgt)[0] - T.mse(m, tgt)[0]) / (2 * h)
        assert g[i, c] == pytest.approx(fd, rel=1e-6)
    assert T.mse(np.zeros((0, 4)), np.zeros((0, 4)))[0] == 0.0


def test_adam_first_step_and_constant_gradient_closed_forms():
    # after t steps of a constant gradient g: m_hat = g and v_hat = g^2
    # exactly, so every step moves theta by -lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    opt = T.Adam(4, lr=1e-2)
    theta = np.zeros(4)
    for t in range(1, 6):
        theta = opt.step(theta, g)
        step = -1e-2 * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(theta, t * step, rtol=1e-12, atol=1e-15)
    assert theta[3] == 0.0  # zero gradient leaves the parameter where it is


def test_adam_minimises_a_quadratic():
    # f(x) = 0.5 |x - c|^2 : Adam reaches c to within a few learning rates
    c = np.array([0.7, -0.2, 0.05])
    x = np.zeros(3)
    opt = T.Adam(3, lr=1e-2)
    for _ in range(3000):
        x = opt.step(x, x - c)
    np.testing.assert_allclose(x, c, atol=3e-2)


def _case():
    g = W.tiny_grid(n_occupied=96, seed=4)
    cams = [W.orbit_camera(24, 20, seed=5)]
    mlp = W.mlp_weights(6)
    start, _ = W.perturbed(mlp, g, seed=7, rel=0.3)
    og = O.OracleGrid(g, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (g.dens, g.rgb, g.feat)))
    target = O.render(og, mlp, cams)["rgba"]
    return g, cams, mlp, start, og, target


def test_weight_gradient_of_the_loss_by_differences():
    g, cams, mlp, start, og, target = _case()
    theta = start.flat().astype(np.float64)
    rgba = O.render(og, theta, cams)["rgba"]
    loss, gr = T.mse(rgba, target)
    gm = O.render_grad(og, theta, cams, gr)[0]
    h = 1e-6
    checked = 0
    for j in [0, 5, 40, 300, 545, 560, 600, 820, 870, 880]:
        p, m = theta.copy(), theta.copy()
        p[j] += h
        m[j] -= h
        fd = (T.mse(O.render(og, p, cams)["rgba"], target)[0] - T.mse(O.render(og, m, cams)["rgba"], target)[0]) / (2 * h)
        assert abs(gm[j] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, j
        checked += 1
    assert checked == 10


def test_finetuning_lowers_the_loss():
    g, cams, mlp, start, og, target = _case()
    n = sum(c.n_rays for c in cams)
    rng = np.random.default_rng(3)
    batches = [np.sort(rng.choice(n, 128, replace=False)) for _ in range(40)]
    _, losses = T.finetune(g, start.flat(), cams, target, batches, lr=3e-3)
    assert np.mean(losses[-5:]) < 0.7 * np.mean(losses[:5])
