"""FP64 reference for the fine-tuning of the deferred shading network
(Section 5.5): the squared-error loss against observed pixels and the Adam
update (Kingma and Ba, "Adam: A method for stochastic optimization",
Algorithm 1), run on the oracle's own MLP gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU
baseline, never by the product path.
"""
from __future__ import annotations

import numpy as np

from . import OracleGrid, render, render_grad


def mse(rgba, target):
    """Loss (1 / 3n) sum over rays and RGB of (rgba - target)^2 and its
    gradient with respect to rgba (alpha column zero: the observed images of
    Section 5.5 are RGB)."""
    rgba = np.asarray(rgba, np.float64)
    target = np.asarray(target, np.float64)
    n = rgba.shape[0]
    if n == 0:
        return 0.0, np.zeros((0, 4))
    e = rgba[:, :3] - target[:, :3]
    g = np.zeros((n, 4))
    g[:, :3] = 2.0 * e / (3.0 * n)
    return float((e * e).sum() / (3.0 * n)), g


class Adam:
    """Algorithm 1 of Kingma and Ba, elementwise on a parameter vector:
    g_t; m_t = b1 m + (1 - b1) g; v_t = b2 v + (1 - b2) g^2; bias-corrected
    m_hat = m_t / (1 - b1^t), v_hat = v_t / (1 - b2^t); theta -= lr m_hat /
    (sqrt(v_hat) + eps)."""

    def __init__(self, n, lr=3e-4, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        g = np.asarray(g, np.float64)
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        m_hat = self.m / (1.0 - self.b1 ** self.t)
        v_hat = self.v / (1.0 - self.b2 ** self.t)
        return np.asarray(theta, np.float64) - self.lr * m_hat / (np.sqrt(v_hat) + self.eps)


def finetune(grid, mlp_vec, cams, targets, batches, lr=3e-4, **opts):
    """Section 5.5 on the oracle: for each minibatch of ray ids, render the
    fixed grid with the current weights, take the squared-error gradient
    against targets[ids], back-propagate to the 883 weights and apply one
    Adam step.  Returns (weights after each step, loss of each step)."""
    og = OracleGrid(grid, values=tuple(np.asarray(a, np.float64) / 255.0 for a in (grid.dens, grid.rgb, grid.feat)))
    theta = np.asarray(mlp_vec, np.float64).copy()
    opt = Adam(theta.size, lr=lr)
    weights, losses = [], []
    for ids in batches:
        rgba = render(og, theta, cams, ray_ids=ids, **opts)["rgba"]
        loss, g = mse(rgba, np.asarray(targets)[ids])
        gm = render_grad(og, theta, cams, g, ray_ids=ids, **opts)[0]
        theta = opt.step(theta, gm)
        weights.append(theta.copy())
        losses.append(loss)
    return weights, losses
