"""Reference for the FP16-MFMA MLP backward: the same arithmetic as the FP64
MLP chain but with every matrix-product operand rounded to IEEE half
precision at the points where the kernel feeds its MFMA tiles (layer
inputs, weights, and the back-propagated gradients), products and sums
kept wide.  Inputs come from the oracle (per-ray C_d, V, gate and the ray
direction); nothing here comes from the GPU path.

Returns the 883 weight gradients and each ray's dL/dC_d, dL/dV (the rows
that the oracle's gradient routine accepts as `g_cv`)."""
from __future__ import annotations

import numpy as np

import oracle as O


def _h(a):
    return np.asarray(a, np.float16).astype(np.float64)


def directions(cams, N):
    return np.array([O.ray_setup(c, N, i, j)[2] for c in cams for j in range(c.H) for i in range(c.W)])


def directions_of(cams, N, ray_ids):
    """Directions of the given global ray ids (cameras in order, rows from the top)."""
    offs = np.cumsum([0] + [c.W * c.H for c in cams])
    out = []
    for r in ray_ids:
        ci = int(np.searchsorted(offs, r, side="right") - 1)
        local = int(r - offs[ci])
        out.append(O.ray_setup(cams[ci], N, local % cams[ci].W, local // cams[ci].W)[2])
    return np.array(out)


def mlp_backward_fp16(mlp, aux, dirs, g_rgba, round_operands=True):
    """aux: oracle aux rows [n, 9] (C_d, V, T, gate); dirs [n, 3]; g_rgba [n, 4]."""
    q = _h if round_operands else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in mlp.params())
    gate = aux[:, 8] != 0
    X = np.stack([O.encode(aux[k, :3], aux[k, 3:7], dirs[k]) for k in range(aux.shape[0])])
    h1p = q(X) @ q(W1).T + b1
    h1 = np.maximum(h1p, 0.0)
    h2p = q(h1) @ q(W2).T + b2
    h2 = np.maximum(h2p, 0.0)
    o = q(h2) @ q(W3).T + b3
    R = 1.0 / (1.0 + np.exp(-o))
    go = np.where(gate[:, None], g_rgba[:, :3] * R * (1.0 - R), 0.0)
    gh2 = (q(go) @ q(W3)) * (h2p > 0)
    gh1 = (q(gh2) @ q(W2)) * (h1p > 0)
    gx = q(gh1) @ q(W1)[:, :7]
    h1 = np.where(gate[:, None], h1, 0.0)
    h2 = np.where(gate[:, None], h2, 0.0)
    dW = np.concatenate([(gh1.T @ X).ravel(), gh1.sum(0), (gh2.T @ h1).ravel(), gh2.sum(0),
                         (go.T @ h2).ravel(), go.sum(0)])
    gcv = np.concatenate([g_rgba[:, :3] + gx[:, :3], gx[:, 3:7]], axis=1)
    return dW, gcv
