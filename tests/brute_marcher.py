"""Brute-force dense marcher in NumPy, an independent cross-check of the C oracle.

It shares nothing with the oracle's march: the block-sparse grid is first
expanded into dense zero-padded N^3 arrays, every lattice index k of every
ray is evaluated at once as a [rays, k] array, corners are read from the
dense arrays with fancy indexing, and transmittance comes from a cumulative
product instead of a running loop.  The only thing taken from the oracle is
the per-ray lattice (origin, step, direction), which has its own pins.
Intended for grids up to 64^3.
"""
from __future__ import annotations

import numpy as np


def dense_arrays(grid, values=None):
    """Dense [N+2]^3 arrays (one voxel of zero padding on each side) of
    density value, colour [.., 3] and features [.., 4] in normalised units,
    plus the dense macroblock occupancy [G, G, G] (z, y, x)."""
    N, B = grid.N, grid.B
    G = N // B
    if values is None:
        d = grid.dens.astype(np.float64) / 255.0
        r = grid.rgb.astype(np.float64) / 255.0
        f = grid.feat.astype(np.float64) / 255.0
    else:
        d, r, f = (np.asarray(a, np.float64) for a in values)
    D = np.zeros((N + 2, N + 2, N + 2))
    R = np.zeros((N + 2, N + 2, N + 2, 3))
    F = np.zeros((N + 2, N + 2, N + 2, 4))
    occ = np.zeros((G, G, G), bool)
    ind = grid.indirection.reshape(G, G, G)
    for bz in range(G):
        for by in range(G):
            for bx in range(G):
                bid = ind[bz, by, bx]
                if bid < 0:
                    continue
                occ[bz, by, bx] = True
                sl = (slice(1 + bz * B, 1 + bz * B + B), slice(1 + by * B, 1 + by * B + B),
                      slice(1 + bx * B, 1 + bx * B + B))
                D[sl] = d[bid]
                R[sl] = r[bid]
                F[sl] = f[bid]
    return D, R, F, occ


def _mlp(mlp, C, V, dirs):
    """The 34-16-16-3 network on rows of (C, V, d) with d's sin/cos encoding."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, np.float64) for p in mlp.params())
    pe = []
    for l in range(4):
        a = (2.0 ** l) * np.pi * dirs
        pe += [np.sin(a), np.cos(a)]
    x = np.concatenate([C, V, dirs] + pe, axis=1)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return 1.0 / (1.0 + np.exp(-(h2 @ W3.T + b3)))


def march(grid, lattice, mlp, values=None, bg=(1.0, 1.0, 1.0), t_stop=1e-3, early_stop=True,
          mlp_on=True, sigma_scale=50.0, nn_gate=False, unpremultiply=False, per_sample_mlp=False):
    """lattice: (o [n,3], s [n,3], d [n,3]) per ray.  Returns rgba [n,4], gate [n],
    visits (list of lists of linear macroblock indices), counts of composited
    samples and counters [n,7]: macroblocks traversed (runs of equal
    consecutive macroblocks over the inside samples up to the stop), occupied
    macroblocks visited, samples in occupied macroblocks up to the stop,
    composited samples, the stopping k (-1 if none), and the sums of the
    composited k and k^2 modulo 2^32 (as int32 bits)."""
    N, B = grid.N, grid.B
    G = N // B
    Dn, Rn, Fn, occ = dense_arrays(grid, values)
    o, s, dirs = (np.asarray(a) for a in lattice)
    o = o.astype(np.int64)
    s = s.astype(np.int64)
    n = o.shape[0]
    L = N * 65536
    kmax = int(((np.abs(o).max() + L) // np.abs(s).max(axis=1).min()) + 2)
    k = np.arange(kmax + 1, dtype=np.int64)
    P = o[:, None, :] + k[None, :, None] * s[:, None, :]           # [n, K, 3]
    inside = np.all((P >= 0) & (P < L), axis=2)
    Pc = np.clip(P, 0, L - 1)
    blk = Pc // (B * 65536)
    blk_occ = occ[blk[..., 2], blk[..., 1], blk[..., 0]] & inside
    lin_blk = (blk[..., 2] * G + blk[..., 1]) * G + blk[..., 0]

    Q = P - 32768
    i0 = np.floor_divide(Q, 65536)
    fr = (Q - i0 * 65536) / 65536.0
    i0c = np.clip(i0, -1, N - 1)  # changes only samples outside the grid (never used)
    sig = np.zeros(P.shape[:2]); col = np.zeros(P.shape[:2] + (3,)); fea = np.zeros(P.shape[:2] + (4,))
    act = np.zeros(P.shape[:2], bool)
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                c = np.array([cx, cy, cz])
                w = np.prod(np.where(c[None, None, :] == 1, fr, 1.0 - fr), axis=2)
                idx = i0c + c[None, None, :] + 1
                dv = Dn[idx[..., 2], idx[..., 1], idx[..., 0]]
                act |= (dv != 0) & (w != 0)
                sig += w * dv
                col += w[..., None] * Rn[idx[..., 2], idx[..., 1], idx[..., 0]]
                fea += w[..., None] * Fn[idx[..., 2], idx[..., 1], idx[..., 0]]
    use = blk_occ & act
    if nn_gate:
        # the voxel whose centre is nearest: floor(P) in voxel units
        nn = np.clip(np.floor_divide(P, 65536), -1, N) + 1
        use &= Dn[nn[..., 2], nn[..., 1], nn[..., 0]] != 0
    sigma = np.where(use, sigma_scale * sig, 0.0)
    delta = 1.0 / N
    one_minus = np.exp(-sigma * delta)                               # 1 - alpha
    T_after = np.cumprod(one_minus, axis=1)
    if early_stop:
        stop = use & (T_after < t_stop)
        first = np.where(stop.any(axis=1), stop.argmax(axis=1), kmax + 1)
        keep = k[None, :] <= first[:, None]
        use = use & keep
        sigma = np.where(use, sigma, 0.0)
        one_minus = np.exp(-sigma * delta)
        T_after = np.cumprod(one_minus, axis=1)
    else:
        first = np.full(n, kmax + 1)
    T_before = np.concatenate([np.ones((n, 1)), T_after[:, :-1]], axis=1)
    if per_sample_mlp and mlp_on and mlp is not None:
        # every sample's colour plus the network's residual on (c_k, v_k, d)
        K = P.shape[1]
        dk = np.repeat(dirs[:, None, :], K, axis=1)
        col = col + _mlp(mlp, col.reshape(-1, 3), fea.reshape(-1, 4), dk.reshape(-1, 3)).reshape(n, K, 3)
    w = np.where(use, T_before * (1.0 - one_minus), 0.0)
    C = np.einsum("nk,nkc->nc", w, col)
    V = np.einsum("nk,nkc->nc", w, fea)
    T = T_after[:, -1]
    gate = use.any(axis=1)
    if unpremultiply:
        a = 1.0 - T
        sc = np.where(a > 0, np.minimum(1.0, 1.5 * a) / np.where(a > 0, a, 1.0), 1.0)
        C, V, T = C * sc[:, None], V * sc[:, None], np.where(a > 0, 1.0 - a * sc, T)

    R = np.zeros((n, 3))
    if mlp_on and mlp is not None and not per_sample_mlp:
        R = np.where(gate[:, None], _mlp(mlp, C, V, dirs), 0.0)
    rgb = C + T[:, None] * np.asarray(bg)[None, :] + R
    rgba = np.concatenate([rgb, (1.0 - T)[:, None]], axis=1)

    # per-ray counters, each from its own definition: the samples up to the
    # stopping one (all inside samples without a stop) ...
    upto = inside & (k[None, :] <= first[:, None])
    # ... their macroblocks, counted once per run of equal consecutive blocks
    runs = upto[:, :1].sum(axis=1) + (upto[:, 1:] & ~upto[:, :-1]).sum(axis=1) + \
        (upto[:, 1:] & upto[:, :-1] & (lin_blk[:, 1:] != lin_blk[:, :-1])).sum(axis=1)
    visit_mask = blk_occ & (k[None, :] <= first[:, None])
    stop_k = np.where(first <= kmax, first, -1)
    kk = np.where(use, k[None, :], 0).astype(np.uint64)
    ksum = (kk.sum(axis=1) % (1 << 32)).astype(np.uint32).view(np.int32)
    ksq = ((kk * kk).sum(axis=1) % (1 << 32)).astype(np.uint32).view(np.int32)
    visits = []
    for r in range(n):
        seq = lin_blk[r][visit_mask[r]]
        if seq.size:
            keep_idx = np.concatenate([[True], seq[1:] != seq[:-1]])
            visits.append([int(v) for v in seq[keep_idx]])
        else:
            visits.append([])
    counters = np.stack([runs, [len(v) for v in visits], visit_mask.sum(axis=1), use.sum(axis=1), stop_k,
                         ksum, ksq], axis=1).astype(np.int64)
    return dict(rgba=rgba, gate=gate, visits=visits, n_used=use.sum(axis=1), counters=counters)
