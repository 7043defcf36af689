"""FP64 reference of the baking culls and the 8-bit quantisation (Section
5.3 and 5.4 of the paper): which macroblocks of a densely evaluated field
are kept, and the bytes they are stored as.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
package smoke check and the benchmark's CPU-baseline leg use it; the
product path never imports it.

The field is given per voxel: sigma [N, N, N] (index [z, y, x]), density
per unit length of the world box [-1, 1]^3, colour rgb [N, N, N, 3] and
features feat [N, N, N, 4], in [0, 1].

 1. Opacity (Section 5.3): alpha = 1 - exp(-sigma v) with v = 1/N (the
    paper's voxel width; in this world box it is also the render step).
 2. Empty-space cull: a macroblock is kept only if its largest voxel alpha
    is at least tau_alpha (0.005).
 3. Visibility cull: a voxel's visibility is the largest transmittance
    between it and any training camera (orc_bake_visibility marches every
    training ray); a macroblock is kept only if its largest voxel visibility
    is at least tau_vis (0.01).
 4. Kept macroblocks get atlas ids 0, 1, ... in scan order (x fastest).
 5. 8-bit quantisation (Section 5.4): density byte rint(sigma * (255 /
    sigma_scale)), colour and feature bytes rint(255 c), clamped to 0..255,
    NaN to 0.  These integer decisions are taken in float32, the precision
    the field is stored in: the products are single IEEE float32
    multiplications and rint rounds half to even.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _cams, _check, _load

TAU_ALPHA = 0.005
TAU_VIS = 0.01


def voxel_alpha(sigma: np.ndarray) -> np.ndarray:
    """Step 1: alpha = 1 - exp(-sigma / N) per voxel, float64."""
    N = sigma.shape[0]
    return 1.0 - np.exp(-np.asarray(sigma, np.float64) / float(N))


def voxel_visibility(sigma: np.ndarray, cams, n_threads: int = 0):
    """Step 3: per-voxel largest transmittance to the training cameras and
    the smallest density prefix sum it comes from (both [N, N, N])."""
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    N = sig.shape[0]
    assert sig.shape == (N, N, N)
    vis = np.zeros((N, N, N), np.float64)
    depth = np.zeros((N, N, N), np.float64)
    c = _cams(cams)
    _check(_load().orc_bake_visibility(N, sig.ctypes.data, c, len(cams), vis.ctypes.data, depth.ctypes.data,
                                       int(n_threads)), "bake_visibility")
    return vis, depth


def block_max(a: np.ndarray, B: int) -> np.ndarray:
    """Largest value of every B^3 macroblock of a [N, N, N] array, returned
    flat in indirection order ((bz G + by) G + bx)."""
    N = a.shape[0]
    G = N // B
    return a.reshape(G, B, G, B, G, B).max(axis=(1, 3, 5)).reshape(-1)


@dataclass
class Culled:
    """Per-macroblock results, flat in indirection order."""
    alpha: np.ndarray        # largest voxel alpha
    vis: np.ndarray          # largest voxel visibility (0 when no training sample reaches it)
    depth: np.ndarray        # smallest density prefix sum behind that visibility (+inf if none)
    keep: np.ndarray         # bool
    indirection: np.ndarray  # int32, -1 = culled, else atlas id in scan order

    @property
    def n_blocks(self) -> int:
        return int(self.keep.sum())


def cull(sigma: np.ndarray, B: int, cams, tau_alpha: float = TAU_ALPHA, tau_vis: float = TAU_VIS,
         n_threads: int = 0) -> Culled:
    """Steps 1-4."""
    alpha = block_max(voxel_alpha(sigma), B)
    vis_v, depth_v = voxel_visibility(sigma, cams, n_threads)
    vis = block_max(vis_v, B)
    depth = -block_max(-depth_v, B)
    keep = (alpha >= tau_alpha) & (vis >= tau_vis)
    ind = np.full(keep.size, -1, np.int32)
    ind[keep] = np.arange(int(keep.sum()), dtype=np.int32)
    return Culled(alpha, vis, depth, keep, ind)


def quantize(x: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """Step 5 on any float32 array: bytes rint(x * float32(255 / scale))."""
    k = np.float32(255.0) / np.float32(scale)
    q = np.rint(np.asarray(x, np.float32) * k)
    return np.minimum(np.fmax(q, np.float32(0.0)), np.float32(255.0)).astype(np.uint8)


def pack_atlas(sigma, rgb, feat, B: int, indirection: np.ndarray, sigma_scale: float):
    """Canonical 8-bit atlas of the kept macroblocks: dens [n, B, B, B],
    rgb [n, B, B, B, 3], feat [n, B, B, B, 4] (voxel (x, y, z) of a block at
    [z, y, x])."""
    N = sigma.shape[0]
    G = N // B
    lin = np.nonzero(indirection >= 0)[0]
    ids = indirection[lin]
    n = len(lin)
    dens = np.zeros((n, B, B, B), np.uint8)
    rgb8 = np.zeros((n, B, B, B, 3), np.uint8)
    feat8 = np.zeros((n, B, B, B, 4), np.uint8)
    for li, bid in zip(lin, ids):
        bz, by, bx = li // (G * G), (li // G) % G, li % G
        sl = (slice(bz * B, (bz + 1) * B), slice(by * B, (by + 1) * B), slice(bx * B, (bx + 1) * B))
        dens[bid] = quantize(sigma[sl], sigma_scale)
        rgb8[bid] = quantize(rgb[sl])
        feat8[bid] = quantize(feat[sl])
    return dens, rgb8, feat8
