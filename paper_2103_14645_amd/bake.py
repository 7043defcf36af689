"""Baking a densely evaluated field into a renderable SNeRG (Section 5.3,
5.4): the two macroblock culls (snerg_bake_cull), the 8-bit canonical atlas
of the kept blocks (snerg_bake_quantize) and the packed layout the renderer
reads (snerg_pack_grid).  Every step runs in the library's kernels; this
module only allocates the outputs and issues the calls on the current
stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import snerg as S


@dataclass
class BakeResult:
    n_blocks: int
    indirection: torch.Tensor  # device int32 [(N/B)^3]
    block_alpha: torch.Tensor  # device float32 [(N/B)^3]: largest voxel alpha
    block_vis: torch.Tensor    # device float32 [(N/B)^3]: largest visibility (0 below tau_vis)
    dens: torch.Tensor         # device uint8 [n_blocks, B, B, B]
    rgb: torch.Tensor          # device uint8 [n_blocks, B, B, B, 3]
    feat: torch.Tensor         # device uint8 [n_blocks, B, B, B, 4]


def bake(handle: S.Handle, sigma: torch.Tensor, rgb: torch.Tensor, feat: torch.Tensor, B: int, cams,
         tau_alpha: float = 0.005, tau_vis: float = 0.01, sigma_scale: float = 50.0) -> BakeResult:
    """sigma [N, N, N], rgb [N, N, N, 3], feat [N, N, N, 4]: contiguous device
    float32 ([z, y, x]); cams: the training views (objects with eye, fwd,
    right, up, W, H, focal)."""
    N = int(sigma.shape[0])
    for t, shape in ((sigma, (N, N, N)), (rgb, (N, N, N, 3)), (feat, (N, N, N, 4))):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"expected a contiguous device float32 tensor of shape {shape}")
    G = N // B
    dev = sigma.device
    opts = S.make_bake_opts(tau_alpha, tau_vis, sigma_scale)
    ind = torch.empty(G ** 3, dtype=torch.int32, device=dev)
    alpha = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    vis = torch.empty(G ** 3, dtype=torch.float32, device=dev)
    n = S.snerg_bake_cull(handle, N, B, sigma, S.make_cameras(cams), opts, ind, alpha, vis)
    d8 = torch.empty((n, B, B, B), dtype=torch.uint8, device=dev)
    r8 = torch.empty((n, B, B, B, 3), dtype=torch.uint8, device=dev)
    f8 = torch.empty((n, B, B, B, 4), dtype=torch.uint8, device=dev)
    S.snerg_bake_quantize(handle, N, B, sigma, rgb, feat, ind, n, opts, d8, r8, f8)
    return BakeResult(n, ind, alpha, vis, d8, r8, f8)


def to_grid(handle: S.Handle, res: BakeResult, N: int, B: int, sigma_scale: float = 50.0) -> S.DeviceGrid:
    """Packs a bake for the renderer."""
    return S.DeviceGrid(handle, N, B, res.indirection, res.dens, res.rgb, res.feat, sigma_scale=sigma_scale)
