"""Fine-tuning of the deferred shading network on a fixed SNeRG (Section
5.5): minibatches of rays are rendered with the current weights, the
squared error against the observed pixels is back-propagated to the 883
weights, and Adam (learning rate 3e-4) updates them.  Every step runs in the
library's kernels (snerg_render, snerg_loss_mse, snerg_render_backward with
SNERG_FLAG_MLP_GRAD_ONLY, snerg_adam_step); this module only holds the
buffers and issues the calls on the current stream.
"""
from __future__ import annotations

import torch

from . import snerg as S


class MlpFineTuner:
    """Holds the weights (device float32 [883], updated in place), the Adam
    moments and per-minibatch scratch for one grid, camera set and set of
    observed pixels (device float32 [total rays][4], camera-major)."""

    def __init__(self, handle: S.Handle, grid: S.snerg_grid, mlp: torch.Tensor, cams, targets: torch.Tensor,
                 lr: float = 3e-4, fp16: bool = False, max_batch: int = 65536):
        if mlp.dtype != torch.float32 or mlp.numel() != 883 or not mlp.is_cuda:
            raise ValueError("mlp must be a device float32 tensor of 883 weights")
        self.h, self.grid, self.mlp, self.targets = handle, grid, mlp, targets
        self.cams = S.make_cameras(cams)
        self.cam_list = list(cams)
        self.n_total = sum(c.n_rays for c in cams)
        if targets.shape != (self.n_total, 4):
            raise ValueError(f"targets must be [{self.n_total}, 4]")
        self.lr = lr
        self.opts = S.make_opts(fp16=fp16)
        self.bopts = S.make_opts(fp16=fp16, mlp_grad_only=True)
        dev = mlp.device
        self.m = torch.zeros(883, device=dev)
        self.v = torch.zeros(883, device=dev)
        self.t = 0
        self.grad = torch.empty(883, device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.out = torch.empty((max_batch, 4), device=dev)
        self.aux = torch.empty((max_batch, 8), device=dev)
        self.g_rgba = torch.empty((max_batch, 4), device=dev)

    def step(self, ray_ids: torch.Tensor) -> torch.Tensor:
        """One Adam step on the rays `ray_ids` (device int64); returns the
        minibatch loss before the step (a device tensor, not synchronised)."""
        n = ray_ids.numel()
        if n > self.out.shape[0]:
            raise ValueError("minibatch larger than max_batch")
        S.snerg_render(self.h, self.grid, self.mlp, self.cams, ray_ids, n, self.opts, self.out, self.aux)
        S.snerg_loss_mse(self.h, self.out, self.targets, n, self.g_rgba, self.loss, target_ids=ray_ids)
        S.snerg_render_backward(self.h, self.grid, self.mlp, self.cams, ray_ids, n, self.bopts, self.aux,
                                self.g_rgba, self.grad, None, None, None)
        self.t += 1
        S.snerg_adam_step(self.h, self.mlp, self.grad, self.m, self.v, 883, self.lr, self.t)
        return self.loss.clone()

    def patch_order(self, generator: torch.Generator, tile: int = 8) -> torch.Tensor:
        """Every ray id once, grouped into tile x tile pixel patches (edge
        patches ragged), the patches in an order drawn from `generator` (a
        CPU generator).  Minibatches cut from it are patches of neighbouring
        pixels, so each wavefront of the render and the backward marches 64
        neighbouring rays (a full 8x8 patch) instead of 64 scattered ones."""
        dev = self.mlp.device
        if not hasattr(self, "_patches"):
            keys, ids, n_tiles, off = [], [], 0, 0
            for c in self.cam_list:
                py, px = torch.meshgrid(torch.arange(c.H), torch.arange(c.W), indexing="ij")
                tx = (c.W + tile - 1) // tile
                t = n_tiles + (py // tile) * tx + px // tile
                keys.append((t * tile * tile + (py % tile) * tile + px % tile).reshape(-1))
                ids.append(off + (py * c.W + px).reshape(-1))
                n_tiles += tx * ((c.H + tile - 1) // tile)
                off += c.W * c.H
            key, rid = torch.cat(keys), torch.cat(ids)
            order = torch.argsort(key)
            flat = rid[order]
            lens = torch.bincount(key[order] // (tile * tile), minlength=n_tiles)
            self._patches = (flat.to(dev), (torch.cumsum(lens, 0) - lens).to(dev), lens.to(dev))
        flat, starts, lens = self._patches
        perm = torch.randperm(len(lens), generator=generator).to(dev)
        lp = lens[perm]
        shift = starts[perm] - (torch.cumsum(lp, 0) - lp)  # where each permuted patch starts in `flat`, minus its new start
        idx = torch.repeat_interleave(shift, lp) + torch.arange(int(lp.sum()), device=dev)
        return flat[idx]

    def epoch(self, batch: int, generator: torch.Generator, patches: bool = False) -> list:
        """One pass over every ray in random minibatches of `batch`; returns
        the per-step losses.  Pixels (default): rays drawn independently
        (order from `generator`), each minibatch handed over in ray-id order
        (rays of one camera and nearby rows side by side), so that the lanes
        of a wavefront march nearby rays: the set of rays and the loss are
        unchanged, the render of a 65,536-ray minibatch is about 30% faster
        than in draw order.  patches=True: minibatches of whole 8x8 pixel
        patches in random order (`generator` on the CPU), see patch_order."""
        if patches:
            order = self.patch_order(generator)
            return [self.step(order[i:i + batch]) for i in range(0, self.n_total, batch)]
        order = torch.randperm(self.n_total, device=self.mlp.device, generator=generator)
        return [self.step(order[i:i + batch].sort().values) for i in range(0, self.n_total, batch)]
