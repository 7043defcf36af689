"""torch.autograd.Function around snerg_render / snerg_render_backward.

The trainable quantities are the deferred-MLP parameter vector (883 floats)
and a float32 shadow of the grid values in canonical atlas layout (density
in [0, 1] units with sigma = sigma_scale * density, colour and features in
[0, 1]): the fine-tuning of Section 5.5 (Adam on the MLP against a pixel
loss, Eq. 3), extended to the grid values.  Each forward call re-packs the
shadow into the renderer's layout (snerg_pack_grid) and renders with the
auxiliary per-ray state that the backward kernels consume; nothing per
sample is stored.
"""
from __future__ import annotations

import torch

from . import snerg as S


class ShadowRenderer:
    """Renders a float32 shadow grid with a fixed indirection grid."""

    def __init__(self, handle: "S.Handle", N: int, B: int, indirection, n_blocks: int,
                 sigma_scale: float = 50.0, device="cuda"):
        self.handle = handle
        self.N, self.B, self.n_blocks = int(N), int(B), int(n_blocks)
        ind = indirection if isinstance(indirection, torch.Tensor) else torch.as_tensor(indirection)
        self.ind = ind.to(device=device, dtype=torch.int32).contiguous()
        self.sigma_scale = float(sigma_scale)
        size = S.snerg_packed_size(self.N, self.B, self.n_blocks, S.SNERG_F32)
        self.packed = torch.empty(max(size, 256), dtype=torch.uint8, device=device)
        self.version = 0

    def pack(self, dens, rgb, feat):
        S.snerg_pack_grid(self.handle, self.N, self.B, self.n_blocks, S.SNERG_F32, self.ind, dens, rgb, feat,
                          self.packed)
        self.version += 1
        return self.version

    def struct(self):
        return S.snerg_grid(self.N, self.B, self.n_blocks, S.SNERG_F32, self.ind.data_ptr(),
                            self.packed.data_ptr(), self.sigma_scale, 0)


class SnergRenderFn(torch.autograd.Function):
    """rgba = SnergRenderFn.apply(dens, rgb, feat, mlp, renderer, cams, ray_ids, opts)

    dens [n_blocks, B, B, B], rgb [.., 3], feat [.., 4]: float32 CUDA tensors;
    mlp: float32 [883]; cams: snerg_camera array (S.make_cameras); ray_ids:
    int64 CUDA tensor or None (all rays); opts: snerg_opts.  Returns rgba
    [n_rays, 4]."""

    @staticmethod
    def forward(ctx, dens, rgb, feat, mlp, renderer: ShadowRenderer, cams, ray_ids, opts):
        dens, rgb, feat, mlp = (t.contiguous() for t in (dens, rgb, feat, mlp))
        version = renderer.pack(dens, rgb, feat)
        n = int(ray_ids.numel()) if ray_ids is not None else sum(int(c.W) * int(c.H) for c in cams)
        out = torch.empty((n, 4), dtype=torch.float32, device=dens.device)
        aux = torch.empty((n, 8), dtype=torch.float32, device=dens.device)
        S.snerg_render(renderer.handle, renderer.struct(), mlp, cams, ray_ids, n, opts, out, aux)
        ctx.renderer, ctx.cams, ctx.opts, ctx.n = renderer, cams, opts, n
        ctx.version = version
        ctx.save_for_backward(mlp, aux, ray_ids if ray_ids is not None else torch.empty(0), dens, rgb, feat)
        ctx.has_ids = ray_ids is not None
        ctx.shapes = (dens.shape, rgb.shape, feat.shape)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mlp, aux, ids, dens, rgb, feat = ctx.saved_tensors
        r = ctx.renderer
        if r.version != ctx.version:  # another forward re-packed the renderer since
            ctx.version = r.pack(dens, rgb, feat)
        dev = aux.device
        g_mlp = torch.empty(S.SNERG_MLP_PARAMS, dtype=torch.float32, device=dev)
        g_d = torch.empty(ctx.shapes[0], dtype=torch.float32, device=dev)
        g_r = torch.empty(ctx.shapes[1], dtype=torch.float32, device=dev)
        g_f = torch.empty(ctx.shapes[2], dtype=torch.float32, device=dev)
        S.snerg_render_backward(r.handle, r.struct(), mlp, ctx.cams, ids if ctx.has_ids else None, ctx.n,
                                ctx.opts, aux, grad_out.contiguous(), g_mlp, g_d, g_r, g_f)
        return g_d, g_r, g_f, g_mlp, None, None, None, None


def render_shadow(renderer, dens, rgb, feat, mlp, cams, ray_ids=None, opts=None):
    return SnergRenderFn.apply(dens, rgb, feat, mlp, renderer, cams, ray_ids, opts or S.make_opts())
