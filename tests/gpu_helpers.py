"""Helpers shared by the GPU parity tests: device set-up through the C ABI
binding and oracle references with the near-threshold early-stop reading
(a ray whose stopping decision lies within a relative 1e-5 of t_stop may
stop on either side; the oracle renders both and the GPU must match one)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle as O
from paper_2103_14645_amd import snerg as S

T_STOP = 1e-3
STOP_BAND = 1e-5


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


_handle = None


def handle():
    global _handle
    if _handle is None:
        _handle = S.Handle()
    return _handle


def device_grid(grid, values=None):
    """DeviceGrid of a workloads.Grid (uint8) or of float32 values (dens, rgb, feat)."""
    if values is None:
        return S.DeviceGrid(handle(), grid.N, grid.B, grid.indirection, grid.dens, grid.rgb, grid.feat)
    d, r, f = (np.ascontiguousarray(v, dtype=np.float32) for v in values)
    return S.DeviceGrid(handle(), grid.N, grid.B, grid.indirection, d, r, f)


def gpu_render(dg, mlp, cams, ids=None, want_aux=False, **kw):
    opts = S.make_opts(**kw)
    m = S.mlp_tensor(mlp) if mlp is not None else None
    idt = torch.from_numpy(np.asarray(ids, np.int64)).cuda() if ids is not None else None
    res = S.render(handle(), dg, m, cams, ray_ids=idt, opts=opts, want_aux=want_aux)
    torch.cuda.synchronize()
    if want_aux:
        return res[0].cpu().numpy(), res[1].cpu().numpy()
    return res.cpu().numpy()


def oracle_variants(og, mlp, cams, ids=None, bg=(1.0, 1.0, 1.0), early_stop=True, mlp_on=True):
    """Oracle rgba at t_stop and, with early stop, at t_stop (1 -+ 1e-5)."""
    outs = [O.render(og, mlp, cams, ray_ids=ids, bg=bg, t_stop=T_STOP, early_stop=early_stop,
                     mlp_on=mlp_on)["rgba"]]
    if early_stop:
        for f in (1.0 - STOP_BAND, 1.0 + STOP_BAND):
            outs.append(O.render(og, mlp, cams, ray_ids=ids, bg=bg, t_stop=T_STOP * f, early_stop=True,
                                 mlp_on=mlp_on)["rgba"])
    return outs


def parity_error(gpu, variants):
    """Per-ray max-abs error against the closest oracle branch, and the
    number of rays whose branches differ (near-threshold rays)."""
    errs = np.stack([np.abs(gpu.astype(np.float64) - v).max(axis=1) for v in variants])
    flagged = int((np.abs(variants[0] - np.stack(variants)).max(axis=(0, 2)) > 0).sum()) if len(variants) > 1 else 0
    return errs.min(axis=0), flagged
