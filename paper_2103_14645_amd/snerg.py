"""Python binding of the gfx950 SNeRG renderer (libsnerg.so, C ABI in include/snerg.h).

Argument marshalling only: every step of the render path runs in the HIP
kernels.  PyTorch supplies device memory (tensors) and the stream.  The
entry points keep the C names:

    snerg_packed_size, snerg_pack_grid, snerg_render, snerg_render_backward,
    snerg_render_counted, snerg_trace_visits, snerg_set_tuning, snerg_get_tuning, snerg_autotune

plus small conveniences (Handle, DeviceGrid, render) that allocate the
output tensors.  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SNERG_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SNERG_LIB") or os.path.join(_HERE, "libsnerg.so")

SNERG_OK = 0
SNERG_ERR_INVALID_ARG = -1
SNERG_ERR_UNSUPPORTED = -2
SNERG_ERR_RANGE = -3
SNERG_ERR_HIP = -4
SNERG_ERR_WORKSPACE = -5

SNERG_U8 = 0
SNERG_F32 = 1

SNERG_FLAG_MLP_FP16 = 1 << 0
SNERG_FLAG_PERSISTENT = 1 << 1
SNERG_FLAG_GRAPH = 1 << 2
SNERG_FLAG_MLP_GRAD_ONLY = 1 << 3
SNERG_FLAG_NN_GATE = 1 << 4
SNERG_FLAG_UNPREMULTIPLY = 1 << 5
SNERG_FLAG_PER_SAMPLE_MLP = 1 << 6
SNERG_FLAG_PATCH_RAYS = 1 << 7
SNERG_FLAG_ACCUMULATE = 1 << 8
SNERG_FLAG_GRAD_PACKED = 1 << 9

SNERG_MLP_PARAMS = 883


class SnergError(RuntimeError):
    def __init__(self, code: int, what: str, message: str):
        super().__init__(f"{what} failed: {message} (status {code})")
        self.code = code


class snerg_grid(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("B", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("indirection", ctypes.c_void_p), ("packed", ctypes.c_void_p),
                ("sigma_scale", ctypes.c_float), ("reserved", ctypes.c_int32)]


class snerg_camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("fwd", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3), ("W", ctypes.c_int32),
                ("H", ctypes.c_int32), ("focal", ctypes.c_double)]


class snerg_opts(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_float * 3), ("t_stop", ctypes.c_float), ("early_stop", ctypes.c_int32),
                ("mlp_on", ctypes.c_int32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class snerg_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class snerg_bake_opts(ctypes.Structure):
    _fields_ = [("tau_alpha", ctypes.c_float), ("tau_vis", ctypes.c_float), ("sigma_scale", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class snerg_tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32)]

    def as_tuple(self):
        return (self.tile_w, self.tile_h, self.waves_per_group, self.groups_per_cu)


_lib = None
_P = ctypes.c_void_p


def lib():
    """Loads libsnerg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_14645_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sig = {
            "snerg_create": [ctypes.POINTER(_P)],
            "snerg_destroy": [_P],
            "snerg_packed_size": [i32, i32, i32, i32, ctypes.POINTER(sz)],
            "snerg_pack_grid": [_P, i32, i32, i32, i32, _P, _P, _P, _P, _P, sz, _P],
            "snerg_render": [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P, _P],
            "snerg_render_backward": [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P, _P, _P, _P, _P, _P],
            "snerg_render_counted": [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P, _P, _P],
            "snerg_render_noalloc": [_P, _P, _P, _P, i32, _P, i64, _P, _P, _P, _P],
            "snerg_trace_visits": [_P, _P, _P, i32, _P, i64, _P, i32, _P, _P, _P, _P],
            "snerg_set_tuning": [_P, _P],
            "snerg_get_tuning": [_P, _P],
            "snerg_autotune": [_P, _P, _P, _P, i32, _P, _P, i32, i32, _P, _P, _P, _P],
            "snerg_loss_mse": [_P, _P, _P, _P, i64, _P, _P, _P],
            "snerg_adam_step": [_P, _P, _P, _P, _P, i64, _P, _P],
            "snerg_bake_cull": [_P, i32, i32, _P, _P, i32, _P, _P, _P, _P, _P, _P],
            "snerg_bake_quantize": [_P, i32, i32, _P, _P, _P, _P, i32, _P, _P, _P, _P, _P],
            "snerg_tuning_lookup": [_P, _P, _P, i32, _P, _P, _P],
            "snerg_tuning_save": [_P, ctypes.c_char_p],
            "snerg_tuning_load": [_P, ctypes.c_char_p],
            "snerg_timing_enable": [_P, i32],
            "snerg_timing_read": [_P, _P, i32, _P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.snerg_status_string.argtypes = [ctypes.c_int]
        L.snerg_status_string.restype = ctypes.c_char_p
        L.snerg_last_error.argtypes = []
        L.snerg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ["snerg_create", "snerg_destroy", "snerg_status_string", "snerg_last_error", "snerg_packed_size",
            "snerg_pack_grid", "snerg_render", "snerg_render_backward", "snerg_render_counted", "snerg_render_noalloc",
            "snerg_trace_visits",
            "snerg_set_tuning", "snerg_get_tuning", "snerg_autotune", "snerg_loss_mse", "snerg_adam_step",
            "snerg_bake_cull", "snerg_bake_quantize", "snerg_timing_enable", "snerg_timing_read",
            "snerg_tuning_lookup", "snerg_tuning_save", "snerg_tuning_load"]


def _check(rc: int, what: str):
    if rc != SNERG_OK:
        L = lib()
        msg = L.snerg_last_error().decode() or L.snerg_status_string(rc).decode()
        raise SnergError(rc, what, msg)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    return t


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_cameras(cams):
    """snerg_camera array from objects with eye, fwd, right, up, W, H, focal."""
    arr = (snerg_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].eye[:] = [float(v) for v in c.eye]
        arr[i].fwd[:] = [float(v) for v in c.fwd]
        arr[i].right[:] = [float(v) for v in c.right]
        arr[i].up[:] = [float(v) for v in c.up]
        arr[i].W, arr[i].H, arr[i].focal = int(c.W), int(c.H), float(c.focal)
    return arr


def make_opts(bg=(1.0, 1.0, 1.0), t_stop=1e-3, early_stop=True, mlp_on=True, fp16=False,
              persistent=False, graph=False, mlp_grad_only=False, nn_gate=False, unpremultiply=False,
              per_sample_mlp=False, patch_rays=False, accumulate=False, grad_packed=False):
    o = snerg_opts()
    o.bg[:] = [float(v) for v in bg]
    o.t_stop = float(t_stop)
    o.early_stop = int(bool(early_stop))
    o.mlp_on = int(bool(mlp_on))
    o.flags = ((SNERG_FLAG_MLP_FP16 if fp16 else 0) | (SNERG_FLAG_PERSISTENT if persistent else 0)
               | (SNERG_FLAG_GRAPH if graph else 0) | (SNERG_FLAG_MLP_GRAD_ONLY if mlp_grad_only else 0)
               | (SNERG_FLAG_NN_GATE if nn_gate else 0) | (SNERG_FLAG_UNPREMULTIPLY if unpremultiply else 0)
               | (SNERG_FLAG_PER_SAMPLE_MLP if per_sample_mlp else 0) | (SNERG_FLAG_PATCH_RAYS if patch_rays else 0)
               | (SNERG_FLAG_ACCUMULATE if accumulate else 0) | (SNERG_FLAG_GRAD_PACKED if grad_packed else 0))
    return o


class Handle:
    def __init__(self):
        h = _P()
        _check(lib().snerg_create(ctypes.byref(h)), "snerg_create")
        self.h = h

    def close(self):
        if self.h:
            lib().snerg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def snerg_packed_size(N, B, n_blocks, dtype) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().snerg_packed_size(N, B, n_blocks, dtype, ctypes.byref(out)), "snerg_packed_size")
    return int(out.value)


def snerg_pack_grid(handle, N, B, n_blocks, dtype, indirection, dens, rgb, feat, packed, stream=None):
    _check(lib().snerg_pack_grid(handle.h, N, B, n_blocks, dtype, _ptr(indirection), _ptr(dens), _ptr(rgb),
                                 _ptr(feat), _ptr(packed), packed.numel() * packed.element_size(),
                                 _stream(stream)), "snerg_pack_grid")


def snerg_render(handle, grid: snerg_grid, mlp, cams, ray_ids, n_rays, opts, out_rgba, aux=None, stream=None):
    _check(lib().snerg_render(handle.h, ctypes.byref(grid), _ptr(mlp), cams, len(cams), _ptr(ray_ids),
                              int(n_rays), ctypes.byref(opts), _ptr(out_rgba), _ptr(aux), _stream(stream)),
           "snerg_render")


def snerg_render_noalloc(handle, grid: snerg_grid, mlp, cams, ray_ids, n_rays, opts, out_rgba, aux=None,
                         stream=None):
    _check(lib().snerg_render_noalloc(handle.h, ctypes.byref(grid), _ptr(mlp), cams, len(cams), _ptr(ray_ids),
                                      int(n_rays), ctypes.byref(opts), _ptr(out_rgba), _ptr(aux), _stream(stream)),
           "snerg_render_noalloc")


def snerg_render_counted(handle, grid: snerg_grid, mlp, cams, ray_ids, n_rays, opts, out_rgba, aux, counters,
                         stream=None):
    _check(lib().snerg_render_counted(handle.h, ctypes.byref(grid), _ptr(mlp), cams, len(cams), _ptr(ray_ids),
                                      int(n_rays), ctypes.byref(opts), _ptr(out_rgba), _ptr(aux), _ptr(counters),
                                      _stream(stream)), "snerg_render_counted")


def snerg_render_backward(handle, grid: snerg_grid, mlp, cams, ray_ids, n_rays, opts, aux, grad_rgba,
                          grad_mlp, grad_dens, grad_rgb, grad_feat, stream=None):
    _check(lib().snerg_render_backward(handle.h, ctypes.byref(grid), _ptr(mlp), cams, len(cams), _ptr(ray_ids),
                                       int(n_rays), ctypes.byref(opts), _ptr(aux), _ptr(grad_rgba),
                                       _ptr(grad_mlp), _ptr(grad_dens), _ptr(grad_rgb), _ptr(grad_feat),
                                       _stream(stream)), "snerg_render_backward")


def snerg_loss_mse(handle, rgba, target, n, grad_rgba, loss, target_ids=None, stream=None):
    _check(lib().snerg_loss_mse(handle.h, _ptr(rgba), _ptr(target), _ptr(target_ids), int(n), _ptr(grad_rgba),
                                _ptr(loss), _stream(stream)), "snerg_loss_mse")


def snerg_adam_step(handle, param, grad, m, v, n, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    cfg = snerg_adam(float(lr), float(beta1), float(beta2), float(eps), int(step), 0)
    _check(lib().snerg_adam_step(handle.h, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), int(n), ctypes.byref(cfg),
                                 _stream(stream)), "snerg_adam_step")


def snerg_timing_enable(handle, on=True):
    """on: False/0 off, True/1 time every render call, n >= 1 every n-th."""
    _check(lib().snerg_timing_enable(handle.h, int(on)), "snerg_timing_enable")


def snerg_timing_read(handle, max_n=256):
    """Render-kernel times (ms) recorded since timing was enabled, oldest first."""
    buf = (ctypes.c_float * max_n)()
    n = ctypes.c_int32(0)
    _check(lib().snerg_timing_read(handle.h, buf, int(max_n), ctypes.byref(n)), "snerg_timing_read")
    return [float(buf[i]) for i in range(n.value)]


def make_bake_opts(tau_alpha=0.005, tau_vis=0.01, sigma_scale=50.0):
    return snerg_bake_opts(float(tau_alpha), float(tau_vis), float(sigma_scale), 0)


def snerg_bake_cull(handle, N, B, sigma, cams, opts, indirection, block_alpha=None, block_vis=None,
                    stream=None) -> int:
    """Returns the number of kept macroblocks (synchronises the stream)."""
    n = ctypes.c_int32(-1)
    _check(lib().snerg_bake_cull(handle.h, int(N), int(B), _ptr(sigma), cams, len(cams), ctypes.byref(opts),
                                 _ptr(block_alpha), _ptr(block_vis), _ptr(indirection), ctypes.byref(n),
                                 _stream(stream)), "snerg_bake_cull")
    return int(n.value)


def snerg_bake_quantize(handle, N, B, sigma, rgb, feat, indirection, n_blocks, opts, dens8, rgb8, feat8,
                        stream=None):
    _check(lib().snerg_bake_quantize(handle.h, int(N), int(B), _ptr(sigma), _ptr(rgb), _ptr(feat),
                                     _ptr(indirection), int(n_blocks), ctypes.byref(opts), _ptr(dens8), _ptr(rgb8),
                                     _ptr(feat8), _stream(stream)), "snerg_bake_quantize")


def snerg_trace_visits(handle, grid: snerg_grid, cams, ray_ids, n_rays, opts, max_visits, visits, counts,
                       counters=None, stream=None):
    _check(lib().snerg_trace_visits(handle.h, ctypes.byref(grid), cams, len(cams), _ptr(ray_ids), int(n_rays),
                                    ctypes.byref(opts), int(max_visits), _ptr(visits), _ptr(counts),
                                    _ptr(counters), _stream(stream)), "snerg_trace_visits")


def snerg_set_tuning(handle, tile_w, tile_h, waves_per_group, groups_per_cu):
    t = snerg_tuning(tile_w, tile_h, waves_per_group, groups_per_cu)
    _check(lib().snerg_set_tuning(handle.h, ctypes.byref(t)), "snerg_set_tuning")


def snerg_get_tuning(handle):
    t = snerg_tuning()
    _check(lib().snerg_get_tuning(handle.h, ctypes.byref(t)), "snerg_get_tuning")
    return t.as_tuple()


def snerg_tuning_lookup(handle, grid: snerg_grid, cams, opts):
    """(launch shape a render of this workload uses, recorded by snerg_autotune?)"""
    t = snerg_tuning()
    found = ctypes.c_int32(0)
    _check(lib().snerg_tuning_lookup(handle.h, ctypes.byref(grid), cams, len(cams), ctypes.byref(opts),
                                     ctypes.byref(t), ctypes.byref(found)), "snerg_tuning_lookup")
    return t.as_tuple(), bool(found.value)


def snerg_tuning_save(handle, path):
    _check(lib().snerg_tuning_save(handle.h, str(path).encode()), "snerg_tuning_save")


def snerg_tuning_load(handle, path):
    _check(lib().snerg_tuning_load(handle.h, str(path).encode()), "snerg_tuning_load")


def snerg_autotune(handle, grid: snerg_grid, mlp, cams, opts, out_rgba, candidates=None, reps=3, stream=None):
    """Returns ((tile_w, tile_h, waves_per_group, groups_per_cu), ms per render)."""
    best = snerg_tuning()
    ms = ctypes.c_float(0.0)
    cand, n = None, 0
    if candidates:
        cand = (snerg_tuning * len(candidates))(*[snerg_tuning(*c) for c in candidates])
        n = len(candidates)
    _check(lib().snerg_autotune(handle.h, ctypes.byref(grid), _ptr(mlp), cams, len(cams), ctypes.byref(opts),
                                cand, n, int(reps), _ptr(out_rgba), ctypes.byref(best), ctypes.byref(ms),
                                _stream(stream)), "snerg_autotune")
    return best.as_tuple(), float(ms.value)


# ------------------------------------------------------------------ conveniences

class DeviceGrid:
    """A grid resident in device memory: canonical arrays, indirection and the packed layout.

    `dens, rgb, feat` are uint8 (SNERG_U8) or float32 (SNERG_F32) arrays or
    tensors in canonical layout; they are copied to `device` and packed."""

    def __init__(self, handle: Handle, N, B, indirection, dens, rgb, feat, sigma_scale=50.0,
                 device="cuda", stream=None):
        def dev(a):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device).contiguous()

        self.handle = handle
        self.N, self.B = int(N), int(B)
        self.ind = dev(np.asarray(indirection, dtype=np.int32) if not isinstance(indirection, torch.Tensor)
                       else indirection)
        self.dens, self.rgb, self.feat = dev(dens), dev(rgb), dev(feat)
        if self.dens.dtype == torch.uint8:
            self.dtype = SNERG_U8
        elif self.dens.dtype == torch.float32:
            self.dtype = SNERG_F32
        else:
            raise TypeError("grid values must be uint8 or float32")
        self.n_blocks = int(self.dens.shape[0])
        self.sigma_scale = float(sigma_scale)
        size = snerg_packed_size(self.N, self.B, self.n_blocks, self.dtype)
        self.packed = torch.empty(max(size, 256), dtype=torch.uint8, device=device)
        self.repack(stream)

    def repack(self, stream=None):
        snerg_pack_grid(self.handle, self.N, self.B, self.n_blocks, self.dtype, self.ind, self.dens, self.rgb,
                        self.feat, self.packed, stream)

    def struct(self) -> snerg_grid:
        return snerg_grid(self.N, self.B, self.n_blocks, self.dtype, self.ind.data_ptr(), self.packed.data_ptr(),
                          self.sigma_scale, 0)


def render(handle, dgrid: DeviceGrid, mlp, cams, ray_ids=None, opts=None, want_aux=False, stream=None):
    """Allocates outputs and calls snerg_render.  mlp: device float32 [883]
    tensor or None; ray_ids: device int64 tensor or None (all rays)."""
    opts = opts or make_opts()
    carr = make_cameras(cams)
    n = int(ray_ids.numel()) if ray_ids is not None else sum(int(c.W) * int(c.H) for c in cams)
    dev = dgrid.packed.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    aux = torch.empty((n, 8), dtype=torch.float32, device=dev) if want_aux else None
    snerg_render(handle, dgrid.struct(), mlp, carr, ray_ids, n, opts, out, aux, stream)
    return (out, aux) if want_aux else out


def render_counted(handle, dgrid: DeviceGrid, mlp, cams, ray_ids=None, opts=None, stream=None):
    """snerg_render_counted with allocated outputs: (rgba [n,4], counters [n,7] int32)."""
    opts = opts or make_opts()
    carr = make_cameras(cams)
    n = int(ray_ids.numel()) if ray_ids is not None else sum(int(c.W) * int(c.H) for c in cams)
    dev = dgrid.packed.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    counters = torch.full((n, 7), -7, dtype=torch.int32, device=dev)
    snerg_render_counted(handle, dgrid.struct(), mlp, carr, ray_ids, n, opts, out, None, counters, stream)
    return out, counters


def trace_visits(handle, dgrid: DeviceGrid, cams, ray_ids=None, opts=None, max_visits=256, stream=None):
    opts = opts or make_opts(mlp_on=False)
    carr = make_cameras(cams)
    n = int(ray_ids.numel()) if ray_ids is not None else sum(int(c.W) * int(c.H) for c in cams)
    dev = dgrid.packed.device
    visits = torch.full((n, max_visits), -1, dtype=torch.int32, device=dev)
    counts = torch.zeros(n, dtype=torch.int32, device=dev)
    counters = torch.zeros((n, 5), dtype=torch.int32, device=dev)
    snerg_trace_visits(handle, dgrid.struct(), carr, ray_ids, n, opts, max_visits, visits, counts, counters,
                       stream)
    return visits, counts, counters


def mlp_tensor(mlp, device="cuda"):
    """Flat float32 [883] device tensor from an object with params() or an array."""
    if hasattr(mlp, "params"):
        v = np.concatenate([np.asarray(p, np.float32).reshape(-1) for p in mlp.params()])
    else:
        v = np.asarray(mlp, np.float32).reshape(-1)
    assert v.size == SNERG_MLP_PARAMS
    return torch.from_numpy(v.copy()).to(device)
