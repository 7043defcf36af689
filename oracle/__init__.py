"""ctypes binding of the FP64 CPU oracle (snerg_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg load this module; the product path (the HIP
library and its Python binding) never imports it, and it imports nothing
from the product.

Every function here takes plain NumPy inputs (grids in the canonical
block-sparse layout of the workload generator) and returns float64 results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "snerg_oracle.c")
_lib = None

U8, F32, F64 = 0, 1, 2
N_PARAMS = 883
DEFAULT_T_STOP = 1e-3
SIGMA_SCALE = 50.0


def build() -> str:
    """Compiles the oracle with gcc: FP64, no contraction, no fast-math."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB_PATH


class _Grid(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("B", ctypes.c_int32), ("indirection", ctypes.c_void_p),
                ("n_blocks", ctypes.c_int32), ("dtype", ctypes.c_int32), ("dens", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("feat", ctypes.c_void_p), ("sigma_scale", ctypes.c_double)]


class _Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("fwd", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3), ("W", ctypes.c_int32),
                ("H", ctypes.c_int32), ("focal", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_double * 3), ("t_stop", ctypes.c_double),
                ("early_stop", ctypes.c_int32), ("mlp_on", ctypes.c_int32),
                ("nn_gate", ctypes.c_int32), ("unpremultiply", ctypes.c_int32), ("per_sample_mlp", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_ray_setup.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, P, P, P]
        lib.orc_sample.argtypes = [P, P, P, P]
        lib.orc_composite.argtypes = [P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, P, P]
        lib.orc_encode.argtypes = [P, P, P, P]
        lib.orc_mlp.argtypes = [P, P, P]
        lib.orc_render.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int64, P, P, P, P,
                                   ctypes.c_int32]
        lib.orc_trace_visits.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int32,
                                         P, P, ctypes.c_int32]
        lib.orc_render_grad.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int64, P, P, P, P, P, P, P]
        lib.orc_bake_visibility.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P, ctypes.c_int32]
        for f in (lib.orc_ray_setup, lib.orc_sample, lib.orc_composite, lib.orc_encode, lib.orc_mlp,
                  lib.orc_render, lib.orc_trace_visits, lib.orc_render_grad, lib.orc_bake_visibility):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _ptr(a):
    return a.ctypes.data if a is not None else None


class OracleGrid:
    """Keeps the arrays alive and the C struct that points at them.

    With `values=None` the grid's uint8 bytes are used (value = byte/255);
    `values=(dens, rgb, feat)` supplies float32/float64 arrays of the same
    shapes instead (the trainable shadow)."""

    def __init__(self, grid, values=None, sigma_scale: float = SIGMA_SCALE):
        self.N, self.B = int(grid.N), int(grid.B)
        self.ind = np.ascontiguousarray(grid.indirection, dtype=np.int32)
        if values is None:
            d, r, f = grid.dens, grid.rgb, grid.feat
            dt = U8
        else:
            d, r, f = values
            dt = F64 if np.asarray(d).dtype == np.float64 else F32
            cast = np.float64 if dt == F64 else np.float32
            d, r, f = (np.asarray(a, dtype=cast) for a in (d, r, f))
        self.arrays = [np.ascontiguousarray(a) for a in (d, r, f)]
        self.dtype = dt
        self.struct = _Grid(self.N, self.B, self.ind.ctypes.data, int(self.arrays[0].shape[0]), dt,
                            self.arrays[0].ctypes.data, self.arrays[1].ctypes.data,
                            self.arrays[2].ctypes.data, float(sigma_scale))


def _cams(cams):
    arr = (_Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].eye[:] = [float(v) for v in c.eye]
        arr[i].fwd[:] = [float(v) for v in c.fwd]
        arr[i].right[:] = [float(v) for v in c.right]
        arr[i].up[:] = [float(v) for v in c.up]
        arr[i].W, arr[i].H, arr[i].focal = int(c.W), int(c.H), float(c.focal)
    return arr


def _opts(bg=(1.0, 1.0, 1.0), t_stop=DEFAULT_T_STOP, early_stop=True, mlp_on=True, nn_gate=False,
          unpremultiply=False, per_sample_mlp=False):
    o = _Opts()
    o.bg[:] = [float(v) for v in bg]
    o.t_stop, o.early_stop, o.mlp_on = float(t_stop), int(bool(early_stop)), int(bool(mlp_on))
    o.nn_gate, o.unpremultiply = int(bool(nn_gate)), int(bool(unpremultiply))
    o.per_sample_mlp = int(bool(per_sample_mlp))
    return o


def _mlp_vec(mlp):
    if mlp is None:
        return None
    if hasattr(mlp, "params"):
        v = np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in mlp.params()])
    else:
        v = np.asarray(mlp, np.float64).reshape(-1)
    assert v.size == N_PARAMS
    return np.ascontiguousarray(v)


def _ids(ray_ids, cams):
    total = sum(c.W * c.H for c in cams)
    if ray_ids is None:
        return None, total
    ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
    return ids, int(ids.size)


def ray_setup(cam, N: int, px: int, py: int):
    """Q16 lattice origin o, step s (int64 [3]) and unit direction d of pixel (px, py)."""
    lib = _load()
    c = _cams([cam])
    o = np.zeros(3, np.int64); s = np.zeros(3, np.int64); d = np.zeros(3, np.float64)
    _check(lib.orc_ray_setup(ctypes.byref(c[0]), N, px, py, o.ctypes.data, s.ctypes.data,
                             d.ctypes.data), "ray_setup")
    return o, s, d


def sample(og: OracleGrid, P):
    """Trilinear sample at Q16 lattice point P: (sigma, c_d[3], v[4]) and the active flag."""
    lib = _load()
    P = np.ascontiguousarray(P, dtype=np.int64)
    out = np.zeros(8, np.float64)
    act = ctypes.c_int32(0)
    _check(lib.orc_sample(ctypes.byref(og.struct), P.ctypes.data, out.ctypes.data, ctypes.byref(act)),
           "sample")
    return out, bool(act.value)


def composite(samples, delta: float, t_stop: float = DEFAULT_T_STOP, early_stop: bool = True):
    """Composites rows (sigma, c_d[3], v[4]); returns (C_d, V, T, n_used)."""
    lib = _load()
    s = np.ascontiguousarray(samples, dtype=np.float64).reshape(-1, 8)
    out = np.zeros(8, np.float64)
    n_used = ctypes.c_int64(0)
    _check(lib.orc_composite(s.ctypes.data, s.shape[0], delta, t_stop, int(early_stop), out.ctypes.data,
                             ctypes.byref(n_used)), "composite")
    return out[0:3], out[3:7], float(out[7]), int(n_used.value)


def encode(C, V, d):
    lib = _load()
    C = np.ascontiguousarray(C, np.float64); V = np.ascontiguousarray(V, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    x = np.zeros(34, np.float64)
    _check(lib.orc_encode(C.ctypes.data, V.ctypes.data, d.ctypes.data, x.ctypes.data), "encode")
    return x


def mlp_eval(mlp, x):
    lib = _load()
    p = _mlp_vec(mlp)
    x = np.ascontiguousarray(x, np.float64)
    R = np.zeros(3, np.float64)
    _check(lib.orc_mlp(p.ctypes.data, x.ctypes.data, R.ctypes.data), "mlp")
    return R


def render(og: OracleGrid, mlp, cams, ray_ids=None, bg=(1.0, 1.0, 1.0), t_stop=DEFAULT_T_STOP,
           early_stop=True, mlp_on=True, threads: int = 0, nn_gate=False, unpremultiply=False,
           per_sample_mlp=False):
    """Renders the given rays (all rays when ray_ids is None).  Returns a dict
    with rgba [n,4], aux [n,9] (C_d, V, T, gate) and counters [n,7]
    (macroblocks traversed, occupied macroblocks visited, in-block samples,
    composited samples, stopping k or -1, and the sums of the composited
    samples' k and k^2 modulo 2^32 as int32 bits)."""
    lib = _load()
    ids, n = _ids(ray_ids, cams)
    c = _cams(cams)
    o = _opts(bg, t_stop, early_stop, mlp_on, nn_gate, unpremultiply, per_sample_mlp)
    p = _mlp_vec(mlp)
    rgba = np.zeros((n, 4), np.float64)
    aux = np.zeros((n, 9), np.float64)
    cnt = np.zeros((n, 7), np.int32)
    _check(lib.orc_render(ctypes.byref(og.struct), _ptr(p), c, len(cams), _ptr(ids), n, ctypes.byref(o),
                          rgba.ctypes.data, aux.ctypes.data, cnt.ctypes.data, int(threads)), "render")
    return dict(rgba=rgba, aux=aux, counters=cnt)


def trace_visits(og: OracleGrid, cams, ray_ids=None, early_stop=False, t_stop=DEFAULT_T_STOP,
                 max_visits: int = 256, threads: int = 0, nn_gate=False):
    """Occupied macroblocks visited per ray (linear indirection index), [n, max_visits], and counts [n]."""
    lib = _load()
    ids, n = _ids(ray_ids, cams)
    c = _cams(cams)
    o = _opts(t_stop=t_stop, early_stop=early_stop, mlp_on=False, nn_gate=nn_gate)
    vis = np.full((n, max_visits), -1, np.int32)
    cnt = np.zeros(n, np.int32)
    _check(lib.orc_trace_visits(ctypes.byref(og.struct), c, len(cams), _ptr(ids), n, ctypes.byref(o),
                                max_visits, vis.ctypes.data, cnt.ctypes.data, int(threads)), "trace")
    return vis, cnt


def render_grad(og: OracleGrid, mlp, cams, g_rgba, ray_ids=None, bg=(1.0, 1.0, 1.0),
                t_stop=DEFAULT_T_STOP, early_stop=True, mlp_on=True, g_cv=None, nn_gate=False):
    """Gradient of sum(g_rgba * rgba) w.r.t. the 883 MLP parameters and the
    grid values (float grids only).  Returns (g_mlp, g_dens, g_rgb, g_feat).
    g_cv [n, 7] (optional) supplies each ray's dL/dC_d, dL/dV in place of the
    MLP backward (the MLP gradient is then zero)."""
    lib = _load()
    assert og.dtype != U8, "gradients need a float (shadow) grid"
    ids, n = _ids(ray_ids, cams)
    c = _cams(cams)
    o = _opts(bg, t_stop, early_stop, mlp_on, nn_gate)
    p = _mlp_vec(mlp)
    g = np.ascontiguousarray(g_rgba, np.float64).reshape(n, 4)
    gm = np.zeros(N_PARAMS, np.float64)
    gd = np.zeros(og.arrays[0].shape, np.float64)
    gr = np.zeros(og.arrays[1].shape, np.float64)
    gf = np.zeros(og.arrays[2].shape, np.float64)
    cv = np.ascontiguousarray(g_cv, np.float64).reshape(n, 7) if g_cv is not None else None
    _check(lib.orc_render_grad(ctypes.byref(og.struct), _ptr(p), c, len(cams), _ptr(ids), n,
                               ctypes.byref(o), g.ctypes.data, gm.ctypes.data, gd.ctypes.data,
                               gr.ctypes.data, gf.ctypes.data, _ptr(cv)), "render_grad")
    return gm, gd, gr, gf
