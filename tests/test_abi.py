"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/snerg.h, and its host-only validation returns the
documented status for each bad argument before touching the device (a NULL
handle is passed, so any call that got past validation would fail with
"handle is NULL" instead)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2103_14645_amd import snerg as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation is host-only


def declared_functions():
    text = open(os.path.join(ROOT, "include", "snerg.h")).read()
    return sorted(set(re.findall(r"\b(snerg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    lib = S.lib()
    names = declared_functions()
    assert {"snerg_render", "snerg_render_backward", "snerg_pack_grid", "snerg_trace_visits"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(S.EXPORTED) == set(names)


def test_status_strings():
    lib = S.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.snerg_status_string(code)
    assert lib.snerg_status_string(-99) == b"unknown status"


def test_packed_size_layout_and_errors():
    # occupancy {bits, rank} words + rank->lin + rank->id (each 256-aligned),
    # then per block a 256-aligned record: (B+1)^3 distance bytes (16-aligned)
    # and (B+2)^3 padded voxels
    def a256(x):
        return (x + 255) // 256 * 256

    n = 433
    head = a256(math.ceil(16 ** 3 / 32) * 8) + 2 * a256(n * 4)
    dist = (33 ** 3 + 15) // 16 * 16
    assert S.snerg_packed_size(512, 32, n, S.SNERG_U8) == head + n * a256(dist + 34 ** 3 * 8)
    assert S.snerg_packed_size(512, 32, n, S.SNERG_F32) == head + n * a256(dist + 34 ** 3 * 32)
    with pytest.raises(S.SnergError) as e:
        S.snerg_packed_size(4096, 32, 1, S.SNERG_U8)          # N/B = 128: occupancy table too large for LDS
    assert e.value.code == S.SNERG_ERR_UNSUPPORTED
    for args, code in [((512, 24, 1, 0), S.SNERG_ERR_UNSUPPORTED), ((500, 32, 1, 0), S.SNERG_ERR_UNSUPPORTED),
                       ((32768, 32, 1, 0), S.SNERG_ERR_RANGE), ((512, 32, 1, 7), S.SNERG_ERR_UNSUPPORTED),
                       ((512, 32, -1, 0), S.SNERG_ERR_INVALID_ARG),
                       ((64, 8, 513, 0), S.SNERG_ERR_INVALID_ARG)]:
        with pytest.raises(S.SnergError) as e:
            S.snerg_packed_size(*args)
        assert e.value.code == code


class NullHandle:
    h = None


def good_camera():
    c = S.snerg_camera()
    c.eye[:] = [0.0, 0.0, -2.0]
    c.fwd[:] = [0.0, 0.0, 1.0]
    c.right[:] = [1.0, 0.0, 0.0]
    c.up[:] = [0.0, 1.0, 0.0]
    c.W, c.H, c.focal = 8, 4, 10.0
    return c


def call_render(grid=None, cams=None, n_cams=1, ray_ids=None, n_rays=32, opts=None, mlp=FAKE, out=FAKE):
    lib = S.lib()
    grid = grid or S.snerg_grid(64, 8, 8, S.SNERG_U8, FAKE.value, FAKE.value, 50.0, 0)
    if cams is None:
        cams = (S.snerg_camera * 1)(good_camera())
    opts = opts or S.make_opts()
    return lib.snerg_render(None, ctypes.byref(grid), mlp, cams, n_cams, ray_ids, n_rays, ctypes.byref(opts),
                            out, None, None)


def last_error():
    return S.lib().snerg_last_error().decode()


def test_render_validation_paths():
    assert call_render() == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()   # all valid, no handle
    assert call_render(grid=S.snerg_grid(64, 6, 8, 0, FAKE.value, FAKE.value, 50.0, 0)) == S.SNERG_ERR_UNSUPPORTED
    assert call_render(grid=S.snerg_grid(64, 8, 8, 0, None, FAKE.value, 50.0, 0)) == S.SNERG_ERR_INVALID_ARG
    assert call_render(grid=S.snerg_grid(64, 8, 8, 0, FAKE.value, None, 50.0, 0)) == S.SNERG_ERR_INVALID_ARG
    assert call_render(grid=S.snerg_grid(64, 8, 8, 0, FAKE.value, FAKE.value, float("nan"), 0)) == -1
    assert call_render(n_rays=31) == S.SNERG_ERR_INVALID_ARG          # must equal W*H without ray_ids
    assert call_render(n_rays=-1) == S.SNERG_ERR_INVALID_ARG
    assert call_render(n_cams=0) == S.SNERG_ERR_INVALID_ARG
    assert call_render(mlp=None) == S.SNERG_ERR_INVALID_ARG and "mlp" in last_error()
    assert call_render(mlp=None, opts=S.make_opts(mlp_on=False)) == S.SNERG_ERR_INVALID_ARG  # handle again
    assert "handle" in last_error()
    assert call_render(out=None) == S.SNERG_ERR_INVALID_ARG
    o = S.make_opts(); o.flags = 1 << 10
    assert call_render(opts=o) == S.SNERG_ERR_UNSUPPORTED
    o = S.make_opts(); o.t_stop = float("inf")
    assert call_render(opts=o) == S.SNERG_ERR_INVALID_ARG
    o = S.make_opts(); o.bg[1] = float("nan")
    assert call_render(opts=o) == S.SNERG_ERR_INVALID_ARG
    assert call_render(ray_ids=FAKE, n_rays=5) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()


@pytest.mark.parametrize("field,value,code", [
    ("W", 0, S.SNERG_ERR_INVALID_ARG), ("focal", 0.0, S.SNERG_ERR_INVALID_ARG),
    ("focal", float("nan"), S.SNERG_ERR_INVALID_ARG), ("eye", [float("inf"), 0, 0], S.SNERG_ERR_INVALID_ARG),
    ("eye", [0.0, 0.0, 1500.0], S.SNERG_ERR_RANGE), ("fwd", [0.0, 0.1, 1.0], S.SNERG_ERR_INVALID_ARG),
    ("up", [1.0, 0.0, 0.0], S.SNERG_ERR_INVALID_ARG),
])
def test_camera_validation(field, value, code):
    c = good_camera()
    setattr(c, field, (ctypes.c_double * 3)(*value)) if isinstance(value, list) else setattr(c, field, value)
    cams = (S.snerg_camera * 1)(c)
    n = max(c.W, 0) * c.H
    assert call_render(cams=cams, n_rays=n) == code


def test_backward_trace_pack_autotune_validation():
    lib = S.lib()
    cams = (S.snerg_camera * 1)(good_camera())
    opts = S.make_opts()
    u8 = S.snerg_grid(64, 8, 8, S.SNERG_U8, FAKE.value, FAKE.value, 50.0, 0)
    f32 = S.snerg_grid(64, 8, 8, S.SNERG_F32, FAKE.value, FAKE.value, 50.0, 0)
    bw = lambda g, o=opts, gm=FAKE: lib.snerg_render_backward(None, ctypes.byref(g), FAKE, cams, 1, None, 32,
                                                              ctypes.byref(o), FAKE, FAKE, gm, FAKE, FAKE, FAKE,
                                                              None)
    assert bw(u8) == S.SNERG_ERR_UNSUPPORTED
    assert bw(f32, gm=None) == S.SNERG_ERR_INVALID_ARG
    assert bw(f32) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert bw(f32, o=S.make_opts(fp16=True)) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    # packed grid gradients: grad_dens only
    assert bw(f32, o=S.make_opts(grad_packed=True)) == S.SNERG_ERR_INVALID_ARG and "GRAD_PACKED" in last_error()
    bwp = lambda gr, gf: lib.snerg_render_backward(None, ctypes.byref(f32), FAKE, cams, 1, None, 32,
                                                   ctypes.byref(S.make_opts(grad_packed=True)), FAKE, FAKE, FAKE,
                                                   FAKE, gr, gf, None)
    assert bwp(FAKE, None) == S.SNERG_ERR_INVALID_ARG and "GRAD_PACKED" in last_error()
    assert bwp(None, None) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    tr = lambda mv, vis: lib.snerg_trace_visits(None, ctypes.byref(u8), cams, 1, None, 32, ctypes.byref(opts),
                                                mv, vis, FAKE, None, None)
    assert tr(-1, FAKE) == S.SNERG_ERR_INVALID_ARG
    assert tr(4, None) == S.SNERG_ERR_INVALID_ARG
    assert tr(0, None) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    pk = lambda nbytes: lib.snerg_pack_grid(None, 64, 8, 8, 0, FAKE, FAKE, FAKE, FAKE, FAKE, nbytes, None)
    assert pk(10) == S.SNERG_ERR_WORKSPACE
    assert pk(1 << 30) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    bad = (S.snerg_tuning * 1)(S.snerg_tuning(8, 4, 4, 8))
    at = lambda cand, n, reps: lib.snerg_autotune(None, ctypes.byref(u8), FAKE, cams, 1, ctypes.byref(opts), cand,
                                                  n, reps, FAKE, None, None, None)
    assert at(bad, 1, 3) == S.SNERG_ERR_INVALID_ARG and "64" in last_error()
    assert at(None, 0, 0) == S.SNERG_ERR_INVALID_ARG
    assert at(None, 0, 3) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        S.lib()


def test_finetuning_entry_point_validation():
    lib = S.lib()
    loss = lambda n, r=FAKE, t=FAKE, g=FAKE, l=FAKE: lib.snerg_loss_mse(None, r, t, None, n, g, l, None)
    assert loss(-1) == S.SNERG_ERR_INVALID_ARG
    assert loss(4, l=None) == S.SNERG_ERR_INVALID_ARG
    assert loss(4, t=None) == S.SNERG_ERR_INVALID_ARG
    assert loss(0, r=None, t=None, g=None) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    adam = lambda cfg, n=8, p=FAKE: lib.snerg_adam_step(None, p, FAKE, FAKE, FAKE, n, ctypes.byref(cfg), None)
    assert adam(S.snerg_adam(3e-4, 0.9, 0.999, 1e-8, 0, 0)) == S.SNERG_ERR_INVALID_ARG        # step 0
    assert adam(S.snerg_adam(3e-4, 1.0, 0.999, 1e-8, 1, 0)) == S.SNERG_ERR_INVALID_ARG        # beta1 = 1
    assert adam(S.snerg_adam(float("nan"), 0.9, 0.999, 1e-8, 1, 0)) == S.SNERG_ERR_INVALID_ARG
    assert adam(S.snerg_adam(3e-4, 0.9, 0.999, 0.0, 1, 0)) == S.SNERG_ERR_INVALID_ARG         # eps = 0
    assert adam(S.snerg_adam(3e-4, 0.9, 0.999, 1e-8, 1, 0), p=None) == S.SNERG_ERR_INVALID_ARG
    assert adam(S.snerg_adam(3e-4, 0.9, 0.999, 1e-8, 1, 0)) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert lib.snerg_adam_step(None, None, None, None, None, 8, None, None) == S.SNERG_ERR_INVALID_ARG


def test_mlp_only_backward_accepts_uint8_grids():
    lib = S.lib()
    cams = (S.snerg_camera * 1)(good_camera())
    u8 = S.snerg_grid(64, 8, 8, S.SNERG_U8, FAKE.value, FAKE.value, 50.0, 0)
    o = S.make_opts(mlp_grad_only=True)
    rc = lib.snerg_render_backward(None, ctypes.byref(u8), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE,
                                   FAKE, None, None, None, None)
    assert rc == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()   # got past every argument check
    rc = lib.snerg_render_backward(None, ctypes.byref(u8), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE,
                                   None, None, None, None, None)
    assert rc == S.SNERG_ERR_INVALID_ARG and "grad_mlp" in last_error()


def test_unpremultiply_has_no_backward():
    lib = S.lib()
    cams = (S.snerg_camera * 1)(good_camera())
    f32 = S.snerg_grid(64, 8, 8, S.SNERG_F32, FAKE.value, FAKE.value, 50.0, 0)
    for kw in (dict(unpremultiply=True), dict(unpremultiply=True, mlp_grad_only=True)):
        o = S.make_opts(**kw)
        rc = lib.snerg_render_backward(None, ctypes.byref(f32), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE,
                                       FAKE, FAKE, FAKE, FAKE, None)
        assert rc == S.SNERG_ERR_UNSUPPORTED and "UNPREMULTIPLY" in last_error()
    o = S.make_opts(nn_gate=True)   # the gate has a backward
    rc = lib.snerg_render_backward(None, ctypes.byref(f32), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE,
                                   FAKE, FAKE, FAKE, FAKE, None)
    assert rc == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()


def test_per_sample_mlp_is_forward_only_without_aux():
    o = S.make_opts(per_sample_mlp=True)
    assert call_render(opts=o) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert call_render(opts=o, out=FAKE) == S.SNERG_ERR_INVALID_ARG
    lib = S.lib()
    grid = S.snerg_grid(64, 8, 8, S.SNERG_U8, FAKE.value, FAKE.value, 50.0, 0)
    cams = (S.snerg_camera * 1)(good_camera())
    rc = lib.snerg_render(None, ctypes.byref(grid), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE, None)
    assert rc == S.SNERG_ERR_UNSUPPORTED and "aux" in last_error()
    f32 = S.snerg_grid(64, 8, 8, S.SNERG_F32, FAKE.value, FAKE.value, 50.0, 0)
    rc = lib.snerg_render_backward(None, ctypes.byref(f32), FAKE, cams, 1, None, 32, ctypes.byref(o), FAKE, FAKE,
                                   FAKE, FAKE, FAKE, FAKE, None)
    assert rc == S.SNERG_ERR_UNSUPPORTED and "PER_SAMPLE" in last_error()


def test_bake_entry_point_validation():
    lib = S.lib()
    cams = (S.snerg_camera * 1)(good_camera())
    ok = S.make_bake_opts()
    cull = lambda N=64, B=8, o=ok, sg=FAKE, c=cams, nc=1, ind=FAKE: lib.snerg_bake_cull(
        None, N, B, sg, c, nc, ctypes.byref(o) if o is not None else None, None, None, ind,
        ctypes.byref(ctypes.c_int32()), None)
    assert cull() == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()       # got past every check
    assert cull(o=None) == S.SNERG_ERR_INVALID_ARG
    assert cull(B=6) == S.SNERG_ERR_UNSUPPORTED
    assert cull(N=60) == S.SNERG_ERR_UNSUPPORTED
    assert cull(N=4096, B=32) == S.SNERG_ERR_UNSUPPORTED                          # N/B > 64
    for bad in (S.make_bake_opts(tau_alpha=1.0), S.make_bake_opts(tau_alpha=-0.1), S.make_bake_opts(tau_vis=0.0),
                S.make_bake_opts(tau_vis=1.5), S.make_bake_opts(tau_vis=float("nan")),
                S.make_bake_opts(sigma_scale=0.0), S.make_bake_opts(sigma_scale=float("inf"))):
        assert cull(o=bad) == S.SNERG_ERR_INVALID_ARG
    assert cull(sg=None) == S.SNERG_ERR_INVALID_ARG and "sigma" in last_error()
    assert cull(ind=None) == S.SNERG_ERR_INVALID_ARG
    assert cull(nc=0) == S.SNERG_ERR_INVALID_ARG
    assert cull(c=None) == S.SNERG_ERR_INVALID_ARG
    quant = lambda n=4, o=ok, sg=FAKE, out=FAKE: lib.snerg_bake_quantize(
        None, 64, 8, sg, FAKE, FAKE, FAKE, n, ctypes.byref(o), out, FAKE, FAKE, None)
    assert quant() == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert quant(n=-1) == S.SNERG_ERR_INVALID_ARG
    assert quant(n=513) == S.SNERG_ERR_INVALID_ARG                               # more than (N/B)^3
    assert quant(sg=None) == S.SNERG_ERR_INVALID_ARG and "NULL" in last_error()
    assert quant(out=None) == S.SNERG_ERR_INVALID_ARG and "NULL" in last_error()
    assert quant(n=0, sg=None, out=None) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert quant(o=S.make_bake_opts(sigma_scale=-1.0)) == S.SNERG_ERR_INVALID_ARG


def test_timing_entry_point_validation():
    lib = S.lib()
    n = ctypes.c_int32(0)
    buf = (ctypes.c_float * 4)()
    assert lib.snerg_timing_enable(None, 1) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
    assert lib.snerg_timing_enable(None, -1) == S.SNERG_ERR_INVALID_ARG and "on must be" in last_error()
    assert lib.snerg_timing_read(None, buf, 4, None) == S.SNERG_ERR_INVALID_ARG
    assert lib.snerg_timing_read(None, None, 4, ctypes.byref(n)) == S.SNERG_ERR_INVALID_ARG
    assert lib.snerg_timing_read(None, buf, -1, ctypes.byref(n)) == S.SNERG_ERR_INVALID_ARG
    assert lib.snerg_timing_read(None, buf, 4, ctypes.byref(n)) == S.SNERG_ERR_INVALID_ARG and "handle" in last_error()
