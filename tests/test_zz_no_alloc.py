"""snerg_render_noalloc (every scratch buffer in the library's fixed device
array, no allocation) against snerg_render on the same inputs: the same
kernels, so the results must agree bit for bit, in every launch mode, with
aux, and on two calls in a row whose second is smaller (the array keeps the
first call's contents).  Limits and rejected options fail on the host."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2103_14645_amd import snerg as S
from tests.gpu_helpers import device_grid, handle, oracle_variants, parity_error, say

pytestmark = pytest.mark.gpu


def both(dg, mlp, cams, ids=None, with_aux=False, **kw):
    """(snerg_render, snerg_render_noalloc) outputs [and aux] on the same inputs."""
    h = handle()
    opts = S.make_opts(**kw)
    m = S.mlp_tensor(mlp)
    carr = S.make_cameras(cams)
    idt = torch.from_numpy(np.asarray(ids, np.int64)).cuda() if ids is not None else None
    n = len(ids) if ids is not None else sum(c.n_rays for c in cams)
    res = []
    for fn in (S.snerg_render, S.snerg_render_noalloc):
        out = torch.full((n, 4), float("nan"), device="cuda")
        aux = torch.full((n, 8), float("nan"), device="cuda") if with_aux else None
        fn(h, dg.struct(), m, carr, idt, n, opts, out, aux)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), aux.cpu().numpy() if with_aux else None))
    return res


def tiny_case(n_occ, seed, sizes):
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    cams = [W.orbit_camera(w, h, seed=seed + i) for i, (w, h) in enumerate(sizes)]
    cams.append(W.look_at((0.05, -0.1, 0.02), 24, 16, 90.0, target=(0.9, 0.3, -0.2)))  # inside the grid
    return g, cams, W.mlp_weights(seed + 2)


@pytest.mark.parametrize("kw", [dict(), dict(persistent=True), dict(fp16=True), dict(fp16=True, persistent=True),
                                dict(mlp_on=False), dict(nn_gate=True)])
def test_noalloc_equals_render_two_calls(kw):
    say(f"noalloc vs render {kw}: a large call, then a smaller one")
    g, cams, mlp = tiny_case(64, 1, [(64, 64), (37, 23), (50, 9)])
    dg = device_grid(g)
    (r1, a1), (n1, b1) = both(dg, mlp, cams, with_aux=True, **kw)
    assert np.array_equal(r1, n1) and np.array_equal(a1, b1)
    small = [W.orbit_camera(13, 7, seed=9)]
    (r2, _), (n2, _) = both(dg, mlp, small, **kw)
    assert np.array_equal(r2, n2)
    # and against the oracle (the bar of the plain render)
    if not kw.get("fp16") and not kw.get("nn_gate"):
        err, _ = parity_error(n2, oracle_variants(O.OracleGrid(g), mlp, small, mlp_on=kw.get("mlp_on", True)))
        say(f"  small call max err vs oracle {err.max():.2e}")
        assert err.max() <= 1e-4


def test_noalloc_ray_list_and_float_grid():
    g, cams, mlp = tiny_case(120, 4, [(40, 30)])
    n = sum(c.n_rays for c in cams)
    ids = np.random.default_rng(2).permutation(n)[: n // 2]
    dg = device_grid(g)
    (r, a), (q, b) = both(dg, mlp, cams, ids=ids, with_aux=True)
    assert np.array_equal(r, q) and np.array_equal(a, b)
    vals = tuple((x / 255.0).astype(np.float32) for x in (g.dens, g.rgb, g.feat))
    dgf = device_grid(g, vals)
    (r, _), (q, _) = both(dgf, mlp, cams)
    assert np.array_equal(r, q)


def test_noalloc_plain512_frame():
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    say("noalloc: the plain512 frame, then a tiny frame on the same grid")
    dg = device_grid(g)
    (r, _), (q, _) = both(dg, mlp, cams)
    assert np.array_equal(r, q)
    (r, _), (q, _) = both(dg, mlp, [W.orbit_camera(16, 16, seed=3)])
    assert np.array_equal(r, q)


def test_noalloc_limits_fail_on_the_host():
    g, cams, mlp = tiny_case(8, 0, [(8, 8)])
    dg = device_grid(g)
    h = handle()
    m = S.mlp_tensor(mlp)
    out = torch.empty((4, 4), device="cuda")
    with pytest.raises(S.SnergError) as e:
        S.snerg_render_noalloc(h, dg.struct(), m, S.make_cameras(cams), None, sum(c.n_rays for c in cams),
                               S.make_opts(graph=True), out)
    assert e.value.code == S.SNERG_ERR_UNSUPPORTED
    many = [W.orbit_camera(1, 1, seed=1)] * 1025
    with pytest.raises(S.SnergError) as e:
        S.snerg_render_noalloc(h, dg.struct(), m, S.make_cameras(many), None, 1025, S.make_opts(), out)
    assert e.value.code == S.SNERG_ERR_WORKSPACE
    big = [W.orbit_camera(16384, 8192, seed=1)] * 2   # 4.2 M tiles of 64 pixels
    with pytest.raises(S.SnergError) as e:
        S.snerg_render_noalloc(h, dg.struct(), m, S.make_cameras(big), None, 2 * 16384 * 8192, S.make_opts(), out)
    assert e.value.code == S.SNERG_ERR_WORKSPACE
