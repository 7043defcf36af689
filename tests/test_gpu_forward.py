"""GPU parity of the forward render and the visit trace against the FP64 oracle.

Bars: visit lists, counts and per-ray counters bit-exact; FP32 RGBA within
1e-4 absolute; the FP16-MFMA MLP path within 2e-3 absolute.  Rays whose
early-stop decision lies within a relative 1e-5 of t_stop may match either
oracle branch.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2103_14645_amd import snerg as S
from tests.gpu_helpers import device_grid, gpu_render, handle, oracle_variants, parity_error, say

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4
TOL_F16 = 2e-3


def tiny_case(n_occ, seed):
    g = W.tiny_grid(n_occupied=n_occ, seed=seed)
    cams = [W.orbit_camera(64, 64, seed=seed + 1), W.orbit_camera(37, 23, seed=seed + 2),
            W.look_at((0.3, -1.7, 0.9), 19, 41, 53.0)]
    return g, cams, W.mlp_weights(seed + 2)


@pytest.mark.parametrize("n_occ,seed,early,mlp_on", [(8, 0, True, True), (64, 1, True, True),
                                                     (200, 2, True, True), (200, 3, False, True),
                                                     (120, 4, True, False)])
def test_tiny_all_rays_fp32(n_occ, seed, early, mlp_on):
    say(f"tiny fp32 n_occ={n_occ} seed={seed} early={early} mlp={mlp_on}")
    g, cams, mlp = tiny_case(n_occ, seed)
    bg = tuple(np.random.default_rng(seed).uniform(0, 1, 3))
    dg = device_grid(g)
    gpu = gpu_render(dg, mlp, cams, bg=bg, early_stop=early, mlp_on=mlp_on)
    og = O.OracleGrid(g)
    err, flagged = parity_error(gpu, oracle_variants(og, mlp, cams, bg=bg, early_stop=early, mlp_on=mlp_on))
    say(f"  rays={len(err)} max_err={err.max():.3e} near_threshold={flagged}")
    assert err.max() <= TOL_F32


def test_tiny_launch_modes_agree_bitwise():
    g, cams, mlp = tiny_case(64, 1)
    dg = device_grid(g)
    base = gpu_render(dg, mlp, cams)
    n = base.shape[0]
    for kw in (dict(persistent=True), dict(persistent=True, graph=True), dict(graph=True)):
        say(f"launch mode {kw}")
        assert np.array_equal(gpu_render(dg, mlp, cams, **kw), base)
    ids = np.random.default_rng(0).permutation(n)[: n // 3]
    say("list mode")
    assert np.array_equal(gpu_render(dg, mlp, cams, ids=ids), base[ids])
    assert np.array_equal(gpu_render(dg, mlp, cams), base)  # deterministic


@pytest.mark.parametrize("tile", [(8, 8, 1, 2), (16, 4, 2, 4), (4, 16, 4, 8), (32, 2, 1, 16), (64, 1, 2, 1)])
def test_tuning_shapes_agree_bitwise(tile):
    g, cams, mlp = tiny_case(64, 1)
    dg = device_grid(g)
    h = handle()
    base = gpu_render(dg, mlp, cams)
    old = S.snerg_get_tuning(h)
    try:
        S.snerg_set_tuning(h, *tile)
        say(f"tuning {tile}")
        assert np.array_equal(gpu_render(dg, mlp, cams), base)
        assert np.array_equal(gpu_render(dg, mlp, cams, persistent=True, graph=True), base)
    finally:
        S.snerg_set_tuning(h, *old)


@pytest.mark.parametrize("n_occ,seed,early", [(8, 0, False), (200, 2, False), (200, 2, True), (64, 5, True)])
def test_visits_and_counters_bit_exact(n_occ, seed, early):
    say(f"trace n_occ={n_occ} seed={seed} early={early}")
    g, cams, _ = tiny_case(n_occ, seed)
    dg = device_grid(g)
    vis, cnt, ctr = S.trace_visits(handle(), dg, cams, opts=S.make_opts(early_stop=early, mlp_on=False),
                                   max_visits=64)
    torch.cuda.synchronize()
    vis, cnt, ctr = vis.cpu().numpy(), cnt.cpu().numpy(), ctr.cpu().numpy()
    og = O.OracleGrid(g)
    ovis, ocnt = O.trace_visits(og, cams, early_stop=early, max_visits=64)
    octr = O.render(og, None, cams, early_stop=early, mlp_on=False)["counters"][:, :5]
    if early:
        # rays whose stop decision is within the band may differ in their tail
        alt = [O.render(og, None, cams, early_stop=True, mlp_on=False, t_stop=1e-3 * f)["counters"][:, :5]
               for f in (1 - 1e-5, 1 + 1e-5)]
        same = np.all(octr == alt[0], axis=1) & np.all(octr == alt[1], axis=1)
    else:
        same = np.ones(len(cnt), bool)
    say(f"  rays={len(cnt)} near_threshold={int((~same).sum())} max_count={int(ocnt.max())}")
    assert np.array_equal(cnt[same], ocnt[same])
    assert np.array_equal(ctr[same], octr[same])
    assert np.array_equal(vis[same], ovis[same])


def test_plain512_frame_sampled_rays():
    say("plain512: full 800x800 frame, 12000 sampled rays vs oracle")
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    dg = device_grid(g)
    frame = gpu_render(dg, mlp, cams)
    rng = np.random.default_rng(7)
    ids = np.sort(rng.choice(frame.shape[0], 12000, replace=False))
    og = O.OracleGrid(g)
    err, flagged = parity_error(frame[ids], oracle_variants(og, mlp, cams, ids=ids))
    say(f"  max_err={err.max():.3e} near_threshold={flagged} hit_frac={(frame[ids, 3] > 0).mean():.3f}")
    assert err.max() <= TOL_F32
    assert np.array_equal(gpu_render(dg, mlp, cams, ids=ids), frame[ids])
    vis, cnt, ctr = S.trace_visits(handle(), dg, cams, ray_ids=torch.from_numpy(ids).cuda(),
                                   opts=S.make_opts(early_stop=False, mlp_on=False), max_visits=48)
    torch.cuda.synchronize()
    ovis, ocnt = O.trace_visits(og, cams, ray_ids=ids, early_stop=False, max_visits=48)
    assert np.array_equal(cnt.cpu().numpy(), ocnt) and np.array_equal(vis.cpu().numpy(), ovis)


def test_plain512_whole_frame_vs_oracle():
    # every one of the 640,000 rays of the headline frame, as the benchmark
    # renders it (tiled launch, heavy-first order), against the FP64 oracle
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    dg = device_grid(g)
    frame = gpu_render(dg, mlp, cams)
    say(f"plain512: whole frame, {frame.shape[0]} rays vs oracle")
    err, flagged = parity_error(frame, oracle_variants(O.OracleGrid(g), mlp, cams))
    say(f"  max_err={err.max():.3e} near_threshold={flagged}")
    assert err.max() <= TOL_F32


def test_plain512_grid_other_cameras_sampled_rays():
    # the headline grid from four more viewpoints (radii 1.3 to 3, one camera
    # inside the bounding box's corner region, elevations -40 to 70 degrees),
    # all cameras in one tiled launch: 6,000 sampled rays vs the oracle
    cfg = W.config("plain512")
    g, mlp = cfg["grid"], cfg["mlp"]
    cams = [W.look_at(W.orbit_eye(r, el, a), 200, 150, fov)
            for r, el, a, fov in ((1.3, -40.0, 0.4, 60.0), (2.0, 70.0, 2.1, 39.0), (3.0, 5.0, 4.0, 25.0),
                                  (1.55, 20.0, 5.5, 90.0))]
    n = sum(c.n_rays for c in cams)
    say(f"plain512 grid, {len(cams)} other cameras, {n} rays")
    dg = device_grid(g)
    frame = gpu_render(dg, mlp, cams)
    ids = np.sort(np.random.default_rng(17).choice(n, 6000, replace=False))
    err, flagged = parity_error(frame[ids], oracle_variants(O.OracleGrid(g), mlp, cams, ids=ids))
    say(f"  max_err={err.max():.3e} near_threshold={flagged} hit_frac={(frame[ids, 3] > 0).mean():.3f}")
    assert err.max() <= TOL_F32
    assert (frame[ids, 3] > 0).mean() > 0.2  # the views do see the shell


@pytest.mark.parametrize("name", ["tiny", "batched1024"])
def test_fp16_mlp_error_report(name):
    cfg = W.config(name)
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    dg = device_grid(g)
    say(f"fp16 {name}: persistent graph launch over {sum(c.n_rays for c in cams)} rays")
    frame = gpu_render(dg, mlp, cams, fp16=True, persistent=True, graph=True)
    n = frame.shape[0]
    ids = np.sort(np.random.default_rng(3).choice(n, min(n, 8000), replace=False))
    og = O.OracleGrid(g)
    err, flagged = parity_error(frame[ids], oracle_variants(og, mlp, cams, ids=ids))
    f32 = gpu_render(dg, mlp, cams, ids=ids)
    err32, _ = parity_error(f32, oracle_variants(og, mlp, cams, ids=ids))
    say(f"  fp16 max_err={err.max():.3e} fp32 max_err={err32.max():.3e} near_threshold={flagged}")
    assert err.max() <= TOL_F16
    assert err32.max() <= TOL_F32
    # the tiled graph launch (the one the batched benchmark keeps) gives the same bits
    tiled = gpu_render(dg, mlp, cams, fp16=True, graph=True)
    assert np.array_equal(tiled, frame)


def test_float32_grid_forward():
    say("float32 shadow grid forward")
    g, cams, mlp = tiny_case(120, 6)
    rng = np.random.default_rng(1)
    d = g.dens / 255.0
    vals = (np.where(d > 0, d + 0.01 * rng.uniform(-1, 1, d.shape), 0.0).astype(np.float32),
            (g.rgb / 255.0 + 0.01 * rng.uniform(-1, 1, g.rgb.shape)).astype(np.float32),
            (g.feat / 255.0 + 0.01 * rng.uniform(-1, 1, g.feat.shape)).astype(np.float32))
    dg = device_grid(g, vals)
    gpu = gpu_render(dg, mlp, cams)
    og = O.OracleGrid(g, values=vals)
    err, _ = parity_error(gpu, oracle_variants(og, mlp, cams))
    say(f"  max_err={err.max():.3e}")
    assert err.max() <= TOL_F32


def test_empty_grid_and_out_of_range_ids():
    g, cams, mlp = tiny_case(64, 1)
    bg = (0.1, 0.2, 0.3)
    empty = W.Grid(g.N, g.B, np.full_like(g.indirection, -1), g.dens, g.rgb, g.feat)
    say("empty indirection")
    out = gpu_render(device_grid(empty), mlp, cams, bg=bg)
    assert np.array_equal(out, np.tile(np.array([0.1, 0.2, 0.3, 0.0], np.float32), (out.shape[0], 1)))
    # atlas ids >= n_blocks read as empty macroblocks
    bad = W.Grid(g.N, g.B, g.indirection.copy(), g.dens, g.rgb, g.feat)
    occ = np.flatnonzero(bad.indirection >= 0)
    bad.indirection[occ[::3]] = 10 ** 6
    ref = W.Grid(g.N, g.B, g.indirection.copy(), g.dens, g.rgb, g.feat)
    ref.indirection[occ[::3]] = -1
    say("out-of-range atlas ids")
    assert np.array_equal(gpu_render(device_grid(bad), mlp, cams), gpu_render(device_grid(ref), mlp, cams))


def test_zero_rays_is_a_no_op():
    g, cams, mlp = tiny_case(8, 0)
    dg = device_grid(g)
    out = torch.full((1, 4), 7.0, device="cuda")
    S.snerg_render(handle(), dg.struct(), S.mlp_tensor(mlp), S.make_cameras(cams),
                   torch.zeros(1, dtype=torch.int64, device="cuda"), 0, S.make_opts(), out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)


def test_large1024_all_cameras_one_launch_sampled():
    # 64 cameras at 1920x1080 in one persistent graph launch with the FP16 MLP,
    # the configuration the benchmark times; 4,000 sampled rays vs the oracle.
    cfg = W.config("large1024")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    n = sum(c.n_rays for c in cams)
    say(f"large1024: {len(cams)} cameras, {n} rays, {g.n_blocks} blocks")
    dg = device_grid(g)
    out = S.render(handle(), dg, S.mlp_tensor(mlp), cams,
                   opts=S.make_opts(fp16=True, persistent=True, graph=True))
    ids = np.sort(np.random.default_rng(11).choice(n, 4000, replace=False))
    got = out[torch.from_numpy(ids).cuda()].cpu().numpy()
    del out
    og = O.OracleGrid(g)
    err, flagged = parity_error(got, oracle_variants(og, mlp, cams, ids=ids))
    say(f"  fp16 max_err={err.max():.3e} near_threshold={flagged} hit_frac={(got[:, 3] > 0).mean():.3f}")
    assert err.max() <= TOL_F16


def test_kernel_timing_ring():
    say("kernel timing: one event pair per timed render, every launch mode, sampling stride")
    g, cams, mlp = tiny_case(64, 1)
    dg = device_grid(g)
    h = handle()
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), device="cuda")
    m = S.mlp_tensor(mlp)
    carr = S.make_cameras(cams)
    ids = torch.arange(0, n, 3, device="cuda")
    S.snerg_timing_enable(h, True)
    for kw in (dict(), dict(persistent=True), dict(persistent=True, graph=True)):
        S.snerg_render(h, dg.struct(), m, carr, None, n, S.make_opts(**kw), out)
    S.snerg_render(h, dg.struct(), m, carr, ids, ids.numel(), S.make_opts(), out)
    ms = S.snerg_timing_read(h)
    S.snerg_timing_enable(h, False)
    S.snerg_render(h, dg.struct(), m, carr, None, n, S.make_opts(), out)
    assert len(ms) == 4 and all(0.0 < t < 1000.0 for t in ms)
    assert len(S.snerg_timing_read(h)) == 4  # disabled: nothing more recorded
    S.snerg_timing_enable(h, True)
    assert S.snerg_timing_read(h) == []
    # every 3rd call: calls 1, 4 and 7 of seven are timed, in every launch mode
    S.snerg_timing_enable(h, 3)
    for i in range(7):
        kw = (dict(), dict(persistent=True), dict(persistent=True, graph=True))[i % 3]
        S.snerg_render(h, dg.struct(), m, carr, None, n, S.make_opts(**kw), out)
    ms = S.snerg_timing_read(h)
    assert len(ms) == 3 and all(0.0 < t < 1000.0 for t in ms)
    S.snerg_timing_enable(h, False)


def _cluster_grid(N, B, radius, seed):
    """Occupied macroblocks in a cube of (2 radius)^3 blocks around the centre
    (random bytes, a quarter of the densities zero), atlas ids permuted."""
    rng = np.random.default_rng(seed)
    G = N // B
    lo, hi = max(0, G // 2 - radius), min(G, G // 2 + radius)
    bz, by, bx = np.meshgrid(np.arange(lo, hi), np.arange(lo, hi), np.arange(lo, hi), indexing="ij")
    lin = ((bz * G + by) * G + bx).reshape(-1)
    n = lin.size
    ind = np.full(G ** 3, -1, np.int32)
    ind[lin] = rng.permutation(n).astype(np.int32)
    dens = rng.integers(0, 256, (n, B, B, B), dtype=np.uint8)
    dens[rng.random(dens.shape) < 0.25] = 0
    rgb = rng.integers(0, 256, (n, B, B, B, 3), dtype=np.uint8)
    feat = rng.integers(0, 256, (n, B, B, B, 4), dtype=np.uint8)
    return W.Grid(N, B, ind, dens, rgb, feat)


def _axis_camera(N, yv, zv):
    # one ray along +x through the point (yv, zv) in voxel units (may sit on a face)
    y = yv * 2.0 / N - 1.0
    z = zv * 2.0 / N - 1.0
    fwd, up = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    return W.Camera(np.array([-2.5, y, z]), fwd, np.cross(fwd, up), up, 1, 1, 1.0)


@pytest.mark.parametrize("N,B,radius,fov", [(4096, 64, 1, 3.0), (2, 2, 1, 25.0), (96, 32, 2, 25.0)])
def test_extreme_grid_shapes(N, B, radius, fov):
    # N = 4096, B = 64: the largest grid whose occupancy table (64^3 blocks,
    # 64 KB) fits in LDS, and lattice coordinates up to 2^28; N = 2: a single
    # macroblock of 8 voxels; G = 3: an odd block count.  Cameras outside and
    # inside the grid, and axis-aligned rays through voxel centres and exactly
    # along macroblock faces.
    say(f"extreme shape N={N} B={B}")
    g = _cluster_grid(N, B, radius, seed=N + B)
    mid = N / 2.0
    cams = [W.orbit_camera(48, 40, fov_deg=fov, seed=1),
            W.look_at((0.05, -0.1, 0.02), 32, 24, 90.0, target=(0.9, 0.3, -0.2)),   # eye inside the grid
            _axis_camera(N, mid + 0.5, mid + 0.5), _axis_camera(N, mid, mid), _axis_camera(N, mid - B, mid + 0.25)]
    mlp = W.mlp_weights(3)
    n = sum(c.n_rays for c in cams)
    ids = None
    dg = device_grid(g)
    gpu = gpu_render(dg, mlp, cams, ids=ids)
    og = O.OracleGrid(g)
    err, flagged = parity_error(gpu, oracle_variants(og, mlp, cams, ids=ids))
    say(f"  rays={len(err)} max_err={err.max():.3e} near_threshold={flagged} hit={np.mean(gpu[:, 3] > 0):.2f}")
    assert err.max() <= TOL_F32
    assert np.mean(gpu[:, 3] > 0) > 0.05
    # visit lists bit-exact without early stop
    nr = n
    idt = torch.arange(n, device="cuda")
    visits = torch.full((nr, 32), -7, dtype=torch.int32, device="cuda")
    counts = torch.empty(nr, dtype=torch.int32, device="cuda")
    S.snerg_trace_visits(handle(), dg.struct(), S.make_cameras(cams), idt, nr, S.make_opts(early_stop=False),
                         32, visits, counts)
    torch.cuda.synchronize()
    ovis, ocnt = O.trace_visits(og, cams, ray_ids=ids, early_stop=False, max_visits=32)
    assert np.array_equal(counts.cpu().numpy(), ocnt)
    gv = visits.cpu().numpy()
    for r in range(nr):
        k = min(int(ocnt[r]), 32)
        assert np.array_equal(gv[r, :k], ovis[r, :k]), r


def test_autotune_records_launch_shape_by_workload(tmp_path):
    say("autotune: launch shapes recorded by workload signature, saved and loaded")
    g, cams, mlp = tiny_case(64, 1)
    dg = device_grid(g)
    h = S.Handle()
    opts = S.make_opts()
    carr = S.make_cameras(cams)
    other = S.make_cameras([W.orbit_camera(31, 17, seed=4)])
    m = S.mlp_tensor(mlp)
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), device="cuda")
    _, found = S.snerg_tuning_lookup(h, dg.struct(), carr, opts)
    assert not found
    best, _ = S.snerg_autotune(h, dg.struct(), m, carr, opts, out, candidates=[(16, 4, 2, 8), (4, 16, 1, 8)], reps=1)
    assert S.snerg_tuning_lookup(h, dg.struct(), carr, opts) == (best, True)
    assert not S.snerg_tuning_lookup(h, dg.struct(), other, opts)[1]
    assert not S.snerg_tuning_lookup(h, dg.struct(), carr, S.make_opts(fp16=True))[1]
    # the handle's tuning changes renders of other workloads only
    S.snerg_set_tuning(h, 32, 2, 1, 2)
    assert S.snerg_tuning_lookup(h, dg.struct(), carr, opts) == (best, True)
    assert S.snerg_tuning_lookup(h, dg.struct(), other, opts) == ((32, 2, 1, 2), False)
    path = tmp_path / "tune.txt"
    S.snerg_tuning_save(h, path)
    h2 = S.Handle()
    S.snerg_tuning_load(h2, path)
    assert S.snerg_tuning_lookup(h2, dg.struct(), carr, opts) == (best, True)
    # every launch shape renders the same bits
    base = gpu_render(dg, mlp, cams)
    S.snerg_render(h2, dg.struct(), m, carr, None, n, opts, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), base)
    # a malformed file is rejected and adds nothing
    bad = tmp_path / "bad.txt"
    bad.write_text("0123 8 8 4\n")
    h3 = S.Handle()
    with pytest.raises(S.SnergError):
        S.snerg_tuning_load(h3, bad)
    assert not S.snerg_tuning_lookup(h3, dg.struct(), carr, opts)[1]
    bad.write_text("0123 7 7 4 8\n")  # 7 x 7 is not a 64-lane tile
    with pytest.raises(S.SnergError):
        S.snerg_tuning_load(h3, bad)
