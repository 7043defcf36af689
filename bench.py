"""Throughput of the SNeRG render path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs plain,batched,adjoint,large,finetune,nondeferred,bake]
    python bench.py --legs plain,copy --no-cpu-baseline   # adds the copy-kernel calibration launches
    python bench.py --source-hash                          # hash of the kernel sources

Headline (value): forward Mrays/s of the plain FP32 path on the 512^3 grid
(B = 32, ~10.6% occupied procedural shell) for one 800x800 camera, with
inputs resident in device memory; fps = value / 0.64.  Further legs, each
timed the same way: the batched FP16-MFMA-MLP forward (1024^3 grid, 16
cameras of mixed size in one launch replayed from a HIP graph, tiled or
persistent as the autotuner finds faster)
with its max-abs error against the FP64 oracle, the adjoint (8 views at
800x800 on a float32 shadow of the 512^3 grid, forward + backward), the
large case (64 x 1920x1080 in one launch, then 65,536-ray minibatch forward
+ backward), and fine-tuning of the deferred network on the fixed uint8
grid (render, squared error, MLP backward, Adam per 65,536-ray step), and
the non-deferred ablation (the network on every sample, FP32 and FP16 MFMA),
and baking a dense 512^3 field (both culls from 100 training views at
800x800, then the 8-bit atlas).
Prints one JSON line on stdout; progress goes to stderr.

ms_per_step is the whole snerg_render call (the tile-order pre-pass and the
render kernel).  The render kernel is bound by vector-ALU instruction issue
(the committed counters: VALUs about 70% busy, HBM traffic about a tenth of
peak), so roofline is the ALU roofline: the algorithmic FP32 work of the
frame (per composited sample and per ray, from the march's exact counters)
over the render kernel's own duration, from HIP events the library records
around that launch during the timed frames (snerg_timing_enable/read),
against the FP32 vector peak.  roofline.hbm gives the algorithmic bytes of
the paper's accounting as an effective rate, and the measured HBM traffic
(FETCH_SIZE + WRITE_SIZE of one launch, from profiles/counters_by_kernel.md)
as a rate; both counter-derived figures are reported only while the hash of
the kernel sources equals the one recorded there, else null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP16_PEAK_TFLOPS = 2500.0  # dense FP16 MFMA
# FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (fused multiply-add) x 2 (packed FP32)
# x 2.4 GHz = 157.3 TFLOP/s; this build emits no packed FP32 instructions, so 78.6 TFLOP/s is
# the most its code can issue
FP32_PEAK_TFLOPS = 157.3
FP32_PEAK_UNPACKED_TFLOPS = 78.6
MLP_FLOP = 2 * (34 * 16 + 16 * 16 + 16 * 3)
# algorithmic FP32 work of the forward (Eq. 2, 5-7, Section 5.2): per composited sample 15 FLOP
# of trilinear weights, 8 channels x 8 corners multiply-adds (128) and 20 of compositing; per
# ray whose network runs, the network (1,696), 36 for the direction encoding, 9 for the sigmoid
# and 7 for the output
SAMPLE_FLOP = 15 + 128 + 20
RAY_FLOP = MLP_FLOP + 36 + 9 + 7
KERNEL_SOURCES = ("render.hip", "render_ps.hip", "backward.hip", "march.h", "mlp.h", "snerg_dev.h",
                  "snerg_launch.h", "api.cpp")  # the kernels and their launch order
# the sources each counter figure describes: the forward render kernels, and the adjoint's
SOURCE_GROUPS = {"render": ("render.hip", "render_ps.hip", "march.h", "mlp.h", "snerg_dev.h", "snerg_launch.h"),
                 "backward": ("backward.hip", "march.h", "mlp.h", "snerg_dev.h", "snerg_launch.h")}
LEG_GROUP = {"plain512": "render", "batched1024": "render", "large1024": "render", "adjoint512_fwd": "render",
             "nondeferred_fp32": "render", "nondeferred_fp16": "render", "large1024_mb_fwd": "render",
             "adjoint512_bwd": "backward", "adjoint512_mlp_bwd": "backward", "large1024_mb_mlp_bwd": "backward",
             "large1024_mb_bwd": "backward", "large1024_mb_bwd_patch": "backward", "large1024_mb_record": "backward",
             "large1024_mb_bwd_packed": "backward"}
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "counters_by_kernel.md")
COPY_BYTES = 1 << 30
TIMING_EVERY = 4  # frames per kernel-timed frame in the plain leg's timed region


def kernel_source_hash(names=KERNEL_SOURCES):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2103_14645_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def group_hashes():
    return {g: kernel_source_hash(names) for g, names in SOURCE_GROUPS.items()}


def file_sha256(path):
    h = hashlib.sha256()
    with open(path, "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def committed_counters():
    """"key = value" figures of the committed counter summary (measured HBM
    traffic per launch, instruction and busy fractions), keeping those of
    the legs whose kernel sources hash to the value recorded with them:
    counters taken on other code say nothing about this code."""
    try:
        kv = {}
        for line in open(COUNTER_SUMMARY):
            if " = " in line and not line.startswith((" ", "|", "#")):
                k, v = line.split(" = ", 1)
                kv[k.strip().strip("`")] = v.strip().strip("`")
    except OSError:
        return {}
    now = group_hashes()
    valid = {g for g in now if kv.get(f"sources_sha256.{g}") == now[g]}
    out = {}
    for k, v in kv.items():
        leg = k.split(".", 1)[1] if k.startswith("traffic.") else k.split(".", 1)[0]
        grp = LEG_GROUP.get(leg)
        if grp is None or grp in valid:
            out[k] = v
    return out if valid else {}


def counter(kv, key, cast=float):
    try:
        return cast(kv[key])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_launches(fn, steps, warmup, torch):
    """Runs fn warmup times, then times `steps` calls with events on the
    current stream (the stream the library launches on).  Returns ms/call."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def launch_spread(fn, n, torch):
    """p10 / p50 / p90 of n individually event-timed launches (ms)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for e0, e1 in ev:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    t = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return [round(float(np.percentile(t, q)), 4) for q in (10, 50, 90)]


def host_cpu():
    """CPU model as lscpu reports it (with family/model/stepping, which name
    the part when the model string is generic), else /proc/cpuinfo's."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("Model name"):
            return (f"{kv['Model name']} (family {kv.get('CPU family', '?')}, model {kv.get('Model', '?')}, "
                    f"stepping {kv.get('Stepping', '?')}; {kv.get('Socket(s)', '?')} socket(s), "
                    f"{kv.get('Thread(s) per core', '?')} thread(s) per core)")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(O, og, mlp, cams, ids, threads):
    """Oracle Mrays/s on the given ray ids with `threads` OpenMP threads."""
    t0 = time.perf_counter()
    out = O.render(og, mlp, cams, ray_ids=ids, threads=threads)["rgba"]
    return out, len(ids) / (time.perf_counter() - t0) / 1e6


def frame_counters(S, h, dg, cams):
    """Exact per-ray counters of the march (GPU trace, bit-identical to the oracle's)."""
    import torch
    _, _, ctr = S.trace_visits(h, dg, cams, opts=S.make_opts(mlp_on=False), max_visits=0)
    torch.cuda.synchronize()
    c = ctr.cpu().numpy().astype(np.int64)
    return dict(blocks=int(c[:, 0].sum()), occupied=int(c[:, 1].sum()), inblock=int(c[:, 2].sum()),
                active=int(c[:, 3].sum()), rays=int(c.shape[0]), gated=int((c[:, 3] > 0).sum()))


def algorithmic_bytes(cnt, value_bytes=8, out_bytes=16):
    """The method's own traffic per the paper's accounting (Appendix A): one
    indirection entry per macroblock traversed (4 B), one density byte per
    in-block sample, 8 corners x value_bytes per composited sample (8 B for
    the uint8 atlas, 32 B for the float32 shadow), out_bytes per ray."""
    return 4 * cnt["blocks"] + cnt["inblock"] + 8 * value_bytes * cnt["active"] + out_bytes * cnt["rays"]


def algorithmic_flop(cnt, network=True):
    """Algorithmic FP32 work of the forward: SAMPLE_FLOP per composited
    sample, RAY_FLOP per ray whose deferred network runs."""
    return SAMPLE_FLOP * cnt["active"] + (RAY_FLOP * cnt["gated"] if network else 0)


def tune_launch(S, h, grid, m, carr, out, reps, tiles=None, persistent=None, cache=None):
    """Autotunes the FP16 graph launch in both launch modes (tiled wavefronts
    issued by the hardware, or persistent workgroups pulling tiles from a
    counter) and keeps the faster: (opts, tuning, ms, mode, modes).  With a
    launch-shape cache file (snerg_tuning_save's format), a shape recorded
    there for this workload is only timed, not searched again, and the file
    is rewritten with this handle's shapes afterwards."""
    import torch
    if cache and os.path.exists(cache):
        S.snerg_tuning_load(h, cache)
    best = None
    modes = {}
    n = sum(c.W * c.H for c in carr)
    for mode, cands in (("tiles", tiles), ("persistent", persistent)):
        opts = S.make_opts(fp16=True, persistent=(mode == "persistent"), graph=True)
        t, found = S.snerg_tuning_lookup(h, grid, carr, opts)
        if found:  # render_impl launches this workload with the recorded shape
            ms = time_launches(lambda: S.snerg_render(h, grid, m, carr, None, n, opts, out), reps, 1, torch)
        else:
            t, ms = S.snerg_autotune(h, grid, m, carr, opts, out, reps=reps, candidates=cands)
        log(f"  {mode}: {t} at {ms:.3f} ms{' (cached shape)' if found else ''}")
        modes[mode] = dict(tuning=list(t), ms=round(ms, 4), cached=found)
        if best is None or ms < best[2]:
            best = (opts, t, ms, mode)
    S.snerg_set_tuning(h, *best[1])
    if cache:
        S.snerg_tuning_save(h, cache)
    return best + (modes,)


def leg_plain(args, torch, S, W, O):
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dg = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    m = S.mlp_tensor(mlp)
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    carr = S.make_cameras(cams)
    opts = S.make_opts()
    grid = dg.struct()

    def step():
        S.snerg_render(h, grid, m, carr, None, n, opts, out)

    log(f"plain512: {g.n_blocks} blocks ({g.meta['occupancy']:.3f}), {n} rays; warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the render kernel's own duration: library events around that launch alone, on every
    # TIMING_EVERY-th frame of the timed region (each event pair costs the stream some
    # microseconds; sampling keeps that out of most frames)
    S.snerg_timing_enable(h, TIMING_EVERY)
    ms = time_launches(step, args.steps, 0, torch)
    kms = S.snerg_timing_read(h)
    S.snerg_timing_enable(h, False)
    kernel_ms = float(np.mean(kms))
    spread = launch_spread(step, args.steps, torch)
    cnt = frame_counters(S, h, dg, cams)
    abytes = algorithmic_bytes(cnt)
    res = dict(ms=ms, kernel_ms=kernel_ms, kernel_n=len(kms), rays=n, mrays=n / ms / 1e3, counters=cnt,
               alg_bytes=abytes, out=out, cams=cams, g=g, mlp=mlp, spread=spread)
    log(f"plain512: {ms:.3f} ms/frame, {res['mrays']:.1f} Mrays/s; render kernel {kernel_ms:.3f} ms, "
        f"{abytes / kernel_ms / 1e6:.1f} GB/s algorithmic")
    return res


def leg_batched(args, torch, S, W, O):
    cfg = W.config("batched1024")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dg = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    m = S.mlp_tensor(mlp)
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    carr = S.make_cameras(cams)
    log(f"batched1024: {g.n_blocks} blocks, {len(cams)} cameras, {n} rays; autotuning")
    grid = dg.struct()
    opts, best, best_ms, mode, modes = tune_launch(S, h, grid, m, carr, out, 2, cache=args.tuning_cache)
    log(f"batched1024: {mode} launch, tuning {best} at {best_ms:.3f} ms")

    def step():
        S.snerg_render(h, grid, m, carr, None, n, opts, out)

    steps = max(2, args.steps // 4)
    ms = time_launches(step, steps, max(1, args.warmup), torch)
    frame = out.cpu().numpy()
    ids = np.sort(np.random.default_rng(3).choice(n, 4096, replace=False))
    ref, cpu_mrays = oracle_rate(O, O.OracleGrid(g), mlp, cams, ids, args.cpu_threads)
    err = float(np.abs(frame[ids] - ref).max())
    # the deferred network: 1,696 FLOP per ray (34x16 + 16x16 + 16x3 multiply-adds); on MFMA tiles
    # 20 v_mfma_f32_16x16x16_f16 of 8,192 FLOP per 64 rays (K and N padded) are executed
    mlp_tflops = n * MLP_FLOP / (ms * 1e-3) / 1e12
    cnt = frame_counters(S, h, dg, cams)
    res = dict(ms=ms, rays=n, mrays=n / ms / 1e3, max_abs_err=err, err_sample=len(ids), tuning=list(best),
               mode=mode, modes=modes, cpu_mrays=cpu_mrays, mlp_tflops=mlp_tflops,
               mfma_frac=mlp_tflops / FP16_PEAK_TFLOPS,
               mfma_tflops_executed=n / 64 * 20 * 8192 / (ms * 1e-3) / 1e12, counters=cnt,
               alg_bytes=algorithmic_bytes(cnt), alg_flop=algorithmic_flop(cnt, network=False))
    log(f"batched1024: {ms:.3f} ms/batch, {res['mrays']:.1f} Mrays/s, fp16 max-abs err {err:.2e}; MLP "
        f"{mlp_tflops:.2f} TFLOP/s = {100 * res['mfma_frac']:.3f}% of the FP16 MFMA peak")
    return res


def leg_adjoint(args, torch, S, W, O):
    """One fine-tuning step of Eq. 3 on the float32 shadow of the 512^3 grid
    over 8 views at 800x800: forward with the per-ray state, squared error
    against targets rendered from a seeded perturbation (features scaled by
    1 + 0.05 U[-1, 1] and clamped to [0, 1], every weight moved by
    0.05 std(W) N(0, 1)), its gradient, and the backward to the 883 MLP
    parameters and every grid value."""
    from paper_2103_14645_amd import autograd as A
    cfg = W.config("adjoint512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dens = torch.from_numpy(g.dens).cuda().float().div_(255.0)
    rgb = torch.from_numpy(g.rgb).cuda().float().div_(255.0)
    feat = torch.from_numpy(g.feat).cuda().float().div_(255.0)
    m = S.mlp_tensor(mlp)
    carr = S.make_cameras(cams)
    n = sum(c.n_rays for c in cams)
    opts = S.make_opts()
    # targets: the perturbed grid and network rendered once
    pmlp, pfeat = W.perturbed(mlp, g)
    rt = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    rt.pack(dens, rgb, torch.from_numpy(pfeat).cuda())
    target = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    S.snerg_render(h, rt.struct(), S.mlp_tensor(pmlp), carr, None, n, opts, target)
    del rt
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    r.pack(dens, rgb, feat)
    grid = r.struct()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    aux = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    gout = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    gm = torch.empty(883, device="cuda")
    gd, gr, gf = torch.empty_like(dens), torch.empty_like(rgb), torch.empty_like(feat)

    def fwd():
        S.snerg_render(h, grid, m, carr, None, n, opts, out, aux)

    def mse():
        S.snerg_loss_mse(h, out, target, n, gout, loss)

    def bwd():
        S.snerg_render_backward(h, grid, m, carr, None, n, opts, aux, gout, gm, gd, gr, gf)

    def step():
        fwd()
        mse()
        bwd()

    log(f"adjoint512: {n} rays over {len(cams)} views, MSE against perturbed targets")
    steps = max(2, args.steps // 4)
    ms_f = time_launches(fwd, steps, 1, torch)
    mse()
    ms_l = time_launches(mse, steps, 1, torch)
    ms_b = time_launches(bwd, steps, 1, torch)
    ms_step = time_launches(step, steps, 1, torch)
    loss_value = float(loss.item())
    # Algorithmic bytes on the float32 shadow (its zero pattern is the uint8 grid's, so the
    # traversal counters are the same): forward = 4 B per macroblock, 1 B per in-block sample,
    # 8 corners x 32 B per composited sample, 16 B RGBA + 32 B aux per ray.  Backward = the same
    # re-march reads, the gradient scatter's read-modify-write of 8 corners x 8 channels x 4 B per
    # composited sample, and 12 B of dL/dRGB + 32 B of aux read per ray.
    dgu = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    cnt = frame_counters(S, h, dgu, cams)
    del dgu
    march = 4 * cnt["blocks"] + cnt["inblock"] + 256 * cnt["active"]
    fwd_bytes = march + 48 * cnt["rays"]
    bwd_bytes = march + 256 * cnt["active"] + 44 * cnt["rays"]
    res = dict(ms_fwd=ms_f, ms_bwd=ms_b, ms_loss=ms_l, ms_step=ms_step, rays=n, fwd_mrays=n / ms_f / 1e3,
               bwd_mrays=n / ms_b / 1e3, step_mrays=n / ms_step / 1e3, loss=loss_value,
               fwd_bytes=fwd_bytes, bwd_bytes=bwd_bytes,
               fwd_alg_gbs=fwd_bytes / (ms_f * 1e-3) / 1e9, bwd_alg_gbs=bwd_bytes / (ms_b * 1e-3) / 1e9,
               counters=cnt)
    log(f"adjoint512: fwd {ms_f:.3f} ms, loss {ms_l:.3f} ms, bwd {ms_b:.3f} ms -> {res['bwd_mrays']:.1f} bwd Mrays/s; "
        f"step {ms_step:.3f} ms; loss {loss_value:.6f}; algorithmic {res['fwd_alg_gbs']:.0f} / "
        f"{res['bwd_alg_gbs']:.0f} GB/s (fwd / bwd)")
    return res


def leg_large(args, torch, S, W, O):
    """64 x 1920x1080 forward in one graph launch (FP16 MLP, tiled or persistent
    as the autotuner finds faster), then
    forward + backward on random 65,536-ray minibatches over all 64 views
    (FP16 MLP forward and backward, float32 shadow of the grid): independent
    pixels, and whole 8x8 patches."""
    from paper_2103_14645_amd import autograd as A
    cfg = W.config("large1024")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dg = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    m = S.mlp_tensor(mlp)
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    carr = S.make_cameras(cams)
    log(f"large1024: {g.n_blocks} blocks ({g.meta['occupancy']:.3f}), {len(cams)} cameras, {n} rays")
    grid = dg.struct()
    opts, best, _, mode, modes = tune_launch(S, h, grid, m, carr, out, 1,
                                      tiles=[(8, 8, 4, 8), (8, 8, 2, 8), (16, 4, 4, 8)],
                                      persistent=[(8, 8, 4, 3), (8, 8, 4, 4), (8, 8, 2, 6), (8, 8, 4, 2)],
                                      cache=args.tuning_cache)

    def step():
        S.snerg_render(h, grid, m, carr, None, n, opts, out)

    ms = time_launches(step, 2, 1, torch)
    cnt = frame_counters(S, h, dg, cams)
    ids = torch.from_numpy(np.sort(np.random.default_rng(3).choice(n, 4096, replace=False))).cuda()
    frame = out[ids].cpu().numpy()
    ref, cpu_mrays = oracle_rate(O, O.OracleGrid(g), mlp, cams, ids.cpu().numpy(), args.cpu_threads)
    err = float(np.abs(frame - ref).max())
    del out
    # backward on minibatches of 65,536 rays
    r = A.ShadowRenderer(h, g.N, g.B, g.indirection, g.n_blocks)
    dens = torch.from_numpy(g.dens).cuda().float().div_(255.0)
    rgb = torch.from_numpy(g.rgb).cuda().float().div_(255.0)
    feat = torch.from_numpy(g.feat).cuda().float().div_(255.0)
    r.pack(dens, rgb, feat)
    sgrid = r.struct()
    bo = [S.make_opts(fp16=True)]
    mb = 65536
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    batches = [torch.randperm(n, device="cuda", generator=gen)[:mb].sort().values for _ in range(4)]
    bout = torch.empty((mb, 4), device="cuda")
    aux = torch.empty((mb, 8), device="cuda")
    gout = torch.randn((mb, 4), device="cuda") / mb
    gm = torch.empty(883, device="cuda")
    gd, gr, gf = torch.empty_like(dens), torch.empty_like(rgb), torch.empty_like(feat)
    grads = [(gd, gr, gf)]
    it = [0]

    def train_step():
        b = batches[it[0] % len(batches)]
        it[0] += 1
        S.snerg_render(h, sgrid, m, carr, b, mb, bo[0], bout, aux)
        S.snerg_render_backward(h, sgrid, m, carr, b, mb, bo[0], aux, gout, gm, *grads[0])

    def fwd_only():
        b = batches[it[0] % len(batches)]
        it[0] += 1
        S.snerg_render(h, sgrid, m, carr, b, mb, bo[0], bout, aux)

    ms_step = time_launches(train_step, 8, 2, torch)
    ms_f = time_launches(fwd_only, 8, 2, torch)
    ms_b = max(ms_step - ms_f, 1e-6)
    # the same minibatches with gradient accumulation (SNERG_FLAG_ACCUMULATE): the
    # backward adds into the arrays instead of clearing the 2.8 GB of grid gradients first
    bo[0] = S.make_opts(fp16=True, accumulate=True)
    gm.zero_(); gd.zero_(); gr.zero_(); gf.zero_()
    ms_step_acc = time_launches(train_step, 8, 2, torch)
    # the same with the grid gradients packed per voxel (SNERG_FLAG_GRAD_PACKED):
    # one cache line of device atomics per voxel hand-over instead of three
    grads[0] = (torch.zeros((dens.numel(), 8), device="cuda"), None, None)
    bo[0] = S.make_opts(fp16=True, grad_packed=True)
    ms_step_pk = time_launches(train_step, 8, 2, torch)
    bo[0] = S.make_opts(fp16=True, grad_packed=True, accumulate=True)
    ms_step_pk_acc = time_launches(train_step, 8, 2, torch)
    grads[0] = (gd, gr, gf)
    bo[0] = S.make_opts(fp16=True)
    # the same with minibatches of 1,024 whole 8x8 patches drawn across the 64 views
    tx, ty = cams[0].W // 8, cams[0].H // 8
    tiles = torch.randperm(len(cams) * tx * ty, device="cuda", generator=gen)[: 4 * (mb // 64)].view(4, -1)
    lane = torch.arange(64, device="cuda")
    def patch_ids(t):
        c, r = t // (tx * ty), t % (tx * ty)
        py = (r // tx)[:, None] * 8 + lane[None, :] // 8
        px = (r % tx)[:, None] * 8 + lane[None, :] % 8
        return (c[:, None] * (cams[0].W * cams[0].H) + py * cams[0].W + px).reshape(-1)
    batches = [patch_ids(t) for t in tiles]
    bo[0] = S.make_opts(fp16=True, patch_rays=True)  # aligned groups of 64 neighbouring rays
    it[0] = 0
    ms_step_p = time_launches(train_step, 8, 2, torch)
    ms_f_p = time_launches(fwd_only, 8, 2, torch)
    res = dict(ms=ms, rays=n, mrays=n / ms / 1e3, max_abs_err=err, tuning=list(best), mode=mode, modes=modes,
               counters=cnt, alg_bytes=algorithmic_bytes(cnt), alg_flop=algorithmic_flop(cnt, network=False),
               mb=mb, cpu_mrays=cpu_mrays,
               ms_train_step=ms_step, ms_mb_fwd=ms_f, bwd_mrays=mb / ms_b / 1e3,
               ms_train_step_accumulate=ms_step_acc, bwd_mrays_accumulate=mb / max(ms_step_acc - ms_f, 1e-6) / 1e3,
               ms_train_step_packed=ms_step_pk, bwd_mrays_packed=mb / max(ms_step_pk - ms_f, 1e-6) / 1e3,
               ms_train_step_packed_accumulate=ms_step_pk_acc,
               bwd_mrays_packed_accumulate=mb / max(ms_step_pk_acc - ms_f, 1e-6) / 1e3,
               ms_train_step_patches=ms_step_p, ms_mb_fwd_patches=ms_f_p,
               bwd_mrays_patches=mb / max(ms_step_p - ms_f_p, 1e-6) / 1e3)
    log(f"large1024: {ms:.1f} ms/launch, {res['mrays']:.1f} Mrays/s, fp16 err {err:.2e}; minibatch fwd+bwd "
        f"{ms_step:.2f} ms (bwd {res['bwd_mrays']:.1f} Mrays/s; accumulating {ms_step_acc:.2f} ms, bwd "
        f"{res['bwd_mrays_accumulate']:.1f} Mrays/s); packed gradients {ms_step_pk:.2f} ms (bwd "
        f"{res['bwd_mrays_packed']:.1f} Mrays/s; accumulating {ms_step_pk_acc:.2f} ms, bwd "
        f"{res['bwd_mrays_packed_accumulate']:.1f} Mrays/s); as 8x8 patches {ms_step_p:.2f} ms "
        f"(bwd {res['bwd_mrays_patches']:.1f} Mrays/s)")
    return res


def leg_nondeferred(args, torch, S, W, plain):
    """The performance ablation of Section 7.1 on the plain 512^3 frame: no
    view network at all, and the view network on every composited sample
    rather than a single time per ray, in FP32 and on FP16 MFMA tiles; the
    deferral speed-up against the deferred FP32 frame and the per-sample
    network's FLOP rate."""
    cfg = W.config("plain512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dg = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    m = S.mlp_tensor(mlp)
    n = sum(c.n_rays for c in cams)
    out = torch.empty((n, 4), device="cuda")
    carr = S.make_cameras(cams)
    grid = dg.struct()
    active = plain["counters"]["active"]
    res = {}
    # ablation row 1 of Section 7.1: no view-dependent network at all (diffuse colour only)
    off = S.make_opts(mlp_on=False)
    ms_off = time_launches(lambda: S.snerg_render(h, grid, m, carr, None, n, off, out), max(4, args.steps // 2), 2,
                           torch)
    res["mlp_off"] = dict(ms=ms_off, mrays=n / ms_off / 1e3, mlp_share_of_deferred_frame=1.0 - ms_off / plain["ms"])
    log(f"no view network: {ms_off:.3f} ms/frame; the deferred network is {100 * (1 - ms_off / plain['ms']):.1f}% "
        f"of the deferred frame")
    # the WebGL viewer's render variants (Appendix A, Eq. 9): the nearest-voxel gate
    # composites fewer samples; the partial un-premultiply rescales each pixel
    for name, kw in (("nn_gate", dict(nn_gate=True)), ("unpremultiply", dict(unpremultiply=True))):
        opts = S.make_opts(**kw)
        ms = time_launches(lambda: S.snerg_render(h, grid, m, carr, None, n, opts, out), max(4, args.steps // 2), 2,
                           torch)
        res[name] = dict(ms=ms, mrays=n / ms / 1e3, vs_exact_frame=ms / plain["ms"])
        log(f"variant {name}: {ms:.3f} ms/frame ({n / ms / 1e3:.1f} Mrays/s)")
    for name, fp16 in (("fp32", False), ("fp16_mfma", True)):
        opts = S.make_opts(fp16=fp16, per_sample_mlp=True)
        ms = time_launches(lambda: S.snerg_render(h, grid, m, carr, None, n, opts, out), max(4, args.steps // 2),
                           2, torch)
        tflops = active * 2 * (34 * 16 + 16 * 16 + 16 * 3) / (ms * 1e-3) / 1e12
        res[name] = dict(ms=ms, mrays=n / ms / 1e3, deferral_speedup=ms / plain["ms"], mlp_tflops=tflops,
                         mlp_frac_fp16_peak=tflops / 2500.0)
        log(f"non-deferred {name}: {ms:.3f} ms/frame ({n / ms / 1e3:.1f} Mrays/s), deferral speed-up "
            f"{ms / plain['ms']:.2f}x, per-sample network {tflops:.2f} TFLOP/s")
    return res


def leg_finetune(args, torch, S, W):
    """Fine-tuning of the deferred network on the fixed 512^3 uint8 SNeRG
    (Section 5.5): 65,536-ray minibatches over the 8 adjoint views, targets
    rendered with the original weights, training from perturbed weights;
    each step is render + squared error + MLP backward + Adam.  Two ways of
    drawing the minibatches: independent pixels (in ray-id order) and whole
    8x8 patches."""
    from paper_2103_14645_amd import finetune as F
    cfg = W.config("adjoint512")
    g, cams, mlp = cfg["grid"], cfg["cams"], cfg["mlp"]
    h = S.Handle()
    dg = S.DeviceGrid(h, g.N, g.B, g.indirection, g.dens, g.rgb, g.feat)
    n = sum(c.n_rays for c in cams)
    target = torch.empty((n, 4), device="cuda")
    S.snerg_render(h, dg.struct(), S.mlp_tensor(mlp), S.make_cameras(cams), None, n, S.make_opts(), target)
    start, _ = W.perturbed(mlp, g, rel=0.3)
    mb = 65536
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    order = torch.randperm(n, device="cuda", generator=gen)
    cgen = torch.Generator()
    cgen.manual_seed(3)
    sampling = {
        # rays drawn independently, each minibatch handed over in ray-id order (MlpFineTuner.epoch)
        "pixels": [order[i * mb:(i + 1) * mb].sort().values for i in range(n // mb)],
        # whole 8x8 patches in random order (MlpFineTuner.epoch(patches=True))
        "patches": None,
    }
    res = dict(minibatch=mb, rays_total=n)
    for kind in ("pixels", "patches"):
        w = S.mlp_tensor(start)
        ft = F.MlpFineTuner(h, dg.struct(), w, cams, target, lr=3e-4, max_batch=mb)
        if kind == "patches":
            po = ft.patch_order(cgen)
            sampling[kind] = [po[i * mb:(i + 1) * mb] for i in range(n // mb)]
        batches = sampling[kind]
        it = [0]
        losses = []

        def step():
            losses.append(ft.step(batches[it[0] % len(batches)]))
            it[0] += 1

        steps = max(4, args.steps)
        ms = time_launches(step, steps, 2, torch)
        ls = [float(x.item()) for x in losses]
        res[kind] = dict(ms_step=ms, steps_per_s=1000.0 / ms, mrays=mb / ms / 1e3, loss_first=ls[0],
                         loss_last=ls[-1], steps_run=len(ls))
        log(f"finetune ({kind}): {ms:.3f} ms/step ({1000.0 / ms:.0f} steps/s, {mb / ms / 1e3:.1f} Mrays/s), "
            f"loss {ls[0]:.5f} -> {ls[-1]:.5f} over {len(ls)} steps")
    return res


def leg_bake(args, torch, S, W):
    """Baking (Section 5.3, 5.4) of a dense 512^3 field (opaque displaced
    shell, hidden interior blobs, faint haze; B = 32) from the 100 training
    views of a synthetic scene (800x800, 39 degrees, eyes on a sphere of
    radius 2): the empty-space and visibility culls (snerg_bake_cull, which
    reads the kept count back) and the 8-bit atlas of the kept blocks
    (snerg_bake_quantize).  Rates: voxels of the dense grid and training
    rays per second over the whole bake; the quantisation's HBM rate from
    its algorithmic bytes (32 B read, 8 B written per kept voxel)."""
    N, B = 512, 32
    f = W.dense_shell_field(N)
    sg = torch.from_numpy(f.sigma).cuda()
    rg = torch.from_numpy(f.rgb).cuda()
    ft = torch.from_numpy(f.feat).cuda()
    del f
    cams = W.sphere_cameras([(800, 800, 39.0)] * 100, seed=1)
    rays = sum(c.n_rays for c in cams)
    h = S.Handle()
    carr = S.make_cameras(cams)
    opts = S.make_bake_opts()
    G3 = (N // B) ** 3
    ind = torch.empty(G3, dtype=torch.int32, device="cuda")
    n_kept = [0]

    def cull():
        n_kept[0] = S.snerg_bake_cull(h, N, B, sg, carr, opts, ind)

    reps = max(3, args.steps // 4)
    ms_cull = time_launches(cull, reps, 1, torch)
    n = n_kept[0]
    d8 = torch.empty((n, B, B, B), dtype=torch.uint8, device="cuda")
    r8 = torch.empty((n, B, B, B, 3), dtype=torch.uint8, device="cuda")
    f8 = torch.empty((n, B, B, B, 4), dtype=torch.uint8, device="cuda")
    ms_q = time_launches(lambda: S.snerg_bake_quantize(h, N, B, sg, rg, ft, ind, n, opts, d8, r8, f8),
                         max(5, args.steps), 2, torch)
    q_bytes = n * B ** 3 * 40
    ms = ms_cull + ms_q
    res = dict(ms=ms, ms_cull=ms_cull, ms_quantize=ms_q, gvox_per_s=N ** 3 / (ms * 1e-3) / 1e9,
               training_mrays=rays / ms_cull / 1e3, training_rays=rays, kept_blocks=n, blocks=G3,
               quantize_gbs=q_bytes / (ms_q * 1e-3) / 1e9, quantize_frac_hbm=q_bytes / (ms_q * 1e-3) / 1e9 / HBM_PEAK_GBS)
    log(f"bake 512^3: cull {ms_cull:.2f} ms ({res['training_mrays']:.0f} training Mrays/s), quantise {ms_q:.3f} ms "
        f"({res['quantize_gbs']:.0f} GB/s), kept {n}/{G3} blocks")
    del sg, rg, ft
    return res


def leg_copy(torch):
    """A plain 1 GiB device-to-device copy (torch's elementwise copy kernel),
    launched three times: what FETCH_SIZE and WRITE_SIZE read for it against
    the 1 GiB it moves each way calibrates those counters."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = time_launches(lambda: dst.copy_(src), 5, 1, torch)
    log(f"copy: {COPY_BYTES} B each way, {ms:.3f} ms, {2 * COPY_BYTES / ms / 1e6:.1f} GB/s")
    del src, dst
    return dict(ms=ms, bytes=COPY_BYTES, gbs=2 * COPY_BYTES / ms / 1e6)


def cpu_baseline(plain, O, threads):
    """The FP64 oracle on the host: all `threads` over the whole 800x800
    frame, and one thread over every 16th ray of it."""
    n = plain["rays"]
    ids = np.arange(0, n, dtype=np.int64)
    og = O.OracleGrid(plain["g"])
    t0 = time.perf_counter()
    ref = O.render(og, plain["mlp"], plain["cams"], ray_ids=ids, threads=threads)["rgba"]
    dt = time.perf_counter() - t0
    err = float(np.abs(plain["out"].cpu().numpy()[ids] - ref).max())
    _, one = oracle_rate(O, og, plain["mlp"], plain["cams"], ids[::16], 1)
    return dict(value=len(ids) / dt / 1e6, unit="Mrays/s", cores=threads, kind="oracle",
                sample=f"all {len(ids)} rays of the 800x800 frame, {dt:.1f} s wall on {threads} threads",
                single_thread_mrays=round(one, 4), host=host_cpu(), nproc=os.cpu_count(),
                gpu_max_abs_err=err)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--legs", default="plain,batched,adjoint,large,finetune,nondeferred,bake")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning-cache", default=None,
                    help="launch-shape cache file: shapes found there are reused, new ones are added")
    ap.add_argument("--source-hash", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the render shards by rays "
              f"with no communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle as O
    import workloads as W
    from paper_2103_14645_amd import snerg as S

    torch.cuda.set_device(0)
    legs = set(args.legs.split(","))
    plain = leg_plain(args, torch, S, W, O)
    extra = {}
    if "batched" in legs:
        extra["batched_fp16_1024"] = leg_batched(args, torch, S, W, O)
    if "adjoint" in legs:
        extra["adjoint_512"] = leg_adjoint(args, torch, S, W, O)
    if "large" in legs:
        extra["large_1024"] = leg_large(args, torch, S, W, O)
    if "finetune" in legs:
        extra["finetune"] = leg_finetune(args, torch, S, W)
    if "nondeferred" in legs:
        extra["nondeferred"] = leg_nondeferred(args, torch, S, W, plain)
    if "bake" in legs:
        extra["bake"] = leg_bake(args, torch, S, W)
    if "copy" in legs:
        extra["copy"] = leg_copy(torch)

    ms = plain["ms"]
    kms = plain["kernel_ms"]
    kv = committed_counters()
    copy_gbs = counter(kv, "copy_read_write_gbs")

    def measured(leg, kernel_ms):
        """HBM traffic of one launch from the committed counters (FETCH_SIZE +
        WRITE_SIZE, scaled by the copy calibration) and its rate at the live
        kernel time; None when the counters describe other code."""
        t = counter(kv, f"traffic.{leg}", int)
        if not t:
            return dict(traffic=None)
        gbs = t / (kernel_ms * 1e-3) / 1e9
        return dict(traffic=t, traffic_gbs=round(gbs, 1), traffic_frac_of_peak=round(gbs / HBM_PEAK_GBS, 4),
                    traffic_frac_of_copy_bw=round(gbs / copy_gbs, 4) if copy_gbs else None)

    def hbm_view(alg_bytes, kernel_ms, leg):
        gbs = alg_bytes / (kernel_ms * 1e-3) / 1e9
        d = dict(alg_bytes_per_launch=alg_bytes, effective_gbs=round(gbs, 1),
                 effective_frac_of_peak=round(gbs / HBM_PEAK_GBS, 4))
        if gbs > HBM_PEAK_GBS:
            d["above_peak"] = ("the algorithmic bytes exceed what HBM could deliver in this time: most of them "
                               "are served by the L2 and the Infinity Cache; traffic is what left the L2")
        d.update(measured(leg, kernel_ms))
        return d

    alg_flop = algorithmic_flop(plain["counters"])
    alu_tflops = alg_flop / (kms * 1e-3) / 1e12
    limiter = {k: counter(kv, f"plain512.{k}") for k in ("valu_busy", "ta_busy", "l2_hit", "valu_insts_per_wave")}
    line = {
        "metric": "Mrays/s and fps at 800x800 (fwd, batched FP16-MLP vs plain FP32); bwd Mrays/s",
        "value": round(plain["mrays"], 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain512: 512^3 SNeRG, B=32, 10.6% occupied procedural shell, uint8 atlas, "
                               "one 800x800 camera (39 deg), FP32 34-16-16-3 MLP",
                   "fps_800x800": round(1000.0 / ms, 2), "rays": plain["rays"],
                   "launch_ms_p10_p50_p90": plain["spread"]},
        # The render kernel is bound by vector-ALU issue (VALU ~70% busy, texture address path ~30%,
        # L2 hit rate ~88%, HBM traffic ~10% of peak, by the committed counters), so the roofline is
        # the ALU one: algorithmic FP32 work over the kernel's live duration against the FP32 peak.
        "roofline": {"bound": "alu", "achieved": round(alu_tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(alu_tflops / FP32_PEAK_TFLOPS, 4),
                     "traffic": counter(kv, "traffic.plain512", int),
                     "kernel": "k_render<u8, fp32-mlp>", "kernel_ms": round(kms, 4),
                     "kernel_ms_source": f"HIP events around the render kernel launch on every {TIMING_EVERY}th of the "
                                         f"{args.steps} timed frames ({plain['kernel_n']} launches)",
                     "alg_flop_per_launch": alg_flop,
                     "alg_flop_basis": f"{SAMPLE_FLOP} FLOP per composited sample, {RAY_FLOP} per ray whose "
                                       f"network runs",
                     "frac_of_unpacked_fp32_peak": round(alu_tflops / FP32_PEAK_UNPACKED_TFLOPS, 4),
                     "limiter_counters": limiter if any(v is not None for v in limiter.values()) else None,
                     "hbm": hbm_view(plain["alg_bytes"], kms, "plain512"),
                     "counters": plain["counters"]},
    }
    legs_out = {}
    if "batched_fp16_1024" in extra:
        b = extra["batched_fp16_1024"]
        legs_out["batched_fp16_1024"] = {"mrays": round(b["mrays"], 3), "ms": round(b["ms"], 4),
                                         "fps_800x800_equiv": round(b["mrays"] / 0.64, 2),
                                         "max_abs_err_vs_oracle": b["max_abs_err"], "err_sample": b["err_sample"],
                                         "rays": b["rays"], "tuning": b["tuning"], "launch": b["mode"],
                                         "launch_modes": b["modes"],
                                         "cpu_oracle_mrays": round(b["cpu_mrays"], 4),
                                         "roofline_hbm": hbm_view(b["alg_bytes"], b["ms"], "batched1024"),
                                         "roofline_alu": {"achieved": round(b["alg_flop"] / (b["ms"] * 1e-3) / 1e12, 3),
                                                          "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                          "frac": round(b["alg_flop"] / (b["ms"] * 1e-3) / 1e12
                                                                        / FP32_PEAK_TFLOPS, 4),
                                                          "note": "march and compositing FP32 work; the network "
                                                                  "runs on MFMA (roofline_mfma)"},
                                         "roofline_mfma": {"bound": "mfma", "achieved": round(b["mlp_tflops"], 3),
                                                           "peak": FP16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                           "frac": round(b["mfma_frac"], 6),
                                                           "executed_tflops": round(b["mfma_tflops_executed"], 3),
                                                           "note": "algorithmic MLP FLOPs over the whole launch, "
                                                                   "which the march bounds"},
                                         "counters": b["counters"]}
    if "adjoint_512" in extra:
        a = extra["adjoint_512"]
        legs_out["adjoint_512"] = {"bwd_mrays": round(a["bwd_mrays"], 3), "fwd_mrays": round(a["fwd_mrays"], 3),
                                   "step_mrays": round(a["step_mrays"], 3),
                                   "ms_bwd": round(a["ms_bwd"], 4), "ms_fwd": round(a["ms_fwd"], 4),
                                   "ms_loss": round(a["ms_loss"], 4), "ms_step": round(a["ms_step"], 4),
                                   "loss": a["loss"], "rays": a["rays"],
                                   "loss_def": "mean over rays and RGB of (rgb - target)^2, targets rendered from "
                                               "features x (1 + 0.05 U[-1,1]) and weights + 0.05 std N(0,1)",
                                   "roofline_hbm_fwd": hbm_view(a["fwd_bytes"], a["ms_fwd"], "adjoint512_fwd"),
                                   "roofline_hbm_bwd": hbm_view(a["bwd_bytes"], a["ms_bwd"], "adjoint512_bwd"),
                                   "bwd_atomics_per_launch": counter(kv, "adjoint512_bwd.atomics", int),
                                   "bwd_valu_busy": counter(kv, "adjoint512_bwd.valu_busy"),
                                   "counters": a["counters"]}
    if "large_1024" in extra:
        b = extra["large_1024"]
        legs_out["large_1024"] = {"mrays": round(b["mrays"], 3), "ms": round(b["ms"], 3),
                                  "fps_800x800_equiv": round(b["mrays"] / 0.64, 2),
                                  "max_abs_err_vs_oracle": b["max_abs_err"], "rays": b["rays"],
                                  "tuning": b["tuning"], "launch": b["mode"], "launch_modes": b["modes"],
                                  "roofline_hbm": hbm_view(b["alg_bytes"], b["ms"], "large1024"),
                                  "roofline_alu": {"achieved": round(b["alg_flop"] / (b["ms"] * 1e-3) / 1e12, 3),
                                                   "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                                   "frac": round(b["alg_flop"] / (b["ms"] * 1e-3) / 1e12
                                                                 / FP32_PEAK_TFLOPS, 4)},
                                  "minibatch": b["mb"],
                                  "ms_minibatch_fwd_bwd": round(b["ms_train_step"], 4),
                                  "bwd_mrays": round(b["bwd_mrays"], 3), "cpu_oracle_mrays": round(b["cpu_mrays"], 4),
                                  "ms_minibatch_fwd_bwd_accumulate": round(b["ms_train_step_accumulate"], 4),
                                  "bwd_mrays_accumulate": round(b["bwd_mrays_accumulate"], 3),
                                  "ms_minibatch_fwd_bwd_packed": round(b["ms_train_step_packed"], 4),
                                  "bwd_mrays_packed": round(b["bwd_mrays_packed"], 3),
                                  "ms_minibatch_fwd_bwd_packed_accumulate": round(b["ms_train_step_packed_accumulate"], 4),
                                  "bwd_mrays_packed_accumulate": round(b["bwd_mrays_packed_accumulate"], 3),
                                  "ms_minibatch_fwd_bwd_patches": round(b["ms_train_step_patches"], 4),
                                  "bwd_mrays_patches": round(b["bwd_mrays_patches"], 3),
                                  "counters": b["counters"]}
    if "nondeferred" in extra:
        legs_out["nondeferred_512"] = {k: {kk: round(vv, 5) for kk, vv in v.items()}
                                       for k, v in extra["nondeferred"].items()}
    if "finetune" in extra:
        f = extra["finetune"]
        legs_out["finetune_mlp_512"] = {k: ({kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                                            if isinstance(v, dict) else v) for k, v in f.items()}
    if "bake" in extra:
        legs_out["bake_512"] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in extra["bake"].items()}
    if "copy" in extra:
        legs_out["copy_calibration"] = {k: round(v, 4) for k, v in extra["copy"].items()}
    line["library"] = {"path": "paper_2103_14645_amd/libsnerg.so",
                       "sha256": file_sha256(os.path.join(ROOT, "paper_2103_14645_amd", "libsnerg.so")),
                       "kernel_source_sha256": kernel_source_hash(),
                       "counter_summary_matches": sorted({LEG_GROUP[k.split(".", 1)[1]] for k in kv
                                                          if k.startswith("traffic.")})}
    line["legs"] = legs_out
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)")
        line["cpu_baseline"] = cpu_baseline(plain, O, args.cpu_threads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
