"""bench.py's host side: the one-GPU contract and the byte model (no GPU)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_bytes_follow_the_per_unit_figures():
    b = _bench()
    # 4 B per macroblock traversed, 1 B per in-block sample, 64 B per composited
    # sample (8 corners x 8 B), 16 B of output per ray
    cnt = {"blocks": 10, "inblock": 100, "active": 7, "rays": 3}
    assert b.algorithmic_bytes(cnt) == 4 * 10 + 100 + 64 * 7 + 16 * 3


def test_algorithmic_flop_follow_the_per_unit_figures():
    b = _bench()
    cnt = {"active": 7, "gated": 3}
    assert b.SAMPLE_FLOP == 15 + 128 + 20 and b.RAY_FLOP == 2 * (34 * 16 + 16 * 16 + 16 * 3) + 36 + 9 + 7
    assert b.algorithmic_flop(cnt) == 7 * b.SAMPLE_FLOP + 3 * b.RAY_FLOP
    assert b.algorithmic_flop(cnt, network=False) == 7 * b.SAMPLE_FLOP
    # float32 shadow: 8 corners x 32 B per composited sample
    cnt = {"blocks": 10, "inblock": 100, "active": 7, "rays": 3}
    assert b.algorithmic_bytes(cnt, value_bytes=32, out_bytes=48) == 4 * 10 + 100 + 256 * 7 + 48 * 3


def test_counter_figures_are_tied_to_the_kernel_sources():
    b = _bench()
    kv = b.committed_counters()
    # a leg's counter figures are kept only while its kernel sources hash to the recorded value
    now = b.group_hashes()
    for k in kv:
        if k.startswith("traffic."):
            grp = b.LEG_GROUP[k.split(".", 1)[1]]
            assert kv[f"sources_sha256.{grp}"] == now[grp]
            assert int(kv[k]) > 0
    with open(b.COUNTER_SUMMARY) as f:
        text = f.read()
    assert "sources_sha256.render = " in text and "sources_sha256.backward = " in text
