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


def test_traffic_figure_is_tied_to_the_render_sources():
    b = _bench()
    traffic, copy_gbs = b.measured_traffic()
    # the committed counter summary either describes these sources or is ignored
    if traffic is None:
        assert copy_gbs is None
    else:
        assert traffic > 0 and copy_gbs > 0
        with open(b.TRAFFIC_SUMMARY) as f:
            assert b.render_source_hash() in f.read()
