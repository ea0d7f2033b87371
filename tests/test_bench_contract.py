"""CPU checks of bench.py's command-line contract: it runs on one GPU only and
reports the update cap the library applies.  No GPU is touched."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_exits_with_a_message():
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2
        msg = json.loads(r.stdout.strip().splitlines()[-1])
        assert "one GPU" in msg["error"] and f"--gpus {n}" in msg["error"]


def test_flops_and_kernel_names():
    b = load_bench()
    # eq. (3): K (2W - 1) FMAs plus ~5 flops of candidate per touched coordinate
    assert b.flops_per_update(25, 64) == 7 * 25 * 127
    assert b.flops_per_update(25, 200) == 7 * 25 * 399
    assert b.wave_kernel_name(25, 64) == "k_lgcd_wave<7, 1, 1>"
    assert b.wave_kernel_name(25, 126) == "k_lgcd_wave<7, 1, 2>"
    assert b.wave_kernel_name(25, 199) == "k_lgcd_wave<7, 1, 4>"
    assert b.wave_kernel_name(5, 40) == "k_lgcd_wave<2, 1, 1>"
    assert b.wave_kernel_name(13, 200) == "k_lgcd_wave<4, 1, 4>"
    assert b.wave_kernel_name(32, 10) == "k_lgcd_wave<8, 4, 1>"
    assert b.wave_kernel_name(20, 100) == "k_lgcd_wave<7, 4, 2>"   # two padded groups
    assert b.wave_kernel_name(27, 100) == "k_lgcd_wave<7, 3, 2>"


def test_roofline_arithmetic():
    b = load_bench()
    st = {"round_launches": [10, 0, 0, 0], "round_kernel_ms": [2.0, 0, 0, 0],
          "round_updates_total": 1_000_000, "round_state": [4, 0, 0, 0]}
    r = b.roofline(st, 25, 64, "nowhere", 63)
    # 1e5 updates per launch of 200 us: 1e5 * 22225 flops / 2e-4 s = 11.1125 TFLOP/s
    assert abs(r["achieved"] - 11.1125) < 1e-9
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert abs(r["frac"] - 11.1125 / 157.3) < 1e-12
    assert r["traffic"] is None and r["kernel"] == "k_lgcd_wave<7, 1, 1>"
    assert abs(r["avg_launch_us"] - 200.0) < 1e-9


def test_segment_rule_mirrors_the_library():
    """The bench's copy of the tuned segment rule: ceil(L / seg_len), lowered
    to keep segments at least max(W - 1, (2W - 2) / (C - 1)) long; the fixed
    rule is floor(L / min_segment(W, 3))."""
    b = load_bench()
    f = b.seg_rule(64, {"seg_len": 128, "colors": 2})
    assert f(1280) == 10 and f(1281) == 10   # 11 segments of 116 < 126 -> 10
    assert f(100) == 1
    g = b.seg_rule(64, None)
    assert g(6300) == 100 and g(62) == 1
