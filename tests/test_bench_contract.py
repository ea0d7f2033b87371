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


def test_effective_update_cap():
    b = load_bench()
    # automatic cap max(4, round(2 sqrt(W))): 28 at the paper's W = 200, 16 at W = 64
    assert b.effective_cap(-1, 200) == 28
    assert b.effective_cap(-1, 64) == 16
    assert b.effective_cap(-1, 1) == 4 and b.effective_cap(-1, 4) == 4
    assert b.effective_cap(-1, 5) == 4   # 2 sqrt(5) = 4.47
    assert b.effective_cap(-1, 7) == 5   # 2 sqrt(7) = 5.29
    # explicit caps pass through; 0 means no cap
    assert b.effective_cap(9, 200) == 9 and b.effective_cap(0, 200) == 0
