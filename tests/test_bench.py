"""The benchmark's contract on the host: one GPU only, and the algorithmic
byte count of the receiver pass it reports against the HBM peak."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_receiver_pass_bytes_at_the_headline_size():
    # n = 1e6, K = 30: n(24K + 16) + nK(10 + s) + 2nK^2(4 + s), s = 8 (FP64 key)
    # or 4 (FP32 cross term); the mixed form adds S(x), x's row (FP32) and
    # logs per receiver and one FP64 log row per rescue
    n, K, D = 1_000_000, 30, 21
    plain = bench.recv_bytes(n, K, D, False, 0)
    assert plain == n * (24 * K + 16) + n * K * 18 + 2 * n * K * K * 12
    assert abs(plain / 1e9 - 22.876) < 1e-3
    mixed = bench.recv_bytes(n, K, D, True, 1000)
    assert mixed == (n * (24 * K + 16) + n * K * 14 + 2 * n * K * K * 8
                     + n * (8 + D * 12) + 1000 * D * 8)
    assert mixed < plain
