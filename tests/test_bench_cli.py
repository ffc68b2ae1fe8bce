"""CPU checks of bench.py: it refuses more than one GPU before touching a device,
and the algorithmic flop count behind its far-field roofline matches the closed
form of the product's four parts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_farfield_flops_closed_form():
    # n = 8192, k = 2: 32 blocks of 256, P = 24 nodes.  Band: every column block
    # multiplies three row blocks except the first and last (two), so
    # 2 n (3 n - 2 * 256) 256 flops; P2M and L2P 2 n^2 kP each; M2L 2 kn (nb P)^2.
    n, k, b, p = 8192, 2, 256, 24
    nb = n // b
    band = 2.0 * n * 256 * (3 * n - 2 * b)
    p2m = l2p = 2.0 * n * n * k * p
    m2l = 2.0 * k * n * (nb * p) ** 2
    assert bench.farfield_flops(n, k) == band + p2m + m2l + l2p
    assert abs(bench.farfield_flops(n, k) - 1.331e11) < 5e7
    # a ragged last block (n = 2500: 9 blocks, the last of 452 rows)
    n = 2500
    sizes = [256] * 8 + [452]
    band = sum(2.0 * n * sizes[i] * sum(sizes[max(0, i - 1):i + 2]) for i in range(9))
    assert bench.farfield_flops(n, 3) == band + 2 * (2.0 * n * n * 3 * p) + 2.0 * 3 * n * (9 * p) ** 2
