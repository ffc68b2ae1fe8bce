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
    # n = 8192, k = 2: 32 column blocks of 256 and 64 row blocks of 128, 20 nodes
    # per row block and 24 per column block.  Band: every column block multiplies
    # the rows within 128 of it, 512 rows, except the first and last (384), so
    # 2 n 256 (2 n - 256) flops; P2M 2 n^2 k 20, L2P 2 n^2 k 24, M2L
    # 2 kn (64 * 20)(32 * 24).
    n, k = 8192, 2
    band = 2.0 * n * 256 * (2 * n - 256)
    p2m, l2p = 2.0 * n * n * k * 20, 2.0 * n * n * k * 24
    m2l = 2.0 * k * n * (64 * 20) * (32 * 24)
    assert bench.farfield_flops(n, k) == band + p2m + m2l + l2p
    assert abs(bench.farfield_flops(n, k) - 1.117e11) < 5e8
    # k = 1 with a ragged last block (n = 2500: 9 column blocks, the last of 452
    # columns; 19 row blocks, the last of 196 rows): rows [0, 384), 512 for blocks
    # 1..7, and [1920, 2500) for the last
    n = 2500
    band = 2.0 * n * (256 * 384 + 7 * 256 * 512 + 452 * 580)
    assert bench.farfield_flops(n, 1) == (band + 2.0 * n * n * 20 + 2.0 * n * n * 24
                                          + 2.0 * n * (19 * 20) * (9 * 24))
    # ranks above 2 take row blocks of 256 with 20 nodes on either side: three
    # row blocks per column block (two at the ends)
    p = 20
    sizes = [256] * 8 + [452]
    band = sum(2.0 * n * sizes[i] * sum(sizes[max(0, i - 1):i + 2]) for i in range(9))
    assert bench.farfield_flops(n, 3) == band + 2 * (2.0 * n * n * 3 * p) + 2.0 * 3 * n * (9 * p) ** 2
