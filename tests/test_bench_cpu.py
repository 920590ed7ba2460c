"""Host-side checks of bench.py's contract: one GPU only (a request for more
exits with a JSON message), the flop count per pair, the algorithmic bytes of
the timed launch, and the source hash that ties the committed counter figures
to the sources they were measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_flops_per_pair_counts_distance_weight_and_accumulation():
    # distance 2D + 3, weight 2 (the exponential itself not counted),
    # accumulation 2D + 1
    for d in (1, 2, 3, 16, 32):
        assert bench.flops_per_pair(d) == (2 * d + 3) + 2 + (2 * d + 1)


def test_algorithmic_bytes_of_the_timed_launch():
    # 512 seeds = 8 tiles of 64; 200,000 points = 391 chunks of 512 points,
    # at most 2048 items: 256 chunks per tile
    m, n = 512, 200_000
    assert bench.algorithmic_bytes("fp32", m, n) == 8 * n * 16 + 2 * m * 256 * 16
    assert bench.algorithmic_bytes("bf16", m, n) == 8 * n * 80 + 2 * m * 256 * 16
    # one tile: every chunk of 512 points is an item
    assert bench.algorithmic_bytes("fp32", 64, 4096) == 4096 * 16 + 2 * 64 * 8 * 16


def test_source_digest_is_stable_and_covers_the_kernel_sources():
    a = bench.source_digest()
    assert a == bench.source_digest()
    assert len(a) == 16 and int(a, 16) >= 0
