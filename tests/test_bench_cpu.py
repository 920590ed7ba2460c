"""Host-side checks of bench.py's contract: one GPU only (a request for more
exits with a JSON message), the flop counts per pair, the algorithmic bytes of
the timed launch, the roofline entry, and the source hash that ties the
committed counter figures to the sources they were measured on."""
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
    # every seed tile streams the n x D points once, 4 bytes per coordinate:
    # 512 seeds = 8 tiles of 64 over 200,000 x 3 points
    assert bench.algorithmic_bytes(512, 200_000, 3) == 8 * 200_000 * 3 * 4
    assert bench.algorithmic_bytes(65, 1000, 2) == 2 * 1000 * 2 * 4
    # the wide BF16 form's tiles hold 128 seeds
    assert bench.algorithmic_bytes(8192, 262_144, 32, 128) == 64 * 262_144 * 32 * 4


def test_adjoint_flops_per_pair():
    # forward 4D+6, recomputed forward 4D+6, dS pass 6D+8, dX pass 8D+8
    for d in (1, 4, 16):
        assert bench.adjoint_flops_per_pair(d) == 22 * d + 28


def test_roofline_entry_fields():
    e = bench.roofline_entry(512 * 200_000, 3, 0.030, 512, 200_000, "bf16", "launch", "kernel")
    assert e["bound"] == "alu" and e["unit"] == "TFLOP/s" and e["peak"] == bench.FP32_VEC_PEAK_TFLOPS
    assert abs(e["achieved"] - 512 * 200_000 * 18 / 0.030e-3 / 1e12) < 1e-9
    assert abs(e["frac"] - e["achieved"] / e["peak"]) < 1e-12
    assert e["contraction_frac_of_bf16_mfma_peak"] > 0 and e["traffic"] is None


def test_source_digest_is_stable_and_covers_the_kernel_sources():
    for which in ("c2", "c3"):
        a = bench.source_digest(which)
        assert a == bench.source_digest(which)
        assert len(a) == 16 and int(a, 16) >= 0
        for f in bench.COUNTER_SOURCES[which]:
            assert os.path.exists(os.path.join(bench.ROOT, "paper_2112_13891_amd", "csrc", f)), f
    # each launch's own step kernels are covered
    assert "k_step_bf16.hip" in bench.COUNTER_SOURCES["c2"]
    assert "k_step_bf16f.hip" in bench.COUNTER_SOURCES["c3"]
    assert bench.source_digest("c2") != bench.source_digest("c3")
