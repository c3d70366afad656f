"""Host-side pieces of bench.py, checked without a GPU.

* the single-GPU contract: --gpus N > 1 exits with a message (status 2);
* the algorithmic byte and flop models against hand counts for the 64^3
  free workload (272 packed slots) and the complex one (528 one-pair slots);
* the traffic record is used only while the kernel source it was measured on
  is unchanged.
"""
import json
import math
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_free64():
    n, slots, N = 64, 272, 32
    a = bench.algorithmic_bytes(n, 2, N, slots)
    x = 2 * n ** 3 * 8  # two x classes of complex FP32 per slot
    assert a["pass_b"] == slots * 2 * x == 2281701376  # read and written once
    assert a["pass_a"] == slots * x + N * n ** 3 * 4
    assert a["pass_c"] == slots * x + N * n ** 3 * 4 + N * n ** 3 * 8
    c = bench.algorithmic_bytes(n, 2, N, 528, cplx=True)
    assert c["pass_b"] == 528 * 2 * x
    assert c["pass_a"] == 528 * x + N * n ** 3 * 8  # complex FP32 orbitals
    assert c["pass_c"] == 528 * x + N * n ** 3 * 8 + N * n ** 3 * 16


def test_fft_flop_model():
    n, slots = 64, 272
    f = 5.0 * n * math.log2(n)  # one complex n-point line
    fl = bench.fft_flops(n, (2, 2, 2), slots)
    # pass B per slab: y forward and inverse per y class (2 x 2n lines) and z
    # forward and inverse per (y, z) class (4 x 2n lines): 12 n lines
    assert fl["pass_b"] == pytest.approx(slots * 2 * n * 12 * n * f)
    assert fl["pass_a"] == pytest.approx(slots * 2 * n * n * f)
    # the wire as the passes see it, (2, 1, 2): 6 n lines per slab; periodic 4 n
    assert bench.fft_flops(n, bench.PASS_CLASSES["wire"], slots)["pass_b"] == pytest.approx(
        slots * 2 * n * 6 * n * f)
    assert bench.fft_flops(n, (1, 1, 1), slots)["pass_b"] == pytest.approx(slots * n * 4 * n * f)


def test_traffic_record_follows_the_kernel_source():
    for kernel in ("pass_a", "pass_b", "pass_c"):
        path = os.path.join(ROOT, "profiles", f"{kernel}_free64_n32_traffic.json")
        with open(path) as fh:
            rec = json.load(fh)
        assert rec["hbm_bytes_per_launch"] > 0
        same = rec["source_sha1"] == bench.kernel_source_sha1(kernel)
        assert bench.measured_traffic(kernel, "free64_n32") == (rec["hbm_bytes_per_launch"] if same else None)
    assert bench.measured_traffic("pass_b", "no_such_workload") is None
