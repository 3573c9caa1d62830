"""Host logic of bench.py (no GPU): the committed HBM counter figures are
reported only for the kernel source and the workload window they were
taken on, and the algorithmic flop counts are the method's."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_candidate_cut_per_dtype():
    # ten times the rounding floor of the tensor the FP64 decomposition sees
    assert bench.TAU_NULL["f64"] == 1e-11 and bench.TAU_NULL["f32"] == 1e-6


def test_algorithmic_counts():
    # two n x n splits, n = k^2: Gram n^3 + tridiagonalisation 4/3 n^3 each
    assert abs(bench.decomposition_flops(32) - 2 * (1 + 4 / 3) * 1024 ** 3) < 1e-6 * 1024 ** 3
    assert bench.gemm_flops(32) == 2 * 1024 ** 3


def test_gemm_floor():
    # k = 32, 256 products of 1024^3: FP64 bound by the MFMA pipe (7.0 ms
    # against 0.8 ms of bytes), BF16 and FP8 by their bytes (8 and 6 MiB per
    # product: 0.27 and 0.20 ms against 0.22 and 0.11 ms of flops)
    nb, tm, th = bench.gemm_floor("f64", 32, 256)
    assert nb == 256 * 1024 ** 2 * (2 * 8 + 8) and tm > th and abs(tm - 6.994) < 0.01
    nb, tm, th = bench.gemm_floor("bf16", 32, 256)
    assert nb == 256 * 8 * 2 ** 20 and th > tm and abs(th - 0.2684) < 1e-3
    nb, tm, th = bench.gemm_floor("fp8", 32, 256)
    assert nb == 256 * 6 * 2 ** 20 and th > tm and abs(tm - 0.1099) < 1e-3


def test_traffic_record_key():
    try:
        rec = json.load(open(bench.TRAFFIC_FILE))
    except OSError:
        return
    for kernel, r in rec.items():
        key = r["window"]
        got = bench.measured_traffic(kernel, key)
        if got is not None:   # the kernel source still matches the counters
            assert got["fetch_bytes_per_launch"] > 0 and got["write_bytes_per_launch"] > 0
        for f, v in (("parts", key["parts"] + 1), ("tau_null", key["tau_null"] * 10), ("batch", 2 * key["batch"]),
                     ("warmup", key["warmup"] + 2), ("steps", 1), ("dtype", "bf16")):
            other = dict(key)
            other[f] = v
            assert bench.measured_traffic(kernel, other) is None
