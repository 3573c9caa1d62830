"""Host logic of bench.py (no GPU): the committed HBM counter figures are
reported only for the workload and kernel source they were taken on."""
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


def test_traffic_record_key():
    rec = json.load(open(bench.TRAFFIC_FILE))
    for kernel in (bench.JACOBI_KERNEL, bench.QR128_KERNEL):
        r = rec[kernel]
        k, b, p, tau = r["k"], r["batch"], r["parts"], r["tau_null"]
        got = bench.measured_traffic(kernel, k, b, p, tau)
        if got is not None:   # the kernel source still matches the counters
            assert got["fetch_bytes_per_launch"] > 0 and got["write_bytes_per_launch"] > 0
        # any other workload: no figure
        assert bench.measured_traffic(kernel, k, b, p + 1, tau) is None
        assert bench.measured_traffic(kernel, k, b, p, tau * 10) is None
        assert bench.measured_traffic(kernel, k, 2 * b, p, tau) is None
