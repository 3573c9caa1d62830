"""GPU against the oracle over the whole timed window of the benchmark.

The benchmark times steps 5..24 of the k = 32 chains at beta_c (256
samples, run as three concurrent parts).  This test runs the same chains
for 25 steps through the C ABI, one step at a time, and compares four
samples (from all three parts) step by step with oracle chains computed in
parallel on the host, in both benchmarked forms:

* FP64 contraction, candidate cut tau_null = 1e-11 (the oracle at 1e-11);
* FP32 contraction, tau_null = 1e-6 (the oracle, FP64, at 1e-6).

Gate (tests/parity.py): at every step the kept sets and candidate counts
must equal the oracle's, or differ by a validated rounding-distance flip
(the uniform within the interval its keep probability sweeps under the
step's perturbation), after which the chain is no longer compared; ln c
within kappa_tau (base + delta_in) and the normalised tensor (Gaussian
fingerprints) within 3 kappa (base + delta_in), kappa from the oracle's
spectrum of the step and delta_in the measured discrepancy of its input.
base is 100 eps for the FP64 contraction; for the FP32 one it is D^2 2^-24
(the worst case of a K = D^2 FP32 accumulation), also the floor of its ln c
tolerance.  The first eight steps (the ramp-up and the first steady steps,
which carry most of ln Z per site) must be compared in every chain; the
FP64 chains without a flip, through step 24."""
import numpy as np
import pytest

import parity
from workloads import BETA_C

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu

B, K, STEPS = 256, 32, 25
PICKS = [0, 85, 128, 255]          # parts 0, 0, 1, 2 of 0..85, 86..170, 171..255
FORMS = {"f64": (1e-11, 100 * parity.EPS64), "f32": (1e-6, K * K * 2.0 ** -24)}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_k32_timed_window(dtype):
    torch, m = need_gpu()
    tau, base = FORMS[dtype]
    log(f"k=32 window, {dtype}, tau {tau:g}: oracle chains {PICKS} started")
    futs = parity.start_oracle_pool([dict(beta=BETA_C, h=0.0, n_steps=STEPS, k=K, seed=0, sid=i, tau_null=tau)
                                     for i in PICKS], workers=len(PICKS))
    ts = m.init_tensor("site", [BETA_C], [0.0])
    g = parity.gpu_chain_trace(m, ts, B, STEPS, K, PICKS, dtype=dtype, tau=tau, log=log)
    stops, tights = [], []
    for i, f in zip(PICKS, futs):
        orc = f.result(timeout=900)
        r = parity.compare_chain(orc, g[i]["sel"], g[i]["c"], g[i]["lnc"], g[i]["fp"], K, 0, tau, base,
                                 lnc_floor=1e-10 if dtype == "f64" else base)
        log(f"sample {i}: compared {r.checked} steps ({r.tensor_checked} with tensors, {r.tight} with a tensor bound <= 1e-4), stop {r.stopped_at} "
            f"({r.reason}), worst delta {r.worst_delta:.2e}, worst |d ln c| {r.worst_dlnc:.2e} (largest tolerance "
            f"{r.worst_tau:.1e}), worst ratio to bound {r.max_ratio:.2e}, |d lnZ|/site "
            f"{abs(g[i]['ln_abs_Z'] - orc.ln_abs_Z) / 2.0 ** STEPS:.2e}")
        for n in r.notes:
            log("   " + n)
        stops.append(r.checked)
        tights.append(r.tight)
        if r.reason == "end" and r.lnZ_tol is not None:
            assert abs(g[i]["ln_abs_Z"] - orc.ln_abs_Z) / 2.0 ** STEPS <= r.lnZ_tol
    assert min(stops) >= 8, stops
    if dtype == "f64":
        assert min(tights) >= 8, tights
