"""The cheaper decomposition (MCTRG_DEC_QR3 / MCTRG_DEC_QR5) on the GPU:
the QR-iteration basis V = P Q2 (Q4) with the exact expansion M = sum_j
(M v_j) v_j^T, whose terms are drawn and reweighted like SVD terms.

* Exactness: a top-k chain with k at least the rank keeps every term, so it
  must reproduce the brute-force Z whatever the basis.
* Unbiasedness (Section II: any inclusion rates r > 0 keep Eqs. Tsum and
  Ssum): the C1 independent estimator with the QR basis, 5 seeds x 1000
  samples, pooled mean of Z~/Z within two standard errors of 1 and the
  z-scores consistent with N(0,1).  Its per-sample spread and run time are
  logged beside the SVD form's (variance traded for work)."""
import math
import time

import numpy as np
import pytest

from oracle import ising
from workloads import BETA_C

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dec", ["qr3", "qr5"])
@pytest.mark.parametrize("L,n", [(2, 2), (4, 4)])
def test_qr_basis_exact_chain(dec, L, n):
    torch, m = need_gpu()
    beta, h = 0.42, 0.1
    ts = m.init_tensor("site", [beta], [h])
    r = m.run_samples(ts, 2, n_steps=n, k=32, mode="topk", decomposition=dec)
    bf = ising.brute_force_lnZ_torus(L, beta, h)
    log(f"{dec} exact {L}x{L}: {r.ln_abs_Z.cpu().numpy()} vs {bf}")
    assert np.all(r.sign.cpu().numpy() == 1)
    assert np.allclose(r.ln_abs_Z.cpu().numpy(), bf, rtol=0, atol=1e-11)


@pytest.mark.parametrize("dec", ["qr3", "qr5"])
def test_qr_basis_unbiased_against_kaufman(dec):
    """Ten seeds of 1000 samples (the QR basis has the larger spread)."""
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    lnZ = ising.kaufman_lnZ_torus(16, BETA_C)
    zs, allv = [], []
    t = {}
    for d, seeds in (("svd", [0]), (dec, range(10))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for seed in seeds:
            r = m.run_samples(ts, 1000, n_steps=8, k=8, mode="independent", seed=seed, decomposition=d)
            assert r.status == m.OK
            v = r.sign.cpu().numpy() * np.exp(r.ln_abs_Z.cpu().numpy() - lnZ)
            if d == dec:
                mean, se = v.mean(), v.std(ddof=1) / math.sqrt(v.size)
                zs.append((mean - 1.0) / se)
                allv.append(v)
            else:
                sd_svd = v.std(ddof=1)
        torch.cuda.synchronize()
        t[d] = (time.perf_counter() - t0) / len(seeds)
    v = np.concatenate(allv)
    mean, se = v.mean(), v.std(ddof=1) / math.sqrt(v.size)
    log(f"C1 with {dec}: mean Z~/Z = {mean:.5f} +- {se:.5f} (z {(mean - 1) / se:+.2f}), per-sample std "
        f"{v.std(ddof=1):.4f} (SVD {sd_svd:.4f}); z-scores {[round(float(z), 2) for z in zs]}; 1000 samples in "
        f"{t[dec]:.2f} s ({dec}) vs {t['svd']:.2f} s (SVD)")
    assert abs(mean - 1.0) <= 2.0 * se
    assert sum(z * z for z in zs) < 23.21     # 99 % point of chi^2 with 10 degrees


def test_qr_basis_k32_speed_and_spread():
    """k = 32 shared chains at beta_c, 12 steps (four at n = 1024): logs the
    step time and the spread of ln|Z~| per site of each decomposition."""
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    out = {}
    for d in ("svd", "qr3", "qr5"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = m.run_samples(ts, 64, n_steps=12, k=32, seed=1, decomposition=d)
        torch.cuda.synchronize()
        ln = r.ln_abs_Z.cpu().numpy() / 2.0 ** 12
        out[d] = (time.perf_counter() - t0, ln.mean(), ln.std(ddof=1))
        assert r.status == m.OK and np.all(np.isfinite(ln))
    for d, (tt, mu, sd) in out.items():
        log(f"k=32 {d}: 64 samples x 12 steps in {tt:.2f} s; mean ln|Z~|/site {mu:.9f}, spread {sd:.2e}")
    # the three estimates of the same quantity agree within their spreads
    for d in ("qr3", "qr5"):
        assert abs(out[d][1] - out["svd"][1]) < 5 * (out[d][2] + out["svd"][2]) / math.sqrt(64) + 1e-9
