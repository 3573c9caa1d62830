"""Deterministic coarse-graining steps before Monte Carlo (Section V,
Discussion) on the GPU, through the C ABI (mctrg_run_config.n_det).

C1 configuration (16 x 16 torus, k = 8, beta_c): the first three Ising
steps keep every candidate (ranks 2, 4, 4), so a deterministic prefix of
three steps followed by the independent estimator must give every sample
of the pure independent estimator (to rounding), while decomposing 68
tensors per sample instead of 510.  The prefix form is also compared with
the oracle position by position, and the shared form with a top-k prefix
step by step."""
import time

import numpy as np
import pytest

import parity
from oracle import ising, trg
from workloads import BETA_C

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


def test_exact_prefix_equals_independent_estimator():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    S = 256
    times = {}
    res = {}
    for nd in (0, 3, 0, 3):    # second pass timed warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res[nd] = m.run_samples(ts, S, n_steps=8, k=8, mode="independent", seed=3, n_det=nd, want_ln_c=True)
        torch.cuda.synchronize()
        times[nd] = time.perf_counter() - t0
    a, b = res[0], res[3]
    assert a.status == b.status == m.OK
    la, lb = a.ln_abs_Z.cpu().numpy(), b.ln_abs_Z.cpu().numpy()
    assert np.array_equal(a.sign.cpu().numpy(), b.sign.cpu().numpy())
    err = np.max(np.abs(la - lb)) / 256
    log(f"prefix n_det=3 vs independent: max |d lnZ|/site {err:.2e}; {S} samples in {times[0] * 1e3:.0f} ms "
        f"(independent) vs {times[3] * 1e3:.0f} ms (prefix)")
    assert err < 1e-12
    assert np.allclose(a.ln_c.cpu().numpy(), b.ln_c.cpu().numpy(), rtol=1e-12, atol=1e-10)


def test_prefix_independent_matches_oracle():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [0.42], [0.1])
    n, k, nd = 8, 6, 3
    r = m.run_samples(ts, 3, n_steps=n, k=k, mode="independent", seed=8, n_det=nd, record=True, want_ln_c=True)
    rec, lnc, ln = r.record.cpu().numpy(), r.ln_c.cpu().numpy(), r.ln_abs_Z.cpu().numpy()
    for i in range(3):
        o = trg.run_independent(ising.site_tensor(0.42, 0.1), n, k, 8, i, n_det=nd)
        g = parity.compare_independent(o, m.split_independent_record(rec[i], n), lnc[i], k, 8, i, 1e-11,
                                       100 * parity.EPS64)
        log(f"prefix sample {i}: {g.checked} steps compared ({g.reason}) {g.notes}")
        assert g.checked >= nd + 2
        if g.reason == "end":
            assert abs(ln[i] - o.ln_abs_Z) / 2.0 ** n < 1e-12


def test_prefix_shared_matches_oracle():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    n, k, nd = 9, 12, 4
    r = m.run_samples(ts, 4, n_steps=n, k=k, seed=2, n_det=nd, record=True, want_ln_c=True)
    rec, lnc, ln = r.record.cpu().numpy(), r.ln_c.cpu().numpy(), r.ln_abs_Z.cpu().numpy()
    for i in range(4):
        o = trg.run_shared(ising.site_tensor(BETA_C), n, k, 2, i, n_det=nd)
        sel = [[list(map(int, rec[i, s, 4:4 + rec[i, s, 2]])), list(map(int, rec[i, s, 4 + k:4 + k + rec[i, s, 3]]))]
               for s in range(n)]
        c = [[int(rec[i, s, 0]), int(rec[i, s, 1])] for s in range(n)]
        orc = parity.OracleChain(i, [parity.OracleStep(st.ln_c, [sp.c for sp in st.splits],
                                                      [list(map(int, sp.sel)) for sp in st.splits],
                                                      [sp.sigma[:min(sp.sigma.size, sp.c + 8)] for sp in st.splits],
                                                      max(parity.kappa_split(sp.sigma, sp.c, sp.sel)
                                                          for sp in st.splits), None, 1.0)
                                     for st in o.records], o.ln_abs_Z, o.sign)
        g = parity.compare_chain(orc, sel, c, lnc[i], None, k, 2, 1e-11, 100 * parity.EPS64)
        log(f"shared prefix sample {i}: {g.checked} steps compared ({g.reason}) {g.notes}")
        # the prefix steps keep the first min(k, c) values
        for s in range(nd):
            assert sel[s][0] == list(range(min(k, c[s][0])))
        assert g.checked >= nd + 2
