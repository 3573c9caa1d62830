"""The failure contract of the C ABI (include/mctrg.h): a sample that fails
numerically comes back with sign 0 and ln|Z~| NaN while every other sample
is exactly what it would have been, the call returns ENUMERIC and the
estimator counts the failure; a workspace budget too small for one sample
gives ENOMEM before anything is enqueued (outputs untouched); the chain
interface reads back the current tensors and records the kept sets."""
import math
import os

import numpy as np
import pytest

import parity
from oracle import ising, trg
from workloads import BETA_C

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


def test_enumeric_isolates_the_failed_sample(monkeypatch):
    torch, m = need_gpu()
    log("ENUMERIC: sample 2 of 5 made non-finite at its last step")
    ts = m.init_tensor("site", [0.42], [0.05])
    good = m.run_samples(ts, 5, n_steps=7, k=6, seed=4, want_ln_c=True)
    assert good.status == m.OK
    monkeypatch.setenv("MCTRG_TEST_FAIL_SAMPLE", "2")
    bad = m.run_samples(ts, 5, n_steps=7, k=6, seed=4, want_ln_c=True)
    assert bad.status == m.ENUMERIC
    sg, ln = bad.sign.cpu().numpy(), bad.ln_abs_Z.cpu().numpy()
    assert sg[2] == 0 and math.isnan(ln[2])
    keep = [0, 1, 3, 4]
    assert np.array_equal(sg[keep], good.sign.cpu().numpy()[keep])
    assert np.array_equal(ln[keep], good.ln_abs_Z.cpu().numpy()[keep])
    est = m.estimate_lnZ(bad.sign, bad.ln_abs_Z, 128.0)
    assert est["n_failed"] == 1 and est["n_used"] == 4
    # the hook names a global sample id: with an offset the same sample is output 0
    monkeypatch.setenv("MCTRG_TEST_FAIL_SAMPLE", "7")
    r = m.run_samples(ts, 3, n_steps=5, k=6, seed=4, sample_offset=7)
    assert r.status == m.ENUMERIC and r.sign.cpu().numpy()[0] == 0 and np.all(r.sign.cpu().numpy()[1:] != 0)
    # the stepping interface reports it the same way at its finish
    ch = m.Chain(ts, 3, n_steps=5, k=6, seed=4, sample_offset=7)
    ch.step(5)
    c = ch.finish()
    ch.close()
    assert c.status == m.ENUMERIC
    assert np.array_equal(c.sign.cpu().numpy(), r.sign.cpu().numpy())
    monkeypatch.delenv("MCTRG_TEST_FAIL_SAMPLE")
    ch = m.Chain(ts, 3, n_steps=5, k=6, seed=4, sample_offset=7)
    ch.step(5)
    assert ch.finish().status == m.OK
    ch.close()


def test_enomem_under_a_workspace_cap_leaves_outputs():
    torch, m = need_gpu()
    log("ENOMEM under a 1 MiB workspace cap")
    ts = m.init_tensor("site", [BETA_C], [0.0])
    sign = torch.full((4,), 7, dtype=torch.int8, device="cuda")
    ln = torch.full((4,), 3.5, dtype=torch.float64, device="cuda")
    r = m.run_samples(ts, 4, n_steps=10, k=32, out_sign=sign, out_ln_abs_Z=ln, max_workspace_bytes=1 << 20,
                      allow=(m.ENOMEM,))
    assert r.status == m.ENOMEM
    assert np.all(sign.cpu().numpy() == 7) and np.all(ln.cpu().numpy() == 3.5)
    # a cap that fits one sample at a time runs the samples in waves with the same results
    a = m.run_samples(ts, 4, n_steps=6, k=8, seed=2)
    b = m.run_samples(ts, 4, n_steps=6, k=8, seed=2, max_workspace_bytes=4 << 20)
    assert np.array_equal(a.ln_abs_Z.cpu().numpy(), b.ln_abs_Z.cpu().numpy())


def test_chain_tensor_and_record():
    torch, m = need_gpu()
    log("chain tensor readout and records")
    ts = m.init_tensor("site", [0.42], [0.05])
    ch = m.Chain(ts, 3, n_steps=6, k=6, seed=9, record=True)
    T0 = ch.tensor().cpu().numpy()
    assert T0.shape == (3, 2, 2, 2, 2)
    assert np.allclose(T0[1], ising.site_tensor(0.42, 0.05), rtol=1e-13, atol=0)
    o = trg.run_shared(ising.site_tensor(0.42, 0.05), 6, 6, 9, 1, keep_tensors=True)
    for s in range(6):
        ch.step(1)
        T = ch.tensor().cpu().numpy()[1]
        To = parity.pad_to_capacity(o.records[s].T_hat, T.shape[0])
        assert T.shape == To.shape
        assert np.linalg.norm(T - To) / np.linalg.norm(To) < 1e-10, s
    ch.finish()
    rec = ch.record.cpu().numpy()[1]
    for s, st in enumerate(o.records):
        assert [int(x) for x in rec[s, 4:4 + rec[s, 2]]] == list(st.splits[0].sel)
        assert [int(x) for x in rec[s, 4 + 6:4 + 6 + rec[s, 3]]] == list(st.splits[1].sel)
        assert int(rec[s, 0]) == st.splits[0].c and int(rec[s, 1]) == st.splits[1].c
    ch.close()
