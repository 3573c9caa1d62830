"""The GPU parity gate (tests/parity.py) checked on the CPU.

The gate is what the GPU chains are held to, so it is pinned here against
cases whose answer is known: the same oracle chain computed with a
different LAPACK SVD driver (a correct implementation that rounds
differently) must pass, and the oracle with a planted mistake - one
reweighted value off by 1e-7 relative, or one kept index exchanged for
another - must fail."""
import numpy as np
import pytest
import scipy.linalg as sla

import parity
from oracle import trg
from workloads import C2

K, STEPS = 16, 14
BETAS = (C2.betas[4], C2.betas[9], C2.betas[15])   # 0.38, 0.48, 0.60


def _gesvd(M, cs):
    U, s, Vt = sla.svd(M, full_matrices=False, lapack_driver="gesvd")
    g = Vt @ trg.gauge_weights(cs)
    f = g < 0
    U[:, f] *= -1.0
    Vt[f, :] *= -1.0
    return U, s, Vt


def _as_gpu(ch):
    return ([st.sel for st in ch.steps], [st.c for st in ch.steps], [st.ln_c for st in ch.steps],
            [st.fp for st in ch.steps])


def _gate(ref, test, tau=1e-11):
    sel, c, lnc, fp = _as_gpu(test)
    return parity.compare_chain(ref, sel, c, lnc, fp, K, 0, tau, base=100 * parity.EPS64)


@pytest.fixture(scope="module")
def refs():
    return [parity.oracle_chain_summary(b, 0.0, STEPS, K, 0, i) for i, b in enumerate(BETAS)]


def test_gate_accepts_another_lapack_driver(refs, monkeypatch):
    monkeypatch.setattr(trg, "decompose", _gesvd)
    checked = 0
    for i, b in enumerate(BETAS):
        other = parity.oracle_chain_summary(b, 0.0, STEPS, K, 0, i)
        r = _gate(refs[i], other)
        checked += r.checked
        assert r.checked >= 6, r
    assert checked >= 20


def test_gate_rejects_a_wrong_weight(refs, monkeypatch):
    orig = trg.factors
    calls = {"n": 0}

    def bad(U, Vt, tr, rs, cs):
        calls["n"] += 1
        if calls["n"] == 7:            # step 3, split A
            tr.weights = tr.weights.copy()
            tr.weights[1] *= 1.0 + 1e-7
        return orig(U, Vt, tr, rs, cs)

    monkeypatch.setattr(trg, "factors", bad)
    other = parity.oracle_chain_summary(BETAS[0], 0.0, STEPS, K, 0, 0)
    with pytest.raises(AssertionError):
        _gate(refs[0], other)


def test_gate_rejects_a_flip_away_from_its_threshold(refs):
    ref = refs[0]
    s = 6
    sel, c, lnc, fp = _as_gpu(ref)
    sel = [list(map(list, x)) for x in sel]
    a = sel[s][0]
    # exchange the last kept candidate for the next one not kept
    last = a[-1]
    nxt = next(i for i in range(last + 1, c[s][0]) if i not in a)
    sel[s][0] = sorted(a[:-1] + [nxt])
    with pytest.raises(AssertionError):
        parity.compare_chain(ref, sel, c, lnc, fp, K, 0, 1e-11, base=100 * parity.EPS64)
