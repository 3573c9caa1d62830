"""Parity and statistics at the measured configurations' shapes, through
the C ABI, with the conditioning-aware gate of tests/parity.py (kept sets
equal or a validated rounding-distance flip; per-step values within the
step's conditioning bound).

C1  16 x 16 torus, k = 8, beta_c, independent mode (the paper's estimator):
    per-position parity with the oracle (also on 32 x 32 and 64 x 64 tori,
    10 and 12 steps), and the sample mean of Z~ against Kaufman's exact Z
    over ten seeds (Section III, Eq. infiniteEnsemble; error bars per
    Section V, Eq. shrunkDev).
C2  k = 16 shared chains over the beta sweep 0.30..0.60 (16 values), 20
    steps (2^20 sites), every chain compared step by step.
C3  mixed k in {16, 24, 32}, beta in [0.35, 0.55], h in {0, 0.05}, bucketed
    in one call.
C4  k = 48 at beta_c and C5 k = 64 at beta = 0.42, h = 0.1: the first steps
    at the full bond dimension (unfoldings of 2304 and 4096 rows).
"""
import math

import numpy as np
import pytest

import parity
from oracle import ising, trg
from workloads import BETA_C, C2, C3

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu

BASE64 = 100 * parity.EPS64


def _independent_gate(m, n_steps, k, picks, seed=0):
    ts = m.init_tensor("site", [BETA_C], [0.0])
    ns = max(picks) + 1
    r = m.run_samples(ts, ns, n_steps=n_steps, k=k, mode="independent", seed=seed, record=True, want_ln_c=True)
    assert r.status == m.OK
    rec, lnc, ln = r.record.cpu().numpy(), r.ln_c.cpu().numpy(), r.ln_abs_Z.cpu().numpy()
    T0 = ising.site_tensor(BETA_C)
    N = 2.0 ** n_steps
    out = []
    for i in picks:
        o = trg.run_independent(T0, n_steps, k, seed, i)
        levels = m.split_independent_record(rec[i], n_steps)
        g = parity.compare_independent(o, levels, lnc[i], k, seed, i, 1e-11, BASE64)
        log(f"independent {n_steps} steps sample {i}: compared {g.checked} steps, stop {g.stopped_at} "
            f"({g.reason}), worst |d sum ln c| {g.worst_dlnc:.2e}, |d lnZ|/site {abs(ln[i] - o.ln_abs_Z) / N:.2e}")
        for n in g.notes:
            log("   " + n)
        if g.reason == "end":
            assert abs(ln[i] - o.ln_abs_Z) / N < 1e-12
        out.append(g)
    return out


def test_c1_independent_parity():
    torch, m = need_gpu()
    log("C1 parity (16 x 16, 8 steps)")
    res = _independent_gate(m, 8, 8, list(range(8)))
    assert sum(g.reason == "end" for g in res) >= 6


@pytest.mark.parametrize("n_steps,picks", [(10, [0, 1, 2]), (12, [0, 1])])
def test_independent_parity_larger_tori(n_steps, picks):
    torch, m = need_gpu()
    log(f"independent parity, {2 ** (n_steps // 2)} x {2 ** (n_steps // 2)} torus")
    res = _independent_gate(m, n_steps, 8, picks)
    assert all(g.checked >= 4 for g in res)


def test_c1_unbiased_against_kaufman():
    """Ten seeds of 1000 samples: the pooled mean of Z~/Z within two
    standard errors of 1 and the ten z-scores consistent with N(0,1) (sum
    of squares below the 99 % point of chi^2 with 10 degrees, 23.21)."""
    torch, m = need_gpu()
    log("C1 1000 samples x 10 seeds vs Kaufman")
    ts = m.init_tensor("site", [BETA_C], [0.0])
    lnZ = ising.kaufman_lnZ_torus(16, BETA_C)
    zs, allv = [], []
    for seed in range(10):
        r = m.run_samples(ts, 1000, n_steps=8, k=8, mode="independent", seed=seed)
        assert r.status == m.OK
        v = r.sign.cpu().numpy() * np.exp(r.ln_abs_Z.cpu().numpy() - lnZ)     # Z~ / Z
        mean, se = v.mean(), v.std(ddof=1) / math.sqrt(v.size)
        zs.append((mean - 1.0) / se)
        allv.append(v)
        log(f"C1 seed {seed}: mean Z~/Z = {mean:.5f} +- {se:.5f} (z = {zs[-1]:+.2f}), negatives "
            f"{int(np.sum(v < 0))}")
        if seed == 0:
            est = m.estimate_lnZ(r.sign, r.ln_abs_Z, 256.0)
            assert est["ln_meanZ_per_site"] == pytest.approx(lnZ / 256 + math.log(mean) / 256, abs=1e-12)
    v = np.concatenate(allv)
    mean, se = v.mean(), v.std(ddof=1) / math.sqrt(v.size)
    log(f"C1 pooled: mean Z~/Z = {mean:.5f} +- {se:.5f} (z = {(mean - 1) / se:+.2f}); z-scores "
        f"{[round(z, 2) for z in zs]}, sum of squares {sum(z * z for z in zs):.2f}")
    assert abs(mean - 1.0) <= 2.0 * se
    assert sum(z * z for z in zs) < 23.21


def test_c2_beta_sweep_parity():
    """All 16 chains (one per beta) over 20 steps, compared step by step
    with fingerprints of the normalised tensor.  The first eight steps must
    be compared in every chain; later steps as far as the gate's
    conditioning bound allows (two LAPACK drivers running the oracle itself
    part within 10-13 steps at most of these temperatures)."""
    torch, m = need_gpu()
    betas = list(C2.betas)
    log("C2 beta sweep")
    futs = parity.start_oracle_pool([dict(beta=b, h=0.0, n_steps=20, k=16, seed=0, sid=i)
                                     for i, b in enumerate(betas)], workers=8)
    ts = m.init_tensor("site", betas, [0.0] * len(betas))
    g = parity.gpu_chain_trace(m, ts, len(betas), 20, 16, list(range(len(betas))), groups=list(range(len(betas))),
                               log=log)
    checked = []
    for i, (b, f) in enumerate(zip(betas, futs)):
        orc = f.result(timeout=900)
        r = parity.compare_chain(orc, g[i]["sel"], g[i]["c"], g[i]["lnc"], g[i]["fp"], 16, 0, 1e-11, BASE64)
        log(f"beta {b:.3f}: compared {r.checked} steps ({r.tensor_checked} with tensors, {r.tight} with a tensor bound <= 1e-4), stop {r.stopped_at} "
            f"({r.reason}), worst delta {r.worst_delta:.2e}, worst |d ln c| {r.worst_dlnc:.2e} (largest tolerance "
            f"{r.worst_tau:.1e})")
        for n in r.notes:
            log("   " + n)
        checked.append(r.checked)
        if r.reason == "end" and r.lnZ_tol is not None:
            assert abs(g[i]["ln_abs_Z"] - orc.ln_abs_Z) / 2.0 ** 20 <= r.lnZ_tol
    log(f"C2 steps compared per chain: {checked}")
    assert min(checked) >= 8


def test_c3_mixed_k_parity():
    torch, m = need_gpu()
    log("C3 mixed k")
    betas = [C3.betas[0], C3.betas[13], C3.betas[31]]
    hs = [0.0, 0.05, 0.05]
    ts = m.init_tensor("site", betas, hs)
    ks = [16, 24, 32, 24, 32, 16]
    groups = [0, 1, 2, 2, 0, 1]
    n_steps = 8
    futs = parity.start_oracle_pool([dict(beta=betas[groups[i]], h=hs[groups[i]], n_steps=n_steps, k=ks[i], seed=0,
                                          sid=i) for i in range(6)], workers=6)
    r = m.run_samples(ts, 6, n_steps=n_steps, k=32, ks=ks, groups=groups, seed=0, dtype="f64", record=True,
                      want_ln_c=True)
    ln, rec, lnc = r.ln_abs_Z.cpu().numpy(), r.record.cpu().numpy(), r.ln_c.cpu().numpy()
    for i, f in enumerate(futs):
        orc = f.result(timeout=900)
        kk = ks[i]
        sel = [[list(map(int, rec[i, s, 4:4 + rec[i, s, 2]])), list(map(int, rec[i, s, 4 + 32:4 + 32 + rec[i, s, 3]]))]
               for s in range(n_steps)]
        c = [[int(rec[i, s, 0]), int(rec[i, s, 1])] for s in range(n_steps)]
        g = parity.compare_chain(orc, sel, c, lnc[i], None, kk, 0, 1e-11, BASE64)
        log(f"C3 sample {i} (k={kk}): compared {g.checked} steps ({g.reason}); {g.notes}")
        assert g.checked >= 6
        if g.reason == "end":
            assert abs(ln[i] - orc.ln_abs_Z) / 2.0 ** n_steps < 1e-12


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("bf16", 5e-3)])
def test_low_precision_topk_error(dtype, tol):
    """Top-k chains are deterministic, so a narrow contraction dtype can be
    compared paired with FP64: |d ln Z|/site stays within a bound set by the
    dtype's unit roundoff."""
    torch, m = need_gpu()
    log(f"precision {dtype}")
    ts = m.init_tensor("site", [BETA_C], [0.0])
    a = m.run_samples(ts, 1, n_steps=12, k=16, mode="topk", dtype="f64").ln_abs_Z.cpu().numpy()
    b = m.run_samples(ts, 1, n_steps=12, k=16, mode="topk", dtype=dtype).ln_abs_Z.cpu().numpy()
    err = abs(a[0] - b[0]) / 2.0 ** 12
    log(f"topk k=16 {dtype}: |d lnZ|/site = {err:.3e}")
    assert err < tol


def _large_k_parity(k, beta, h, n_steps, ns):
    torch, m = need_gpu()
    futs = parity.start_oracle_pool([dict(beta=beta, h=h, n_steps=n_steps, k=k, seed=1, sid=i) for i in range(ns)],
                                    workers=ns)
    ts = m.init_tensor("site", [beta], [h])
    r = m.run_samples(ts, ns, n_steps=n_steps, k=k, seed=1, dtype="f64", want_ln_c=True, record=True)
    ln, lnc, rec = r.ln_abs_Z.cpu().numpy(), r.ln_c.cpu().numpy(), r.record.cpu().numpy()
    res = []
    for i, f in enumerate(futs):
        orc = f.result(timeout=1200)
        sel = [[list(map(int, rec[i, s, 4:4 + rec[i, s, 2]])), list(map(int, rec[i, s, 4 + k:4 + k + rec[i, s, 3]]))]
               for s in range(n_steps)]
        c = [[int(rec[i, s, 0]), int(rec[i, s, 1])] for s in range(n_steps)]
        g = parity.compare_chain(orc, sel, c, lnc[i], None, k, 1, 1e-11, BASE64)
        log(f"k={k} sample {i}: compared {g.checked} steps ({g.reason}), worst |d ln c| {g.worst_dlnc:.2e}, "
            f"|d lnZ|/site {abs(ln[i] - orc.ln_abs_Z) / 2.0 ** n_steps:.2e}; {g.notes}")
        res.append(g)
    return res


def test_c4_k48_parity():
    log("C4 k=48")
    res = _large_k_parity(48, BETA_C, 0.0, 8, 2)
    assert all(g.checked >= 5 for g in res)


def test_c5_k64_parity():
    log("C5 k=64")
    res = _large_k_parity(64, 0.42, 0.1, 8, 1)
    assert all(g.checked >= 5 for g in res)
