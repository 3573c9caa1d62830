"""Chain-level parity: whole Monte Carlo TRG samples on the GPU against the
CPU oracle with identical Philox draws (paper Section III).

For every sample both sides must make the same selections at every step
(a "flip" is a selection that differs; with FP64 on both sides flips can
only come from a uniform falling within rounding distance of its threshold)
and then agree on ln|Z~| per site to 1e-12 and on the final normalised
tensor to 1e-10 relative (FP64 form).  Exact contraction (k >= rank) must
reproduce brute-force Z."""
import math

import numpy as np
import pytest

from oracle import ising, trg
from oracle.estimate import estimate_lnZ
from workloads import BETA_C

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


def oracle_records(res):
    rows = []
    for st in res.records:
        a, b = st.splits
        rows.append((a.c, b.c, len(a.sel), len(b.sel), list(a.sel), list(b.sel)))
    return rows


def gpu_records(rec, k):
    rows = []
    for st in rec:
        cA, cB, kA, kB = (int(x) for x in st[:4])
        rows.append((cA, cB, kA, kB, [int(x) for x in st[4:4 + kA]], [int(x) for x in st[4 + k:4 + k + kB]]))
    return rows


def align_gauge(Tg, To):
    """Per-index sign gauge on bonds: T[a,b,c,e] -> s_a t_b s_c t_e T; choose
    the signs from the largest entries and return the aligned GPU tensor."""
    D = To.shape[0]
    s = np.ones(D)
    t = np.ones(D)
    # s_a s_c from T[a, b*, c, b*] slices with the dominant b*
    for a in range(D):
        sl_o = To[0, :, a, :]
        sl_g = Tg[0, :, a, :]
        idx = np.unravel_index(np.argmax(np.abs(sl_o)), sl_o.shape)
        if abs(sl_o[idx]) > 0:
            s[a] = np.sign(sl_g[idx] * sl_o[idx])   # s_0 s_a with s_0 = 1
    for b in range(D):
        sl_o = To[:, 0, :, b]
        sl_g = Tg[:, 0, :, b] * s[:, None] * s[None, :]
        idx = np.unravel_index(np.argmax(np.abs(sl_o)), sl_o.shape)
        if abs(sl_o[idx]) > 0:
            t[b] = np.sign(sl_g[idx] * sl_o[idx])
    return np.einsum("abce,a,b,c,e->abce", Tg, s, t, s, t)


# k = 9, 12, 13, 14, 20: steady unfoldings with n_pad = 96, 160, 192, 224,
# 416, which end the 128-column steps of the QR preconditioning after one
# panel, one 64-column block, one and a half blocks, or several full steps
@pytest.mark.parametrize("k,n_steps,beta,h,dtype", [(4, 6, BETA_C, 0.0, "f64"), (8, 8, BETA_C, 0.0, "f64"),
                                                    (6, 7, 0.42, 0.1, "f64"), (16, 6, 0.35, 0.05, "f64"),
                                                    (9, 6, BETA_C, 0.0, "f64"), (12, 6, 0.42, 0.1, "f64"),
                                                    (13, 6, BETA_C, 0.0, "f64"), (14, 6, 0.35, 0.05, "f64"),
                                                    (20, 6, BETA_C, 0.0, "f64")])
def test_shared_chain_matches_oracle(k, n_steps, beta, h, dtype):
    torch, m = need_gpu()
    log(f"shared chain k={k} steps={n_steps} beta={beta} h={h}")
    ts = m.init_tensor("site", [beta], [h])
    ns, seed, off = 12, 3, 40
    r = m.run_samples(ts, ns, n_steps=n_steps, k=k, seed=seed, sample_offset=off, want_ln_c=True, record=True,
                      want_tensor=True, dtype=dtype)
    assert r.status == m.OK
    sign, ln = r.sign.cpu().numpy(), r.ln_abs_Z.cpu().numpy()
    rec, ten, lnc = r.record.cpu().numpy(), r.tensor.cpu().numpy(), r.ln_c.cpu().numpy()
    T0 = ising.site_tensor(beta, h)
    N = 2.0 ** n_steps
    flips = 0
    for i in range(ns):
        o = trg.run_shared(T0, n_steps, k, seed, off + i, keep_tensors=True)
        ro, rg = oracle_records(o), gpu_records(rec[i], k)
        if ro != rg:
            flips += 1
            continue
        assert sign[i] == o.sign
        assert abs(ln[i] - o.ln_abs_Z) / N < 1e-12
        assert np.allclose(lnc[i], o.ln_c, rtol=0, atol=1e-10)
        To = o.records[-1].T_hat
        Dc = ten.shape[1]
        Tg = ten[i][:To.shape[0], :To.shape[1], :To.shape[2], :To.shape[3]]
        assert np.max(np.abs(ten[i])) == pytest.approx(1.0)
        if Tg.shape[0] == To.shape[0] and To.shape[0] == Dc:
            Ta = align_gauge(Tg, To)
            assert np.linalg.norm(Ta - To) / np.linalg.norm(To) < 1e-10
    assert flips <= 1, f"{flips} of {ns} samples made a different selection"


@pytest.mark.parametrize("L,n", [(2, 2), (4, 4)])
def test_exact_contraction_equals_brute_force(L, n):
    torch, m = need_gpu()
    log(f"exact L={L}")
    beta, h = 0.42, 0.1
    ts = m.init_tensor("site", [beta], [h])
    # k = 64 keeps every nonzero singular value at these sizes
    r = m.run_samples(ts, 2, n_steps=n, k=64, mode="topk")
    bf = ising.brute_force_lnZ_torus(L, beta, h)
    assert np.all(r.sign.cpu().numpy() == 1)
    assert np.allclose(r.ln_abs_Z.cpu().numpy(), bf, rtol=0, atol=1e-11)


def test_plaquette_exact():
    torch, m = need_gpu()
    ts = m.init_tensor("plaquette", [0.5], [0.2])
    r = m.run_samples(ts, 1, n_steps=2, k=64, mode="topk")
    assert r.ln_abs_Z.cpu().numpy()[0] == pytest.approx(ising.brute_force_lnZ_medial(2, 0.5, 0.2), abs=1e-11)


@pytest.mark.parametrize("k,n_steps", [(2, 4), (4, 4), (8, 6)])
def test_independent_matches_oracle(k, n_steps):
    """Independent mode, every position of every level: the kept sets must
    be the oracle's (a differing one must be a validated rounding-distance
    flip, after which the sample is no longer compared), the per-step sums
    of ln c within the conditioning bound, and ln|Z~| per site to 1e-12
    for samples compared to the end."""
    import parity
    torch, m = need_gpu()
    log(f"independent k={k} steps={n_steps}")
    beta = BETA_C
    ts = m.init_tensor("site", [beta], [0.0])
    ns, seed = 6 if n_steps == 4 else 3, 11
    r = m.run_samples(ts, ns, n_steps=n_steps, k=k, mode="independent", seed=seed, want_ln_c=True, record=True)
    ln, lnc, rec = r.ln_abs_Z.cpu().numpy(), r.ln_c.cpu().numpy(), r.record.cpu().numpy()
    T0 = ising.site_tensor(beta)
    N = 2.0 ** n_steps
    ends = 0
    for i in range(ns):
        o = trg.run_independent(T0, n_steps, k, seed, i)
        g = parity.compare_independent(o, m.split_independent_record(rec[i], n_steps), lnc[i], k, seed, i, 1e-11,
                                       100 * parity.EPS64)
        log(f"sample {i}: {g.checked} steps compared ({g.reason}) {g.notes}")
        if g.reason == "end":
            ends += 1
            assert abs(ln[i] - o.ln_abs_Z) / N <= 1e-12
    assert ends >= ns - 1


def test_topk_matches_oracle():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    r = m.run_samples(ts, 2, n_steps=8, k=8, mode="topk")
    o = trg.run(ising.site_tensor(BETA_C), 8, 8, 0, 0, mode="topk")
    assert np.allclose(r.ln_abs_Z.cpu().numpy(), o.ln_abs_Z, rtol=0, atol=256 * 1e-12)


def test_batch_independence_and_groups():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [0.40, 0.45], [0.0, 0.02])
    groups = [0, 1, 1, 0, 1, 0]
    ks = [4, 6, 4, 6, 6, 4]
    a = m.run_samples(ts, 6, n_steps=6, k=6, groups=groups, ks=ks, seed=5)
    b = m.run_samples(ts, 3, n_steps=6, k=6, groups=groups[3:], ks=ks[3:], seed=5, sample_offset=3)
    la, lb = a.ln_abs_Z.cpu().numpy(), b.ln_abs_Z.cpu().numpy()
    assert np.array_equal(la[3:], lb)
    # every sample equals the oracle sample of its own group and k
    for i in range(6):
        beta, h = (0.40, 0.0) if groups[i] == 0 else (0.45, 0.02)
        o = trg.run_shared(ising.site_tensor(beta, h), 6, ks[i], 5, i)
        assert abs(la[i] - o.ln_abs_Z) / 64 < 1e-11


def test_estimate_matches_oracle():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [BETA_C], [0.0])
    r = m.run_samples(ts, 40, n_steps=6, k=4, seed=1)
    est = m.estimate_lnZ(r.sign, r.ln_abs_Z, 64.0)
    o = estimate_lnZ(r.sign.cpu().numpy(), r.ln_abs_Z.cpu().numpy(), 64.0)
    assert est["n_used"] == o.n_used and est["n_negative"] == o.n_negative
    assert est["ln_meanZ_per_site"] == pytest.approx(o.ln_meanZ_per_site, rel=1e-13)
    assert est["rel_stderr_Z"] == pytest.approx(o.rel_stderr_Z, rel=1e-10)
    assert est["mean_lnZ_per_site"] == pytest.approx(o.mean_lnZ_per_site, rel=1e-13)
    assert est["stderr_mean_lnZ"] == pytest.approx(o.stderr_mean_lnZ, rel=1e-10)


def test_argument_errors_leave_outputs():
    torch, m = need_gpu()
    ts = m.init_tensor("site", [0.4], [0.0])
    sign = torch.full((4,), 7, dtype=torch.int8, device="cuda")
    ln = torch.full((4,), 3.5, dtype=torch.float64, device="cuda")
    for kw in ({"k": 0}, {"k": 65}, {"n_steps": 0}, {"n_steps": 41}):
        args = dict(n_steps=4, k=4)
        args.update(kw)
        with pytest.raises(m.MctrgError) as e:
            m.run_samples(ts, 4, out_sign=sign, out_ln_abs_Z=ln, **args)
        assert e.value.status == m.EINVAL
    with pytest.raises(m.MctrgError):
        m.run_samples(ts, 4, n_steps=5, k=4, mode="independent", out_sign=sign, out_ln_abs_Z=ln)
    with pytest.raises(m.MctrgError):
        m.run_samples(ts, 4, n_steps=4, k=4, groups=[0, 1, 0, 0], out_sign=sign, out_ln_abs_Z=ln)
    assert np.all(sign.cpu().numpy() == 7) and np.all(ln.cpu().numpy() == 3.5)
    r = m.run_samples(ts, 0, n_steps=4, k=4)
    assert r.status == m.OK


def test_chain_api_matches_run_samples():
    torch, m = need_gpu()
    log("chain api")
    ts = m.init_tensor("site", [0.42], [0.05])
    a = m.run_samples(ts, 5, n_steps=7, k=6, seed=9, want_ln_c=True)
    ch = m.Chain(ts, 5, n_steps=7, k=6, seed=9, profile=True)
    ch.step(3)
    ch.step(4)
    b = ch.finish(want_ln_c=True)
    prof = ch.profile()
    # five samples run as three parts (2 + 2 + 1), one GEMM per part and step
    assert prof["parts"] == 3
    assert prof["steps_done"] == 7 and prof["jacobi_launches"] > 0 and prof["gemm_launches"] == 7 * prof["parts"]
    assert np.array_equal(a.ln_abs_Z.cpu().numpy(), b.ln_abs_Z.cpu().numpy())
    assert np.array_equal(a.ln_c.cpu().numpy(), b.ln_c.cpu().numpy())
    # a partial chain traces the 2^s-site lattice: compare with the oracle
    ch2 = m.Chain(ts, 2, n_steps=7, k=6, seed=9)
    ch2.step(4)
    p = ch2.finish()
    for i in range(2):
        o = trg.run_shared(ising.site_tensor(0.42, 0.05), 4, 6, 9, i)
        assert abs(p.ln_abs_Z.cpu().numpy()[i] - o.ln_abs_Z) / 16 < 1e-12


@pytest.mark.parametrize("mode,k,n_steps,ns", [("shared", 8, 8, 5), ("independent", 4, 4, 3), ("topk", 8, 6, 4)])
def test_two_parts_match_one(mode, k, n_steps, ns):
    """A wave of two or more samples runs as up to three parts on their own streams; the
    results must be those of a single part, bit for bit (every draw is
    addressed by the global sample id, every decomposition is independent)."""
    torch, m = need_gpu()
    log(f"several parts vs one: {mode} k={k} steps={n_steps} samples={ns}")
    ts = m.init_tensor("site", [BETA_C, 0.42], [0.0, 0.1])
    kw = dict(n_steps=n_steps, k=k, mode=mode, seed=7, sample_offset=11, groups=[i % 2 for i in range(ns)],
              want_ln_c=True, record=True)
    if mode != "independent":
        kw.update(want_tensor=True)
    a = m.run_samples(ts, ns, **kw)
    b = m.run_samples(ts, ns, one_stream=True, **kw)
    assert a.status == b.status == m.OK
    for f in ("sign", "ln_abs_Z", "ln_c", "record", "tensor"):
        x, y = getattr(a, f), getattr(b, f)
        if x is None:
            assert y is None
            continue
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy(), equal_nan=True), f


def test_chain_parts_profile():
    torch, m = need_gpu()
    log("chain parts profile")
    ts = m.init_tensor("site", [BETA_C], [0.0])
    ch = m.Chain(ts, 6, n_steps=6, k=8, seed=3, profile=True)
    ch.step(6)
    p = ch.profile()
    assert p["parts"] == 3 and p["steps_done"] == 6
    assert p["jacobi_launches"] > 0 and 0.0 < p["jacobi_busy_ms"] <= p["jacobi_ms"] + 1e-3
    r = ch.finish()
    one = m.Chain(ts, 6, n_steps=6, k=8, seed=3, profile=True, one_stream=True)
    one.step(6)
    assert one.profile()["parts"] == 1
    r1 = one.finish()
    assert torch.equal(r.sign, r1.sign) and torch.equal(r.ln_abs_Z, r1.ln_abs_Z)
    ch.close()
    one.close()


def test_mixed_k_buckets_run_concurrently_with_unchanged_results():
    """Samples of different k run as concurrent buckets; every sample must be
    the sample that a call with only that sample gives, bit for bit (draws
    are addressed by the global sample id, each bucket has its own
    workspace, and every decision of the decomposition is taken per job)."""
    torch, m = need_gpu()
    log("mixed k buckets")
    ts = m.init_tensor("site", [0.41, 0.46], [0.0, 0.03])
    ks = [8, 12, 8, 16, 12, 16, 8]
    groups = [0, 1, 1, 0, 0, 1, 0]
    a = m.run_samples(ts, len(ks), n_steps=7, k=16, ks=ks, groups=groups, seed=4, want_ln_c=True, record=True)
    la, lca, ra = a.ln_abs_Z.cpu().numpy(), a.ln_c.cpu().numpy(), a.record.cpu().numpy()
    for i, (k, g) in enumerate(zip(ks, groups)):
        b = m.run_samples(ts, 1, n_steps=7, k=16, ks=[k], groups=[g], seed=4, sample_offset=i, want_ln_c=True,
                          record=True)
        assert np.array_equal(ra[i], b.record.cpu().numpy()[0]), i
        assert la[i] == b.ln_abs_Z.cpu().numpy()[0], i
        assert np.array_equal(lca[i], b.ln_c.cpu().numpy()[0]), i


@pytest.mark.parametrize("dtype,tau", [("f64", 1e-11), ("f32", 1e-6)])
def test_results_do_not_depend_on_the_batch(dtype, tau):
    """A sample's result depends only on its global id and parameters, not on
    the samples that share its batch or part: at k = 32 (unfoldings of 1024
    rows through the re-ordered first QR with its early stop, the rank
    limit, the three-or-five QR choice and the deflation, all of which vary
    between the two temperature groups and between the steps), six samples
    in one part, in three parts, and each alone give the same per-step ln c,
    kept sets and ln|Z~|, bit for bit."""
    torch, m = need_gpu()
    log(f"batch independence k=32 {dtype}")
    ts = m.init_tensor("site", [BETA_C, 0.42], [0.0, 0.1])
    groups = [0, 1, 0, 1, 1, 0]
    kw = dict(n_steps=9, k=32, seed=21, dtype=dtype, tau_null=tau, want_ln_c=True, record=True)
    one = m.run_samples(ts, 6, groups=groups, one_stream=True, **kw)
    three = m.run_samples(ts, 6, groups=groups, **kw)
    for f in ("sign", "ln_abs_Z", "ln_c", "record"):
        assert np.array_equal(getattr(one, f).cpu().numpy(), getattr(three, f).cpu().numpy()), f
    for i, g in enumerate(groups):
        b = m.run_samples(ts, 1, groups=[g], sample_offset=i, **kw)
        for f in ("sign", "ln_abs_Z", "ln_c", "record"):
            assert np.array_equal(getattr(one, f).cpu().numpy()[i], getattr(b, f).cpu().numpy()[0]), (i, f)
