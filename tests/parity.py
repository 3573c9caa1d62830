"""Conditioning-aware comparison of GPU chains with oracle chains.

Test infrastructure (imports the oracle).  A Monte Carlo TRG chain is a
sequence of SVD truncations, each of which amplifies a perturbation of its
input: a kept singular vector whose value lies close to a value that was not
kept, or a small kept value, moves by up to kappa times the perturbation,
with (singular values relative to s_1, over both splits of the step)

    kappa_s = max(1 / min |s_i - s_j| over kept i and not-kept neighbours j,
                  1 / min kept s_i).

Two correct FP64 implementations therefore agree on step s only to about
    delta_s <= kappa_s * (base + delta_{s-1}),
where delta is the relative Frobenius distance of the normalised tensors and
base the rounding level of one step.  Two LAPACK drivers running the same
oracle chain obey this with a margin of ~30 and still drift apart to O(1)
within 10-13 steps at the C2 temperatures.  The gate below checks every
step until the kept sets differ: the tensors within 3 kappa_s (base +
delta_in) and ln c within kappa_tau (base + delta_in) (kappa_tau adds the
squared smallest kept value, which governs the inclusion rates), delta_in
being the measured discrepancy of the step's input.  A step where the kept
sets differ (a flip) must be a rounding-distance event: the uniform u of the
first differing decision must lie within the interval that q (the
probability of keeping that candidate, Section II's sequential draw) sweeps
when every singular value moves by (2 base + delta_in) s_1; the chain is
compared no further.

Tensors are compared through J = 64 Gaussian fingerprints
f_j = vec(P_j)^T M_A(T) vec(Q_j), whose mean square estimates ||T||_F^2.
"""
from __future__ import annotations

import math
import multiprocessing as mp
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

EPS64 = 2.0 ** -52
HOST_THREADS = 16          # host cores the oracle pools may use together


def kappa_tau(sigma: np.ndarray, c: int, sel) -> float:
    """The conditioning of the per-step tolerance tau_T = max(floor, 100 u
    kappa) of one decomposition: max(1 / min gap between a kept value and a
    neighbour not kept, 1 / (smallest kept value)^2), values relative to
    s_1 (the squared term covers the inclusion rates, which depend on the
    squared values of every candidate)."""
    sig = np.asarray(sigma[:c], dtype=np.float64) / float(sigma[0])
    sel = set(int(j) for j in sel)
    if not sel:
        return 1.0
    gmin = math.inf
    for j in sel:
        for j2 in (j - 1, j + 1):
            if 0 <= j2 < c and j2 not in sel:
                gmin = min(gmin, abs(sig[j] - sig[j2]))
    k1 = 1.0 / gmin if gmin > 0 else math.inf
    smin = min(sig[j] for j in sel)
    return max(k1, 1.0 / (smin * smin))


def kappa_split(sigma: np.ndarray, c: int, sel) -> float:
    sig = np.asarray(sigma[:c], dtype=np.float64) / float(sigma[0])
    sel = set(int(j) for j in sel)
    if not sel:
        return 1.0
    gmin = math.inf
    for j in sel:
        for j2 in (j - 1, j + 1):
            if 0 <= j2 < c and j2 not in sel:
                gmin = min(gmin, abs(sig[j] - sig[j2]))
    k1 = 1.0 / gmin if gmin > 0 else math.inf
    k2 = 1.0 / min(sig[j] for j in sel)
    return max(k1, k2)


def pad_to_capacity(T: np.ndarray, D: int) -> np.ndarray:
    """The oracle keeps exactly the kept count on every new leg; the library
    stores every tensor at the capacity bond dimension D = min(k, D_prev^2)
    with zero padding after the kept indices.  Same padding here."""
    out = np.zeros((D, D, D, D))
    a, b, c, e = T.shape
    out[:a, :b, :c, :e] = T
    return out


def fingerprint(T: np.ndarray, P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    D = T.shape[0]
    M = np.asarray(T, dtype=np.float64).reshape(D * D, D * D)
    return np.einsum("ja,ab,jb->j", P, M, Q)


@dataclass
class OracleStep:
    ln_c: float
    c: List[int]
    sel: List[List[int]]
    sigma: List[np.ndarray]          # candidate spectra (first c values), both splits
    kappa: float                     # amplification of a tensor perturbation (kappa_split)
    fp: np.ndarray
    norm: float
    kappa_t: float = 1.0             # conditioning of the ln c tolerance (kappa_tau)


@dataclass
class OracleChain:
    sid: int
    steps: List[OracleStep]
    ln_abs_Z: float
    sign: int


def oracle_chain_summary(beta, h, n_steps, k, seed, sid, tau_null=1e-11, mode="shared", J=64, threads=None):
    """Runs one oracle chain and keeps, per step, what the gate needs
    (``threads``: BLAS threads of this process, None = unchanged)."""
    if threads:
        from threadpoolctl import threadpool_limits
        threadpool_limits(threads)
    from oracle import ising, trg
    from workloads import projection_pairs
    res = trg.run_shared(ising.site_tensor(beta, h), n_steps, k, seed, sid, mode=mode, tau_null=tau_null,
                         keep_tensors=True)
    steps = []
    D = 2
    for st in res.records:
        D = min(k, D * D)
        T = pad_to_capacity(st.T_hat, D)
        P, Q = projection_pairs(D, J)
        kap = max(kappa_split(sp.sigma, sp.c, sp.sel) for sp in st.splits)
        steps.append(OracleStep(st.ln_c, [sp.c for sp in st.splits], [list(map(int, sp.sel)) for sp in st.splits],
                                [np.array(sp.sigma[:min(sp.sigma.size, sp.c + 64)]) for sp in st.splits], kap,
                                fingerprint(T, P, Q), float(np.linalg.norm(T)),
                                max(kappa_tau(sp.sigma, sp.c, sp.sel) for sp in st.splits)))
    return OracleChain(sid, steps, res.ln_abs_Z, res.sign)


def start_oracle_pool(specs, workers=8):
    """Starts the oracle chains (dicts of oracle_chain_summary arguments) in
    spawned worker processes; returns the futures in order."""
    workers = max(1, min(workers, len(specs)))
    threads = max(1, HOST_THREADS // workers)
    ex = ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))
    futs = [ex.submit(oracle_chain_summary, **dict(sp, threads=sp.get("threads", threads))) for sp in specs]
    ex.shutdown(wait=False)
    return futs


def _suffix_table(ll: np.ndarray, kmax: int) -> np.ndarray:
    c = ll.size
    LS = np.full((kmax + 1, c + 1), -math.inf)
    LS[0, :] = 0.0
    for m in range(c - 1, -1, -1):
        LS[1:, m] = np.logaddexp(LS[1:, m + 1], ll[m] + LS[:-1, m + 1])
    return LS


def decision_q(sigma: np.ndarray, c: int, k: int, sel_prefix: List[int], m: int) -> Optional[float]:
    """Probability that the sequential draw keeps candidate m given the kept
    indices before m (Section II's p(e), conditioned on the earlier
    decisions); None when the decision at m is forced."""
    rem = k - len(sel_prefix)
    if rem <= 0:
        return None
    if rem == c - m:
        return None
    s = np.asarray(sigma[:c], dtype=np.float64)
    ll = 2.0 * np.log(s / s[0])
    LS = _suffix_table(ll[m + 1:], rem)
    lr = ll[m] + LS[rem - 1, 0] - np.logaddexp(LS[rem, 0], ll[m] + LS[rem - 1, 0])
    return math.exp(lr)


def q_interval(sigma, c, k, sel_prefix, m, delta):
    """Range of the decision probability at m when every candidate value
    moves by at most delta * s_1 (q grows with s_m and falls with the later
    values, so the extremes move them in opposite directions; q does not
    change when all values are scaled)."""
    s = np.asarray(sigma[:c], dtype=np.float64) / float(sigma[0])
    hi_s, lo_s = s.copy(), s.copy()
    hi_s[m] += delta
    hi_s[m + 1:] = np.maximum(s[m + 1:] - delta, s[m + 1:] * 1e-3)
    lo_s[m] = max(s[m] - delta, s[m] * 1e-3)
    lo_s[m + 1:] += delta
    qa = decision_q(hi_s, c, k, sel_prefix, m)
    qb = decision_q(lo_s, c, k, sel_prefix, m)
    return min(qa, qb), max(qa, qb)


@dataclass
class GateResult:
    checked: int = 0                           # steps whose kept sets and ln c were compared
    tensor_checked: int = 0                    # of those, steps whose tensors were compared too
    tight: int = 0                             # steps compared with a tensor bound <= 1e-4
    stopped_at: Optional[int] = None           # first step not compared (a flip)
    reason: str = "end"                        # end | flip
    max_ratio: float = 0.0                     # worst measured / bound over compared values
    worst_delta: float = 0.0
    worst_dlnc: float = 0.0
    worst_tau: float = 0.0                     # largest ln c tolerance used
    lnZ_tol: Optional[float] = None            # tolerance of ln|Z~| per site (None: not comparable)
    notes: List[str] = field(default_factory=list)


def check_flip(sigma, c, sel, gsel, gc, k, tau, delta, u_of, notes, label):
    """Asserts that a decomposition whose kept set or candidate count differs
    from the oracle's (spectrum sigma, c candidates, kept set sel) does so
    by a rounding-distance event; u_of(m) is the uniform of candidate m."""
    a, b = [int(x) for x in gsel], [int(x) for x in sel]
    co, cg = int(c), int(gc)
    sig = np.asarray(sigma, dtype=np.float64) / float(sigma[0])
    if cg != co:
        # the values between the two counts must lie within the perturbation of the cut
        lo_i, hi_i = min(cg, co), max(cg, co)
        v = sig[lo_i:hi_i]
        # values beyond the stored spectrum lie below its last entry
        beyond = hi_i > sig.size
        assert not beyond or 10.0 * delta >= tau, (label, cg, co, "candidate counts differ beyond the stored spectrum")
        assert np.all(np.abs(v - tau) <= 10.0 * delta + 1e-3 * tau), (label, cg, co, v, tau, delta)
        notes.append(f"{label}: candidate count {cg} vs {co} (values {v} at the cut {tau:g})")
    if a == b:
        return
    m = min(set(a).symmetric_difference(set(b)))
    prefix = [i for i in b if i < m]
    q = decision_q(sig, co, k, prefix, m)
    if q is None:
        assert cg != co, (label, m, "a forced decision differs")
        return
    u = u_of(m)
    lo, hi = q_interval(sig, co, k, prefix, m, 10.0 * delta)
    notes.append(f"{label}: flip at candidate {m}, u={u:.9g} q={q:.9g} interval [{lo:.9g}, {hi:.9g}]")
    assert lo <= u <= hi, (label, m, u, q, lo, hi, "flip outside the rounding interval")


def compare_chain(orc: OracleChain, gpu_sel, gpu_c, gpu_lnc, gpu_fp, k, seed, tau, base, lnc_floor=1e-10,
                  tensor_floor=1e-12):
    """Gate of one shared-mode chain.  gpu_sel[s][split], gpu_c[s][split]:
    kept indices and candidate counts; gpu_lnc[s]; gpu_fp[s]: fingerprints of
    the GPU's normalised tensor after step s (None: not compared).

    At every step until a flip: the kept sets equal the oracle's;
    |d ln c| <= max(lnc_floor, kappa_tau (base + delta_in)); the tensors
    (fingerprints) within max(tensor_floor, 3 kappa (base + delta_in)),
    where delta_in is the discrepancy the step inherits - the measured
    tensor distance after the previous step, or with no fingerprints the
    previous step's bound - and kappa, kappa_tau come from the oracle's
    spectrum of the step.  A step whose kept set differs must be a validated
    rounding-distance flip; the chain is compared no further.  Returns a
    GateResult; raises AssertionError on a violation."""
    from oracle.philox import selection_uniforms

    def u_of(s, p, m):
        return float(selection_uniforms(seed, orc.sid, 0, s, p, m + 1)[m])

    r = GateResult()
    dprev = 0.0
    wsum = 0.0
    for s, o in enumerate(orc.steps):
        same = all(list(gpu_sel[s][p]) == o.sel[p] and int(gpu_c[s][p]) == o.c[p] for p in (0, 1))
        if not same:
            for p in (0, 1):
                if list(gpu_sel[s][p]) != o.sel[p] or int(gpu_c[s][p]) != o.c[p]:
                    check_flip(o.sigma[p], o.c[p], o.sel[p], gpu_sel[s][p], gpu_c[s][p], k, tau,
                               2.0 * base + dprev, lambda m, s=s, p=p: u_of(s, p, m), r.notes,
                               f"step {s} split {p}")
            if any(list(gpu_sel[s][p]) != o.sel[p] for p in (0, 1)):
                r.stopped_at, r.reason = s, "flip"
                return r
        dl = abs(float(gpu_lnc[s]) - o.ln_c)
        tau_t = max(lnc_floor, o.kappa_t * (base + dprev))
        r.worst_tau = max(r.worst_tau, tau_t)
        r.worst_dlnc = max(r.worst_dlnc, dl)
        r.max_ratio = max(r.max_ratio, dl / tau_t)
        assert dl <= tau_t, (s, "ln c", dl, tau_t, o.kappa_t, dprev)
        r.checked += 1
        bound = max(tensor_floor, 3.0 * o.kappa * (base + dprev))
        if gpu_fp is not None and gpu_fp[s] is not None:
            d = float(np.sqrt(np.mean((np.asarray(gpu_fp[s]) - o.fp) ** 2)) / o.norm)
            r.max_ratio = max(r.max_ratio, d / bound)
            r.worst_delta = max(r.worst_delta, d)
            assert d <= bound, (s, "tensor", d, bound, o.kappa, dprev)
            r.tensor_checked += 1
            r.tight += bound <= 1e-4
            dprev = max(d, dl)
        else:
            dprev = min(1.0, max(bound, dl))
        wsum += 2.0 ** -(s + 1) * tau_t
    # ln|Z~| per site = sum_s 2^-(s+1) ln c_s + ln|Tr| / N: comparable while the
    # final tensors agree to 1e-6 (the trace then moves by about as much)
    n = len(orc.steps)
    if dprev <= 1e-6:
        r.lnZ_tol = max(1e-12, wsum + 10.0 * dprev / 2.0 ** n)
    return r


def compare_independent(orc, gpu_levels, gpu_lnc, k, seed, sid, tau, base, floor=1e-12):
    """Gate of one independent-mode sample (the paper's estimator): orc is
    the oracle's ChainResult (per-position records), gpu_levels[s] the
    GPU's record rows (c, kept, sel[k]) of step s's positions, gpu_lnc[s]
    the sum of ln c over the step's new tensors.  Every position must keep
    the oracle's set (else the flip is validated and the comparison stops);
    the per-step sums agree within the conditioning bound (kappa_tau times
    the rounding level plus the bound inherited from the previous step)
    times the number of new tensors."""
    from oracle.philox import selection_uniforms
    r = GateResult()
    dprev = 0.0
    for s, recs in enumerate(orc.positions):
        g = np.asarray(gpu_levels[s])
        flipped = False
        for p, sp in enumerate(recs):
            gc, gk = int(g[p, 0]), int(g[p, 1])
            gsel = [int(x) for x in g[p, 2:2 + gk]]
            if gsel != [int(x) for x in sp.sel] or gc != int(sp.c):
                def u_of(m, p=p, split=sp.split):
                    return float(selection_uniforms(seed, sid, p, s, split, m + 1)[m])
                check_flip(sp.sigma, sp.c, sp.sel, gsel, gc, k, tau, 2.0 * base + dprev, u_of, r.notes,
                           f"step {s} position {p}")
                flipped = flipped or gsel != [int(x) for x in sp.sel]
        if flipped:
            r.stopped_at, r.reason = s, "flip"
            return r
        kap = max(kappa_tau(sp.sigma, sp.c, sp.sel) for sp in recs)
        bound = max(floor, kap * (base + dprev))
        n_new = 2 ** (len(orc.positions) - s - 1)      # new tensors of the level (also for a prefix step)
        dl = abs(float(gpu_lnc[s]) - orc.ln_c[s])
        tol = bound * n_new
        r.max_ratio = max(r.max_ratio, dl / tol)
        r.worst_dlnc = max(r.worst_dlnc, dl)
        assert dl <= tol, (s, dl, tol, kap, dprev)
        r.checked += 1
        dprev = min(1.0, bound)
    return r


def gpu_chain_trace(m, ts, n_samples, n_steps, k, picks, dtype="f64", seed=0, tau=1e-11, groups=None,
                    mode="shared", J=64, log=print):
    """Steps a GPU chain one step at a time through the C ABI and keeps, for
    the picked samples, what the gate compares: kept sets and candidate
    counts (MCTRG_RECORD), ln c per step, fingerprints of the normalised
    tensor after every step (mctrg_chain_tensor), ln|Z~| and its sign."""
    from workloads import projection_pairs
    ch = m.Chain(ts, n_samples, n_steps=n_steps, k=k, dtype=dtype, seed=seed, tau_null=tau, groups=groups,
                 record=True, mode=mode)
    fps = {i: [] for i in picks}
    for s in range(n_steps):
        ch.step(1)
        T = ch.tensor()
        D = T.shape[1]
        P, Q = projection_pairs(D, J)
        for i in picks:
            fps[i].append(fingerprint(T[i].cpu().numpy(), P, Q))
        del T
        if log and (s % 5 == 4 or s == n_steps - 1):
            log(f"  gpu step {s} done (D={D})")
    res = ch.finish(want_ln_c=True)
    rec = ch.record.cpu().numpy()
    lnc = res.ln_c.cpu().numpy()
    ln = res.ln_abs_Z.cpu().numpy()
    sg = res.sign.cpu().numpy()
    ch.close()
    out = {}
    for i in picks:
        sel, c = [], []
        for s in range(n_steps):
            row = rec[i, s]
            kA, kB = int(row[2]), int(row[3])
            sel.append([list(map(int, row[4:4 + kA])), list(map(int, row[4 + k:4 + k + kB]))])
            c.append([int(row[0]), int(row[1])])
        out[i] = dict(sel=sel, c=c, lnc=lnc[i], fp=fps[i], ln_abs_Z=float(ln[i]), sign=int(sg[i]))
    return out
