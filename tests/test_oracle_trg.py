"""Pins of the oracle's TRG step, chains and lattice bookkeeping.

* With no truncation the chain must reproduce Z exactly: against
  brute-force Ising sums (site construction), the medial-lattice spin sum
  (plaquette construction, Section III Fig. 1), and a direct contraction
  of the torus network built from the bond definitions (generic tensors,
  distinct per site) - so a transposed leg or wrong plaquette wiring fails.
* Unbiasedness (Section III, Eqs. infiniteSum/infiniteEnsemble): summing
  p(path) * Z~(path) over every sampling path of the independent estimator
  gives Z exactly; the shared chain does not.
* Deterministic top-k TRG (Eq. approxSVD) at the C1 size is close to the
  exact Kaufman value; the independent estimator is statistically
  unbiased against Kaufman on a 4 x 4 torus.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import esp, ising, lattice, trg
from workloads import BETA_C, gaussian_tensor, positive_tensor


network_lnZ = lattice.network_Z


@pytest.mark.parametrize("L,n", [(2, 2), (4, 4)])
@pytest.mark.parametrize("beta,h", [(0.3, 0.0), (BETA_C, 0.0), (0.42, 0.1)])
def test_exact_chain_equals_brute_force(L, n, beta, h):
    T = ising.site_tensor(beta, h)
    bf = ising.brute_force_lnZ_torus(L, beta, h)
    assert trg.run(T, n, 10**6, 0, 0, mode="exact").ln_abs_Z == pytest.approx(bf, abs=1e-12)
    assert trg.run_independent(T, n, 10**6, 0, 0, mode="exact").ln_abs_Z == pytest.approx(bf, abs=1e-12)


@pytest.mark.parametrize("beta,h", [(0.3, 0.0), (0.5, 0.2)])
def test_plaquette_construction_is_medial_ising(beta, h):
    A = ising.plaquette_tensor(beta, h)
    bf = ising.brute_force_lnZ_medial(2, beta, h)
    assert trg.run(A, 2, 10**6, 0, 0, mode="exact").ln_abs_Z == pytest.approx(bf, abs=1e-12)


def test_direct_network_matches_brute_force():
    # the network helper itself, against the Ising sum
    T = ising.site_tensor(0.4, 0.15)
    for L in (2, 4):
        assert math.log(network_lnZ([T] * (L * L), L)) == pytest.approx(
            ising.brute_force_lnZ_torus(L, 0.4, 0.15), abs=1e-12)


@pytest.mark.parametrize("L,n", [(2, 2), (4, 4)])
def test_generic_tensors_exact_chain(L, n):
    T = positive_tensor(2, seed=11)
    Z = network_lnZ([T] * (L * L), L)
    assert trg.run(T, n, 10**6, 0, 0, mode="exact").ln_abs_Z == pytest.approx(math.log(Z), abs=1e-11)
    # distinct tensor on every site: pins the independent-mode bookkeeping
    Ts = np.stack([positive_tensor(2, seed=100 + i) for i in range(L * L)])
    Zs = network_lnZ(list(Ts), L)
    r = trg.run_independent(Ts, n, 10**6, 0, 0, mode="exact")
    assert r.sign == 1 and r.ln_abs_Z == pytest.approx(math.log(Zs), abs=1e-11)


def test_generic_signed_tensor_exact_chain():
    L = 2
    Ts = np.stack([gaussian_tensor(2, seed=200 + i) for i in range(4)])
    Z = network_lnZ(list(Ts), L)
    r = trg.run_independent(Ts, 2, 10**6, 0, 0, mode="exact")
    assert r.sign == (1 if Z > 0 else -1)
    assert r.ln_abs_Z == pytest.approx(math.log(abs(Z)), abs=1e-11)


def test_lattice_levels_16x16():
    lev = lattice.square_torus(16)
    sizes = []
    while lev.n > 1:
        plaq, lev = lattice.coarsen(lev)
        sizes.append(lev.n)
        # every old site is used exactly twice (once as G, once as F)
        used = np.bincount(plaq.reshape(-1), minlength=2 * lev.n)
        assert np.all(used == 2)
    assert sizes == [128, 64, 32, 16, 8, 4, 2, 1]
    assert np.all(lev.nbr == 0)


def _subsets_with_p(sigma, k, tau):
    c = esp.n_candidates(sigma, tau)
    if c <= k:
        return [(None, 1.0)]
    lam = (sigma[:c] / sigma[0]) ** 2
    subs = list(itertools.combinations(range(c), k))
    w = np.array([np.prod(lam[list(e)]) for e in subs])
    return list(zip(subs, w / w.sum()))


def _expected_Z_independent(T0s, k, tau=1e-11, basis="svd"):
    """sum over every path of p(path) * Z~(path) for a 2 x 2 torus."""
    lev0 = lattice.square_torus(2)
    tensors0 = [T0s[i] for i in range(4)]
    total = 0.0

    def options(tensors, lev):
        opts = []
        for p in range(lev.n):
            M, _, cs = trg.unfold(tensors[p], 0 if lev.is_a[p] else 1)
            if basis == "svd":
                s = np.linalg.svd(M, compute_uv=False)
            else:
                s = trg.decompose_qr(M, cs, {"qr3": 3, "qr5": 5}[basis])[1]
            opts.append(_subsets_with_p(s, k, tau))
        return opts

    opts0 = options(tensors0, lev0)
    for path0 in itertools.product(*opts0):
        p0 = math.prod(pe for _, pe in path0)
        ch0 = lambda pos, step, split, s, c, path=path0: path[pos][0]
        out = trg.step_independent(tensors0, lev0, k, "independent", 0, 0, 0, tau, ch0, basis=basis)
        t1, lev1, sum1 = out
        opts1 = options(t1, lev1)
        for path1 in itertools.product(*opts1):
            p1 = math.prod(pe for _, pe in path1)
            ch1 = lambda pos, step, split, s, c, path=path1: path[pos][0]
            t2, lev2, sum2 = trg.step_independent(t1, lev1, k, "independent", 0, 0, 1, tau, ch1, basis=basis)
            total += p0 * p1 * math.exp(sum1 + sum2) * trg.trace(t2[0])
    return total


def test_independent_estimator_is_exactly_unbiased():
    # generic distinct tensors, k = 2 < rank 4: every decomposition is random
    Ts = np.stack([positive_tensor(2, seed=300 + i) for i in range(4)])
    Z = network_lnZ(list(Ts), 2)
    EZ = _expected_Z_independent(Ts, 2)
    assert EZ == pytest.approx(Z, rel=1e-12)


def test_shared_chain_is_biased():
    T = positive_tensor(2, seed=301)
    Z = network_lnZ([T] * 4, 2)
    M0 = [trg.unfold(T, s)[0] for s in (0, 1)]
    opts = [_subsets_with_p(np.linalg.svd(M, compute_uv=False), 2, 1e-11) for M in M0]
    EZ = 0.0
    for (eA, pA), (eB, pB) in itertools.product(*opts):
        step0 = {0: eA, 1: eB}
        # level-1 options depend on the level-0 choice
        def ch0(pos, step, split, s, c):
            return step0[split]
        r1 = trg.run_shared(T, 1, 2, 0, 0, chooser=ch0, keep_tensors=True)
        T1 = r1.records[0].T_hat
        opts1 = [_subsets_with_p(np.linalg.svd(trg.unfold(T1, s)[0], compute_uv=False), 2, 1e-11) for s in (0, 1)]
        for (fA, qA), (fB, qB) in itertools.product(*opts1):
            seq = {(0, 0): eA, (0, 1): eB, (1, 0): fA, (1, 1): fB}
            r = trg.run_shared(T, 2, 2, 0, 0, chooser=lambda pos, step, split, s, c: seq[(step, split)])
            EZ += pA * pB * qA * qB * r.sign * math.exp(r.ln_abs_Z)
    assert abs(EZ / Z - 1.0) > 1e-6


def test_topk_trg_close_to_kaufman():
    r = trg.run(ising.site_tensor(BETA_C), 8, 8, 0, 0, mode="topk")
    exact = ising.kaufman_lnZ_torus(16, BETA_C)
    assert abs(r.ln_abs_Z - exact) / 256 < 1e-4
    # rank schedule of the Ising chain: 2, 4, 4, 16 ... then capped at k
    assert [int(x.splits[0].c) for x in r.records[:4]] == [2, 4, 4, 16]


def test_independent_estimator_statistically_unbiased():
    beta = BETA_C
    T = ising.site_tensor(beta)
    Z = math.exp(ising.kaufman_lnZ_torus(4, beta))
    vals = []
    for s in range(300):
        r = trg.run_independent(T, 4, 2, 0, s)
        vals.append(r.sign * math.exp(r.ln_abs_Z))
    vals = np.array(vals)
    mean, se = vals.mean(), vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(mean - Z) < 4 * se
    assert se / Z < 0.05          # the test has power


def test_chain_reproducible_by_sample_id():
    T = ising.site_tensor(0.4, 0.05)
    a = trg.run(T, 6, 4, 7, 123)
    b = trg.run(T, 6, 4, 7, 123)
    c = trg.run(T, 6, 4, 7, 124)
    assert a.ln_abs_Z == b.ln_abs_Z and a.ln_c == b.ln_c
    assert a.ln_abs_Z != c.ln_abs_Z
