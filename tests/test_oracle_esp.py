"""Pins of the oracle's subset sampler and inclusion rates (Section II).

Inclusion rates and subset probabilities are checked against exact
rational arithmetic over every subset (Python fractions), against closed
forms (k = 1 and k = c - 1), and the sequential draw is checked against
the exact p(e) by a chi-square test on Philox-driven draws."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import esp
from oracle.philox import selection_uniforms


def exact_rates(lams, k):
    """p(e) and r_i by enumerating all size-k subsets with rationals."""
    subsets = list(itertools.combinations(range(len(lams)), k))
    w = [math.prod((lams[i] for i in e), start=Fraction(1)) for e in subsets]
    tot = sum(w)
    p = {e: wi / tot for e, wi in zip(subsets, w)}
    r = [sum(pe for e, pe in p.items() if i in e) for i in range(len(lams))]
    return p, r


SIGMAS = [
    [Fraction(1), Fraction(7, 8), Fraction(3, 4), Fraction(1, 2), Fraction(1, 3), Fraction(1, 10)],
    [Fraction(1), Fraction(1), Fraction(9, 10), Fraction(1, 100), Fraction(1, 1000), Fraction(1, 1000),
     Fraction(1, 10**5), Fraction(3, 10**6), Fraction(1, 10**7), Fraction(1, 10**9)],
]


@pytest.mark.parametrize("sig", SIGMAS)
@pytest.mark.parametrize("kfrac", [0.2, 0.5, 0.8])
def test_inclusion_rates_exact_enumeration(sig, kfrac):
    c = len(sig)
    k = max(1, min(c - 1, int(round(kfrac * c))))
    lams = [(s / sig[0]) ** 2 for s in sig]
    _, r = exact_rates(lams, k)
    sigma = np.array([float(s) for s in sig])
    ll = esp.log_lambdas(sigma, c)
    got = np.exp(esp.log_inclusion_rates(ll, k))
    want = np.array([float(x) for x in r])
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    assert got.sum() == pytest.approx(k, rel=1e-13)


def test_closed_forms():
    rng = np.random.default_rng(3)
    sigma = np.sort(rng.uniform(0.01, 1.0, 9))[::-1]
    c = sigma.size
    lam = (sigma / sigma[0]) ** 2
    ll = esp.log_lambdas(sigma, c)
    r1 = np.exp(esp.log_inclusion_rates(ll, 1))
    assert np.allclose(r1, lam / lam.sum(), rtol=1e-13)
    rc1 = np.exp(esp.log_inclusion_rates(ll, c - 1))
    assert np.allclose(rc1, 1.0 - (1.0 / lam) / np.sum(1.0 / lam), rtol=1e-12)
    tr = esp.truncate(sigma, c, "stochastic", None)
    assert np.array_equal(tr.sel, np.arange(c)) and np.all(tr.log_r == 0)


def test_rates_wide_dynamic_range():
    # 1024 candidates spanning 22 decades, k = 32: log-domain tables stay exact
    sigma = np.logspace(0, -11, 1024)
    ll = esp.log_lambdas(sigma, 1024)
    r = np.exp(esp.log_inclusion_rates(ll, 32))
    assert r.sum() == pytest.approx(32, rel=1e-11)
    assert np.all(r > 0) and np.all(r <= 1 + 1e-12)
    assert np.all(np.diff(r) <= 1e-15)        # monotone in lambda


def test_sequential_draw_follows_p():
    sig = SIGMAS[0]
    c, k = len(sig), 3
    lams = [(s / sig[0]) ** 2 for s in sig]
    p, _ = exact_rates(lams, k)
    sigma = np.array([float(s) for s in sig])
    ll = esp.log_lambdas(sigma, c)
    LS = esp.suffix_table(ll, k)
    n = 12000
    counts = {e: 0 for e in p}
    for s in range(n):
        sel = esp.select(ll, k, selection_uniforms(1, s, 0, 0, 0, c), LS)
        counts[tuple(int(i) for i in sel)] += 1
    obs = np.array([counts[e] for e in p], dtype=float)
    exp = np.array([float(p[e]) * n for e in p])
    assert stats.chisquare(obs, exp).pvalue > 1e-4


def test_reweighted_spectrum_is_unbiased():
    # Eq. Ssum: sum_e p(e) S^(e) = S, with S^(e)_ii = S_ii / r_i on e
    sig = SIGMAS[1]
    c, k = len(sig), 4
    lams = [(s / sig[0]) ** 2 for s in sig]
    p, _ = exact_rates(lams, k)
    sigma = np.array([float(s) for s in sig])
    ll = esp.log_lambdas(sigma, c)
    acc = np.zeros(c)
    for e, pe in p.items():
        tr = esp.truncate(sigma, k, "stochastic", None, forced_sel=np.array(e))
        acc[tr.sel] += float(pe) * tr.weights ** 2
    assert np.allclose(acc, sigma, rtol=1e-12, atol=0)


def test_candidates_threshold():
    sigma = np.array([2.0, 1.0, 3e-11, 2e-11, 1e-11, 0.0])   # cut at 1e-11 * s_1 = 2e-11
    assert esp.n_candidates(sigma, 1e-11) == 3
    assert esp.n_candidates(np.zeros(4), 1e-11) == 0
