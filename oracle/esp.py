"""Stochastic truncation of a singular-value spectrum (oracle).

Test infrastructure only (see the package docstring).

Section II: an ensemble element e is a subset of chi-tilde (here ``k``) of
the nonzero singular values; e is drawn with probability
p(e) = w(e) / sum_n w(n), w(e) = prod_{j in e} s_j^2, and every kept value
is divided by its inclusion rate r(S_ii) = sum_{e containing i} p(e), so
that the average of S^(e) is S (Eq. Ssum).

The paper defers the sampling algorithm to Ferris (2015) and only states
its O(chi * chi-tilde) cost.  This oracle draws e exactly from p(e) with
the elementary-symmetric-polynomial (ESP) sequential method: with
lambda_i = (s_i / s_1)^2 over the candidates in descending order, and
E_j(m) = e_j(lambda_m, ..., lambda_{c-1}) the j-th elementary symmetric
polynomial of the suffix starting at m, candidate m is kept with
probability  lambda_m * E_{rem-1}(m+1) / E_rem(m)  given that ``rem``
values remain to be chosen; this telescopes to p(e).  The inclusion rate is
r_i = lambda_i * e_{k-1}(lambda without i) / e_k(lambda) with
e_{k-1}(lambda without i) = sum_a e_a(prefix before i) e_{k-1-a}(suffix
after i).  Everything is evaluated in the log domain because products of
up to k squared ratios underflow FP64.

Readings where the paper is silent:
* "nonzero" singular values are those with s_i > tau_null * s_1
  (tau_null = 1e-11 by default);
* when at most k candidates exist they are all kept with r = 1;
* top-k (deterministic TRG, Eq. approxSVD) keeps the first min(k, c)
  candidates with r = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NEG_INF = -math.inf


def n_candidates(sigma: np.ndarray, tau_null: float) -> int:
    """Number of singular values (descending) above tau_null * s_1."""
    if sigma.size == 0 or not (sigma[0] > 0.0):
        return 0
    return int(np.count_nonzero(sigma > tau_null * sigma[0]))


def log_lambdas(sigma: np.ndarray, c: int) -> np.ndarray:
    """ln lambda_i = 2 ln(s_i / s_1) for the c candidates."""
    return 2.0 * np.log(sigma[:c] / sigma[0])


def suffix_table(loglam: np.ndarray, kmax: int) -> np.ndarray:
    """LS[j, m] = ln e_j(lambda_m, ..., lambda_{c-1}) for j = 0..kmax,
    m = 0..c (m = c is the empty suffix).  Recurrence over m downwards:
    e_j(m) = e_j(m+1) + lambda_m e_{j-1}(m+1)."""
    c = loglam.size
    LS = np.full((kmax + 1, c + 1), NEG_INF)
    LS[0, :] = 0.0
    for m in range(c - 1, -1, -1):
        LS[1:, m] = np.logaddexp(LS[1:, m + 1], loglam[m] + LS[:-1, m + 1])
    return LS


def prefix_table(loglam: np.ndarray, kmax: int) -> np.ndarray:
    """LP[j, m] = ln e_j(lambda_0, ..., lambda_{m-1}) for m = 0..c."""
    c = loglam.size
    LP = np.full((kmax + 1, c + 1), NEG_INF)
    LP[0, :] = 0.0
    for m in range(c):
        LP[1:, m + 1] = np.logaddexp(LP[1:, m], loglam[m] + LP[:-1, m])
    return LP


def select(loglam: np.ndarray, k: int, uniforms: np.ndarray, LS: np.ndarray | None = None) -> np.ndarray:
    """Indices (ascending) of the kept subset, drawn from p(e) with one
    uniform per candidate index.  Requires c > k."""
    c = loglam.size
    assert c > k
    if LS is None:
        LS = suffix_table(loglam, k)
    sel = []
    rem = k
    for m in range(c):
        if rem == 0:
            break
        if rem == c - m:           # every remaining candidate must be kept
            take = True
        else:
            q = math.exp(loglam[m] + LS[rem - 1, m + 1] - LS[rem, m])
            take = uniforms[m] < q
        if take:
            sel.append(m)
            rem -= 1
    return np.array(sel, dtype=np.int64)


def log_inclusion_rates(loglam: np.ndarray, k: int, idx: np.ndarray | None = None,
                        LS: np.ndarray | None = None, LP: np.ndarray | None = None) -> np.ndarray:
    """ln r_i for the candidates in ``idx`` (default: all c)."""
    c = loglam.size
    if LS is None:
        LS = suffix_table(loglam, k)
    if LP is None:
        LP = prefix_table(loglam, k)
    if idx is None:
        idx = np.arange(c)
    out = np.empty(len(idx))
    a = np.arange(k)
    for n, i in enumerate(idx):
        terms = LP[a, i] + LS[k - 1 - a, i + 1]
        mx = np.max(terms)
        s = mx + math.log(np.sum(np.exp(terms - mx))) if mx > NEG_INF else NEG_INF
        out[n] = loglam[i] + s - LS[k, 0]
    return out


@dataclass
class Truncation:
    """Result of truncating one spectrum: kept indices (ascending, i.e.
    descending singular value), their inclusion rates and the factor
    weights sqrt(s_i / r_i)."""
    c: int
    sel: np.ndarray
    log_r: np.ndarray
    weights: np.ndarray


def truncate(sigma: np.ndarray, k: int, mode: str, uniforms_fn, tau_null: float = 1e-11,
             forced_sel: np.ndarray | None = None) -> Truncation:
    """Choose the kept singular values of one decomposition.

    mode "stochastic": exact draw from p(e) (Section II) when more than k
    candidates exist; mode "topk": the first min(k, c) (Eq. approxSVD);
    mode "exact": every candidate (no truncation).  ``uniforms_fn(c)``
    returns the c uniforms for this decomposition (called only when a
    random choice is made).  ``forced_sel`` replaces the random draw by a
    given subset (used to enumerate every outcome in tests)."""
    c = n_candidates(sigma, tau_null)
    if mode == "exact" or c <= k:
        sel = np.arange(c)
        log_r = np.zeros(c)
    elif mode == "topk":
        sel = np.arange(k)
        log_r = np.zeros(k)
    elif mode == "stochastic":
        ll = log_lambdas(sigma, c)
        LS = suffix_table(ll, k)
        if forced_sel is None:
            sel = select(ll, k, uniforms_fn(c), LS)
        else:
            sel = np.sort(np.asarray(forced_sel, dtype=np.int64))
        log_r = log_inclusion_rates(ll, k, sel, LS=LS)
    else:
        raise ValueError(mode)
    w = np.sqrt(sigma[sel] * np.exp(-log_r))
    return Truncation(c, sel, log_r, w)
