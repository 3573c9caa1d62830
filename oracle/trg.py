"""TRG coarse-graining with stochastic truncation (oracle).

Test infrastructure only (see the package docstring).

One step, following Section III of the paper (Levin-Nave TRG with every
SVD truncated as in Section II):
  unfold   each tensor T[l,u,r,d] is viewed as a matrix (Section II, the
           index grouping before Eq. exactSVD): A split (l,u)|(r,d),
           B split (u,r)|(d,l);
  SVD      full SVD of the unfolding (Eq. exactSVD), singular values in
           descending order;
  truncate keep a random subset drawn from p(e) and divide the kept values
           by their inclusion rates (``esp.truncate``);
  factor   F = U_sel sqrt(S/r), G = sqrt(S/r) V_sel^T (the reweighted values
           are split symmetrically between the two halves);
  contract the four halves around a plaquette give the coarse tensor
           T'[a,b,c,e] = sum_{p,q,s,t} G_A[a,p,t] G_B[b,q,p] F_A[s,q,c] F_B[t,s,e];
  normalise T' = c * T_hat with c = max |T'|, ln c accumulated in FP64.
After the last step the single remaining tensor is traced over its
periodic legs, Tr = sum_{a,b} T_hat[a,b,a,b] (the explicit final trace the
paper describes after Eq. infiniteSum).

Readings where the paper is silent (each is also listed in the design
notes): the TRG wiring above; the symmetric sqrt split of S/r; the
per-step max-abs normalisation; the sign gauge of singular vectors
(``decompose``); tau_null for "nonzero".

Modes:
  shared       one tensor per level per sample: all tensors of a level are
               the same random tensor (translation-invariant chain);
  independent  every tensor of every level on an L x L torus gets its own
               independent truncation (the paper's estimator);
  topk         deterministic TRG, keeping the k largest values (Eq. approxSVD);
  exact        no truncation (only the numerically zero values dropped).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import esp, lattice
from .philox import selection_uniforms

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def unfold(T: np.ndarray, split: int):
    """Matrix view of T for a split; returns (M, row_shape, col_shape)."""
    Dl, Du, Dr, Dd = T.shape
    if split == 0:
        return T.reshape(Dl * Du, Dr * Dd), (Dl, Du), (Dr, Dd)
    Tp = T.transpose(1, 2, 3, 0)   # (u, r, d, l)
    return Tp.reshape(Du * Dr, Dd * Dl), (Du, Dr), (Dd, Dl)


def gauge_weights(col_shape) -> np.ndarray:
    """Fixed generic weights g(i1, i2) = 1 / (1 + i1 + phi * i2) over the
    column multi-index of an unfolding (phi = golden ratio).  A singular
    pair is signed so that sum_j v_j g_j > 0.  The weights depend on the
    leg indices, not on the flattened position, so padding a leg with zeros
    does not change the gauge."""
    i1, i2 = np.meshgrid(np.arange(col_shape[0]), np.arange(col_shape[1]), indexing="ij")
    return (1.0 / (1.0 + i1 + GOLDEN * i2)).reshape(-1)


def decompose(M: np.ndarray, col_shape):
    """FP64 SVD (LAPACK via numpy) with the sign gauge of ``gauge_weights``."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    g = Vt @ gauge_weights(col_shape)
    flip = g < 0
    U[:, flip] *= -1.0
    Vt[flip, :] *= -1.0
    return U, s, Vt


def qr_basis(M: np.ndarray, n_qr: int):
    """An orthonormal basis V from n_qr steps of QR iteration: M P = Q1 R1
    with column pivoting (LAPACK geqp3 via scipy), then R_i^T = Q_{i+1}
    R_{i+1}; V = P Q2 Q4 ... (the even-numbered Q factors).  Each pair of
    steps is one unshifted QR iteration on M^T M, so V tends to the right
    singular vectors; for any n_qr it is orthonormal."""
    import scipy.linalg as sla
    n = M.shape[1]
    _, R, piv = sla.qr(M, pivoting=True, mode="economic")
    V = np.eye(n)[:, piv]                     # P
    for step in range(2, n_qr + 1):
        Q, R = np.linalg.qr(R.T)
        if step % 2 == 0:
            V = V @ Q
    return V


def decompose_qr(M: np.ndarray, col_shape, n_qr: int):
    """The cheaper decomposition: M = sum_j (M v_j) v_j^T for the
    orthonormal basis V of ``qr_basis``, written like an SVD - s_j = |M v_j|
    (descending), U[:, j] = M v_j / s_j (unit, not orthogonal), Vt = V^T -
    so that the same truncation keeps a random subset of the terms and
    divides each by its inclusion rate.  Section II's argument (the
    average of the kept terms over p(e) is the full sum whenever every
    inclusion rate is positive) needs only the exact expansion, not the
    orthogonality of the U columns: the estimator stays unbiased and only
    its variance depends on the basis."""
    V = qr_basis(M, n_qr)
    A = M @ V
    s = np.linalg.norm(A, axis=0)
    order = np.argsort(-s, kind="stable")
    s, A, V = s[order], A[:, order], V[:, order]
    U = np.divide(A, s, out=np.zeros_like(A), where=s > 0)
    Vt = V.T.copy()
    g = Vt @ gauge_weights(col_shape)
    flip = g < 0
    U[:, flip] *= -1.0
    Vt[flip, :] *= -1.0
    return U, s, Vt


def factors(U, Vt, tr: esp.Truncation, row_shape, col_shape):
    w = tr.weights
    kk = len(tr.sel)
    F = (U[:, tr.sel] * w[None, :]).reshape(row_shape[0], row_shape[1], kk)
    G = (w[:, None] * Vt[tr.sel, :]).reshape(kk, col_shape[0], col_shape[1])
    return F, G


def contract(GA, GB, FA, FB) -> np.ndarray:
    """T'[a,b,c,e] = sum_{p,q,s,t} G_A[a,p,t] G_B[b,q,p] F_A[s,q,c] F_B[t,s,e]."""
    return np.einsum("apt,bqp,sqc,tse->abce", GA, GB, FA, FB, optimize=True)


def trace(T: np.ndarray) -> float:
    """Final trace over periodic legs: sum_{a,b} T[a,b,a,b]."""
    return float(np.einsum("abab->", T))


@dataclass
class SplitRecord:
    sigma: np.ndarray
    c: int
    sel: np.ndarray
    log_r: np.ndarray
    split: int = 0


@dataclass
class StepRecord:
    splits: List[SplitRecord]
    ln_c: float
    T_hat: Optional[np.ndarray] = None


@dataclass
class ChainResult:
    sign: int
    ln_abs_Z: float
    ln_c: List[float]
    records: List[StepRecord] = field(default_factory=list)
    positions: List[List[SplitRecord]] = field(default_factory=list)   # independent mode: per step, per position


def _split_mode(mode: str) -> str:
    return {"shared": "stochastic", "independent": "stochastic", "topk": "topk", "exact": "exact"}[mode]


def decompose_and_truncate(T, split, k, mode, seed, sample_id, position, step, tau_null,
                           chooser=None, basis="svd"):
    """Unfold, decompose, truncate and factor one tensor.  ``chooser``, if
    given, is called as chooser(position, step, split, sigma, c) and returns
    the kept subset instead of a random draw (None: draw as usual).
    ``basis``: "svd" (Section II's exact SVD) or "qr3" / "qr5" (the
    QR-iteration basis of ``decompose_qr``)."""
    M, rs, cs = unfold(T, split)
    if basis == "svd":
        U, s, Vt = decompose(M, cs)
    else:
        U, s, Vt = decompose_qr(M, cs, {"qr3": 3, "qr5": 5}[basis])
    forced = None
    if chooser is not None:
        forced = chooser(position, step, split, s, esp.n_candidates(s, tau_null))
    tr = esp.truncate(s, k, _split_mode(mode),
                      lambda c: selection_uniforms(seed, sample_id, position, step, split, c),
                      tau_null, forced_sel=forced)
    F, G = factors(U, Vt, tr, rs, cs)
    return F, G, SplitRecord(s, tr.c, tr.sel, tr.log_r, split)


def run_shared(T0: np.ndarray, n_steps: int, k: int, seed: int, sample_id: int,
               mode: str = "shared", tau_null: float = 1e-11, keep_tensors: bool = False,
               chooser=None, n_det: int = 0, basis: str = "svd") -> ChainResult:
    """One sample of the translation-invariant chain on 2**n_steps sites.
    The first ``n_det`` steps keep the largest values deterministically
    (top-k), the later ones use ``mode``.

    ln|Z~| = sum_s (N / 2^(s+1)) ln c_s + ln|Tr T_hat_final|, N = 2**n_steps."""
    T = np.array(T0, dtype=np.float64)
    ln_c: List[float] = []
    recs: List[StepRecord] = []
    for step in range(n_steps):
        md = "topk" if step < n_det else mode
        FA, GA, ra = decompose_and_truncate(T, 0, k, md, seed, sample_id, 0, step, tau_null, chooser, basis)
        FB, GB, rb = decompose_and_truncate(T, 1, k, md, seed, sample_id, 0, step, tau_null, chooser, basis)
        Tn = contract(GA, GB, FA, FB)
        c = float(np.max(np.abs(Tn))) if Tn.size else 0.0
        if not (c > 0.0 and math.isfinite(c)):
            return ChainResult(0, math.nan, ln_c, recs)
        T = Tn / c
        ln_c.append(math.log(c))
        recs.append(StepRecord([ra, rb], math.log(c), T.copy() if keep_tensors else None))
    tr = trace(T)
    N = 2.0 ** n_steps
    ln_abs = sum((N / 2.0 ** (s + 1)) * lc for s, lc in enumerate(ln_c))
    if tr == 0.0:
        return ChainResult(0, -math.inf, ln_c, recs)
    return ChainResult(1 if tr > 0 else -1, ln_abs + math.log(abs(tr)), ln_c, recs)


def step_independent(tensors, lev, k, mode, seed, sample_id, step, tau_null=1e-11, chooser=None, records=None,
                     basis="svd"):
    """One independent-mode TRG step over a whole lattice level.

    Returns (new_tensors, next_level, sum of ln c over the new positions),
    or None if a coarse tensor is zero or not finite.  ``records``, if a
    list, receives the step's SplitRecord of every position."""
    plaq, nxt = lattice.coarsen(lev)
    F, G = [None] * lev.n, [None] * lev.n
    recs = [None] * lev.n
    for p in range(lev.n):
        split = 0 if lev.is_a[p] else 1
        F[p], G[p], recs[p] = decompose_and_truncate(tensors[p], split, k, mode, seed, sample_id, p, step,
                                                     tau_null, chooser, basis)
    new = []
    step_sum = 0.0
    for P, (p0, q0, p1, q1) in enumerate(plaq):
        Tn = contract(G[p0], G[q0], F[p1], F[q1])
        c = float(np.max(np.abs(Tn))) if Tn.size else 0.0
        if not (c > 0.0 and math.isfinite(c)):
            return None
        new.append(Tn / c)
        step_sum += math.log(c)
    if records is not None:
        records.append(recs)
    return new, nxt, step_sum


def run_independent(T0: np.ndarray, n_steps: int, k: int, seed: int, sample_id: int,
                    mode: str = "independent", tau_null: float = 1e-11, chooser=None,
                    n_det: int = 0, basis: str = "svd") -> ChainResult:
    """One sample of the paper's estimator on an L x L torus, L = 2**(n_steps/2):
    every tensor of every level gets its own independent truncation.
    ``T0`` is one tensor for every site or an array of per-site tensors.

    ``n_det`` > 0 (one tensor for every site): the Discussion's deterministic
    coarse-graining steps before Monte Carlo.  The first n_det steps
    coarse-grain the one tensor with top-k truncation (every tensor of those
    levels is the same); its result starts every position of level n_det,
    from where each tensor is truncated independently.  A prefix step adds
    (number of new tensors) * ln c; its record holds the A and B split.

    ln|Z~| = sum over levels and positions of ln c + ln|Tr T_hat_final|."""
    if n_steps % 2:
        raise ValueError("independent mode needs an even number of steps (L x L torus)")
    L = 2 ** (n_steps // 2)
    lev = lattice.square_torus(L)
    T0 = np.asarray(T0, dtype=np.float64)
    if T0.ndim == 5:      # one tensor per site, site id x + L*y
        if T0.shape[0] != lev.n or n_det:
            raise ValueError("need one tensor per site (and no deterministic prefix)")
        tensors = [T0[i].copy() for i in range(lev.n)]
    else:
        tensors = [T0.copy() for _ in range(lev.n)]
    total = 0.0
    ln_c_steps: List[float] = []
    positions: List[List[SplitRecord]] = []
    if n_det:
        pre = run_shared(T0, n_det, k, seed, sample_id, mode="topk", tau_null=tau_null, keep_tensors=True,
                         basis=basis)
        if pre.sign == 0 and len(pre.ln_c) < n_det:
            return ChainResult(0, math.nan, pre.ln_c, positions=positions)
        for step in range(n_det):
            lev = lattice.coarsen(lev)[1]
            n_new = lev.n
            total += n_new * pre.ln_c[step]
            ln_c_steps.append(n_new * pre.ln_c[step])
            positions.append(list(pre.records[step].splits))
        tensors = [pre.records[-1].T_hat.copy() for _ in range(lev.n)]
    for step in range(n_det, n_steps):
        out = step_independent(tensors, lev, k, mode, seed, sample_id, step, tau_null, chooser, positions, basis)
        if out is None:
            return ChainResult(0, math.nan, ln_c_steps, positions=positions)
        tensors, lev, step_sum = out
        total += step_sum
        ln_c_steps.append(step_sum)
    tr = trace(tensors[0])
    if tr == 0.0:
        return ChainResult(0, -math.inf, ln_c_steps, positions=positions)
    return ChainResult(1 if tr > 0 else -1, total + math.log(abs(tr)), ln_c_steps, positions=positions)


def run(T0, n_steps, k, seed, sample_id, mode="shared", tau_null=1e-11, keep_tensors=False) -> ChainResult:
    if mode == "independent":
        return run_independent(T0, n_steps, k, seed, sample_id, mode, tau_null)
    return run_shared(T0, n_steps, k, seed, sample_id, mode, tau_null, keep_tensors)
