"""Seeded synthetic workloads for Monte Carlo TRG on the 2-D Ising model.

This module only produces *inputs*: temperatures, fields, kept counts, sample
ids, their assignment to samples, and generic random starting tensors for
tests.  It contains none of the method's arithmetic (no tensors built from
Boltzmann weights, no decompositions, no random draws of the method itself),
so both the CPU oracle and the HIP path may use it.

The workloads follow the paper's benchmark, the zero-field 2-D Ising model on
a periodic square lattice (Section IV, Eq. ising_model), scaled to the sizes
of the measured configurations below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Critical coupling of the square-lattice Ising model, beta_c = ln(1+sqrt 2)/2.
BETA_C = 0.5 * math.log(1.0 + math.sqrt(2.0))


@dataclass(frozen=True)
class Workload:
    """One measured configuration.

    ``k`` is the kept count per decomposition (the paper's chi-tilde, which is
    also the new bond dimension).  ``n_steps`` coarse-graining steps contract a
    lattice of ``2**n_steps`` site tensors down to one tensor.
    """

    name: str
    mode: str                    # "shared" | "independent" | "topk"
    n_steps: int
    ks: Tuple[int, ...]
    betas: Tuple[float, ...]
    hs: Tuple[float, ...]
    n_samples: int               # total samples over all (k, beta, h) groups
    contract_dtypes: Tuple[str, ...] = ("f64",)
    seed: int = 0
    model: str = "vertex"

    @property
    def n_sites(self) -> float:
        return float(2 ** self.n_steps)

    def groups(self) -> List[Tuple[int, float, float]]:
        """Balanced factorial list of (k, beta, h) groups."""
        return [(k, b, h) for k in self.ks for b in self.betas for h in self.hs]


def linspace_inclusive(lo: float, hi: float, n: int) -> Tuple[float, ...]:
    return tuple(float(x) for x in np.linspace(lo, hi, n))


# Configurations: a 16x16 torus at beta_c with k=8 (exact Z known), a beta
# sweep at k=16 on 2^20 sites, the mixed-k batched form on 2^30 sites, a
# precision study at k=48 and a large-k form at k=64.
C1 = Workload("ising16x16_k8_betac", "independent", 8, (8,), (BETA_C,), (0.0,), 1000)
C1_SHARED = Workload("ising16x16_k8_betac_shared", "shared", 8, (8,), (BETA_C,), (0.0,), 1000)
C2 = Workload("ising2p20_k16_beta_sweep", "shared", 20, (16,),
              linspace_inclusive(0.30, 0.60, 16), (0.0,), 160000)
C3 = Workload("ising2p30_mixed_k16_24_32", "shared", 30, (16, 24, 32),
              linspace_inclusive(0.35, 0.55, 32), (0.0, 0.05), 65536,
              contract_dtypes=("f32",))
C3H = Workload("ising2p30_k32_betac", "shared", 30, (32,), (BETA_C,), (0.0,), 8192,
               contract_dtypes=("f32",))
C4 = Workload("ising2p24_k48_betac", "shared", 24, (48,), (BETA_C,), (0.0,), 8192,
              contract_dtypes=("bf16", "f32", "f64"))
C5 = Workload("ising2p20_k64_b042_h01", "shared", 20, (64,), (0.42,), (0.1,), 256,
              contract_dtypes=("fp8", "bf16", "f64"))

ALL = (C1, C1_SHARED, C2, C3, C3H, C4, C5)


def assign_groups(w: Workload, n_samples: Optional[int] = None,
                  shuffle_seed: int = 12345) -> np.ndarray:
    """Per-sample group index into ``w.groups()``: a balanced assignment
    (sample i gets group i mod G) followed by a seeded permutation."""
    n = w.n_samples if n_samples is None else n_samples
    g = len(w.groups())
    idx = np.arange(n, dtype=np.int64) % g
    rng = np.random.default_rng(shuffle_seed)
    rng.shuffle(idx)
    return idx.astype(np.int32)


def gaussian_tensor(d: int, seed: int, shape: Optional[Sequence[int]] = None) -> np.ndarray:
    """A generic dense real tensor (standard normal entries, seeded).  Used as
    a starting tensor for exactness and unbiasedness tests, where generic
    (full-rank, non-degenerate) unfoldings are wanted."""
    rng = np.random.default_rng(seed)
    shp = tuple(shape) if shape is not None else (d, d, d, d)
    return rng.standard_normal(shp)


def positive_tensor(d: int, seed: int) -> np.ndarray:
    """A generic tensor with positive entries (so that Z > 0 for every
    lattice): exp of seeded normal entries scaled by 0.5."""
    rng = np.random.default_rng(seed)
    return np.exp(0.5 * rng.standard_normal((d, d, d, d)))


def sample_ids(offset: int, n: int) -> np.ndarray:
    return np.arange(offset, offset + n, dtype=np.int64)


def projection_pairs(D: int, J: int = 64, seed: int = 20171010):
    """J pairs of seeded standard-normal D x D matrices (P_j, Q_j) that the
    parity tests use to fingerprint a D^4 tensor: f_j = sum P_j[a,b]
    T[a,b,c,e] Q_j[c,e].  Inputs only: the same arrays serve both sides."""
    rng = np.random.default_rng([seed, D, J])
    P = rng.standard_normal((J, D * D))
    Q = rng.standard_normal((J, D * D))
    return P, Q
