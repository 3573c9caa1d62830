"""Deterministic coarse-graining steps before Monte Carlo (Section V,
Discussion): the first n_det steps coarse-grain one tensor with top-k
truncation (the system is translation invariant, so every tensor of those
levels is the same), the rest run the paper's independent estimator on the
coarse lattice.

Pins: while the prefix keeps every candidate (c <= k; the 2-D Ising chain
has ranks 2, 4, 4 at its first three steps), the independent estimator
itself makes those steps exact and equal at every position, and draws the
later ones with the same (sample, position, step, split) counters - so each
sample must equal the pure independent sample.  With k at least the rank
everywhere, an all-deterministic chain is exact (brute force)."""
import pytest

from oracle import ising, trg
from workloads import BETA_C


@pytest.mark.parametrize("sid", [0, 1, 2])
def test_exact_prefix_equals_independent_sample(sid):
    T = ising.site_tensor(BETA_C)
    a = trg.run_independent(T, 6, 8, 0, sid)
    b = trg.run_independent(T, 6, 8, 0, sid, n_det=3)
    # the prefix steps keep every candidate
    assert all(sp.c <= 8 and len(sp.sel) == sp.c for rec in b.positions[:3] for sp in rec)
    assert b.sign == a.sign
    assert abs(b.ln_abs_Z - a.ln_abs_Z) < 1e-10
    for s in range(6):
        assert b.ln_c[s] == pytest.approx(a.ln_c[s], rel=1e-12, abs=1e-12)


def test_prefix_then_monte_carlo_uses_the_coarse_lattice():
    # 4 x 4 torus, two deterministic steps, then two independent ones: the
    # independent levels have 4 and 2 positions
    T = ising.site_tensor(0.42, 0.1)
    r = trg.run_independent(T, 4, 3, 5, 9, n_det=2)
    assert [len(x) for x in r.positions] == [2, 2, 4, 2]


def test_all_deterministic_exact_chain_is_exact():
    beta, h = 0.42, 0.1
    T = ising.site_tensor(beta, h)
    r = trg.run_independent(T, 4, 64, 0, 0, n_det=4)
    assert r.ln_abs_Z == pytest.approx(ising.brute_force_lnZ_torus(4, beta, h), abs=1e-11)
