"""Pins of the oracle's Ising tensors and exact partition functions.

Each exact route is checked against a different one: brute-force
enumeration, the row transfer matrix, Kaufman's closed form and Onsager's
integral, plus a value fixed by mathematics (Onsager at beta_c equals
ln2/2 + 2G/pi with G Catalan's constant, computed here from its own
integral definition).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import ising, trg
from workloads import BETA_C

BETAS = (0.3, BETA_C, 0.6)


@pytest.mark.parametrize("L", [2, 3, 4])
@pytest.mark.parametrize("beta,h", [(0.3, 0.0), (BETA_C, 0.0), (0.42, 0.1), (0.25, -0.3)])
def test_brute_force_equals_transfer_matrix(L, beta, h):
    assert ising.brute_force_lnZ_torus(L, beta, h) == pytest.approx(
        ising.transfer_matrix_lnZ_torus(L, beta, h), abs=1e-12)


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("beta", BETAS)
def test_kaufman_equals_brute_force(L, beta):
    assert ising.kaufman_lnZ_torus(L, beta) == pytest.approx(
        ising.brute_force_lnZ_torus(L, beta), abs=1e-12)


@pytest.mark.parametrize("L", [6, 8, 10])
@pytest.mark.parametrize("beta", BETAS)
def test_kaufman_equals_transfer_matrix(L, beta):
    assert ising.kaufman_lnZ_torus(L, beta) == pytest.approx(
        ising.transfer_matrix_lnZ_torus(L, beta), abs=1e-10)


def test_onsager_at_criticality_is_catalan_closed_form():
    catalan, _ = integrate.quad(lambda x: math.atan(x) / x, 0.0, 1.0, epsabs=1e-15, epsrel=1e-15)
    assert ising.onsager_lnZ_per_site(BETA_C) == pytest.approx(
        0.5 * math.log(2.0) + 2.0 * catalan / math.pi, abs=1e-13)


def test_kaufman_approaches_onsager():
    # disordered phase: finite-size corrections are exponentially small
    L = 64
    assert ising.kaufman_lnZ_torus(L, 0.3) / L**2 == pytest.approx(ising.onsager_lnZ_per_site(0.3), abs=1e-13)
    # ordered phase: two degenerate ground states add ln 2 to ln Z
    d = ising.kaufman_lnZ_torus(L, 0.6) - L * L * ising.onsager_lnZ_per_site(0.6)
    assert d == pytest.approx(math.log(2.0), abs=1e-8)


@pytest.mark.parametrize("beta,h", [(BETA_C, 0.0), (0.4, 0.1)])
def test_site_tensor_unfolding_has_rank_two(beta, h):
    T = ising.site_tensor(beta, h)
    for split in (0, 1):
        M, _, _ = trg.unfold(T, split)
        s = np.linalg.svd(M, compute_uv=False)
        assert s[1] > 1e-3 * s[0] and s[2] < 1e-13 * s[0]


def test_site_tensor_bond_factorisation():
    # contracting two half-bonds reproduces the nearest-neighbour weight
    beta = 0.37
    T = ising.site_tensor(beta)
    c, s = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
    W = np.array([[c, s], [c, -s]])
    B = W @ W.T
    assert np.allclose(B, [[math.exp(beta), math.exp(-beta)], [math.exp(-beta), math.exp(beta)]], atol=1e-14)
    assert T.shape == (2, 2, 2, 2)
