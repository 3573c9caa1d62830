"""The cheaper decomposition (oracle ``decompose_qr``): a few steps of QR
iteration give an orthonormal basis V, and M = sum_j (M v_j) v_j^T holds
for any orthonormal V, so sampling the terms with p(e) proportional to the
product of |M v_j|^2 and dividing each kept term by its inclusion rate
(Section II) still averages to M exactly (Eqs. Tsum, Ssum need only r > 0).
Pinned here: the expansion is exact and V orthonormal; with many steps the
term norms tend to the singular values (so the iteration is what it says);
summing p(path) * Z~(path) over every sampling path of the independent
estimator with this basis gives Z exactly; and a Monte Carlo run is
unbiased against Kaufman's Z."""
import math

import numpy as np
import pytest

from oracle import ising, trg
from workloads import BETA_C, gaussian_tensor

from test_oracle_trg import _expected_Z_independent, network_lnZ


@pytest.mark.parametrize("n_qr", [3, 5])
def test_basis_is_orthonormal_and_expansion_exact(n_qr):
    M = trg.unfold(gaussian_tensor(5, seed=11), 0)[0]
    V = trg.qr_basis(M, n_qr)
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[0]))) < 1e-13
    U, s, Vt = trg.decompose_qr(M, ((5, 5)), n_qr)
    assert np.all(np.diff(s) <= 0)
    assert np.linalg.norm((U * s) @ Vt - M) < 1e-13 * np.linalg.norm(M)


def test_many_steps_give_the_singular_values():
    rng = np.random.default_rng(3)
    Q1, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    Q2, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    sv = 0.7 ** np.arange(40)
    M = Q1 @ np.diag(sv) @ Q2.T
    s3 = trg.decompose_qr(M, (40, 1), 3)[1]
    s41 = trg.decompose_qr(M, (40, 1), 41)[1]
    assert np.max(np.abs(s41[:10] - sv[:10])) < 1e-10
    assert np.max(np.abs(s3[:10] - sv[:10])) > np.max(np.abs(s41[:10] - sv[:10]))


@pytest.mark.parametrize("basis", ["qr3"])
def test_qr_basis_estimator_is_exactly_unbiased(basis):
    Ts = [gaussian_tensor(2, seed=200 + i) for i in range(4)]
    Z = network_lnZ(Ts, 2)
    EZ = _expected_Z_independent(Ts, 2, basis=basis)
    assert EZ == pytest.approx(Z, rel=1e-12)


def test_qr_basis_statistically_unbiased():
    T = ising.site_tensor(BETA_C)
    Z = math.exp(ising.kaufman_lnZ_torus(4, BETA_C))
    v = np.array([(lambda r: r.sign * math.exp(r.ln_abs_Z))(trg.run_independent(T, 4, 2, 0, s, basis="qr3"))
                  for s in range(300)])
    mean, se = v.mean(), v.std(ddof=1) / math.sqrt(v.size)
    assert abs(mean - Z) < 4 * se
    assert se / Z < 0.05
