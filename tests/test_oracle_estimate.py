"""Pins of the oracle's estimator against direct evaluation on values small
enough to exponentiate (Section III Eq. infiniteEnsemble, Section V
Eq. shrunkDev)."""
import math

import numpy as np
import pytest

from oracle.estimate import estimate_lnZ


def test_signed_mean_and_stderr():
    z = np.array([3.0, 1.5, -0.5, 2.0, 4.0])
    sign = np.sign(z).astype(np.int8)
    est = estimate_lnZ(sign, np.log(np.abs(z)), n_sites=4.0)
    assert est.ln_meanZ_per_site == pytest.approx(math.log(z.mean()) / 4.0, rel=1e-14)
    assert est.rel_stderr_Z == pytest.approx(z.std(ddof=1) / math.sqrt(5) / z.mean(), rel=1e-13)
    l = np.log(np.abs(z))
    assert est.mean_lnZ_per_site == pytest.approx(l.mean() / 4.0, rel=1e-14)
    assert est.stderr_mean_lnZ == pytest.approx(l.std(ddof=1) / math.sqrt(5) / 4.0, rel=1e-13)
    assert est.n_negative == 1 and est.n_used == 5 and est.n_failed == 0


def test_large_logs_do_not_overflow():
    l = np.array([1e6, 1e6 + 1.0, 1e6 - 2.0])
    est = estimate_lnZ(np.ones(3, np.int8), l, n_sites=2.0**20)
    want = (1e6 + math.log(np.mean(np.exp(l - 1e6)))) / 2.0**20
    assert est.ln_meanZ_per_site == pytest.approx(want, rel=1e-15)


def test_failed_samples_are_excluded():
    est = estimate_lnZ(np.array([1, 0, 1], np.int8), np.array([0.0, np.nan, math.log(3.0)]), 1.0)
    assert est.n_failed == 1 and est.n_used == 2
    assert est.ln_meanZ_per_site == pytest.approx(math.log(2.0))
