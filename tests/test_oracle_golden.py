"""The stored exact references (tests/golden/exact_refs.json, written by
make_exact_refs.py from the oracle alone) against a fresh evaluation of
their closed forms: Kaufman's finite-torus ln Z per site at beta_c and
Onsager's thermodynamic limit, whose value at beta_c is also the closed
form ln(2)/2 + 2 G / pi (G = Catalan's constant)."""
import json
import math
import os

import pytest

from oracle import ising
from workloads import BETA_C

HERE = os.path.dirname(os.path.abspath(__file__))
CATALAN = 0.915965594177219015054603514932384110774


def test_exact_refs_are_current():
    refs = json.load(open(os.path.join(HERE, "golden", "exact_refs.json")))
    assert refs["beta_c"] == BETA_C
    for name, v in refs["kaufman_lnZ_per_site"].items():
        L = int(name[1:].split("_")[0])
        assert ising.kaufman_lnZ_torus(L, BETA_C) / (L * L) == pytest.approx(v, abs=1e-13), name
    for b, v in refs["onsager_lnZ_per_site"].items():
        assert ising.onsager_lnZ_per_site(float(b)) == pytest.approx(v, abs=1e-13), b
    assert refs["onsager_lnZ_per_site"][f"{BETA_C:.17g}"] == pytest.approx(
        0.5 * math.log(2.0) + 2.0 * CATALAN / math.pi, abs=1e-12)
    # finite tori approach the limit from above at beta_c
    k = refs["kaufman_lnZ_per_site"]
    assert k["L4_betac"] > k["L16_betac"] > k["L1024_betac"] > refs["onsager_lnZ_per_site"][f"{BETA_C:.17g}"]
