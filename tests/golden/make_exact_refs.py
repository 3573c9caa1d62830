"""Writes exact_refs.json: exact ln Z references used by the tests and the
bench, computed only with the CPU oracle (Kaufman's finite torus formula
and Onsager's free energy).  Run from the repository root:
    python tests/golden/make_exact_refs.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ising  # noqa: E402
from workloads import BETA_C  # noqa: E402


def main():
    refs = {
        "beta_c": BETA_C,
        "kaufman_lnZ_per_site": {},
        "onsager_lnZ_per_site": {},
    }
    for L in (4, 16, 1024):
        refs["kaufman_lnZ_per_site"][f"L{L}_betac"] = ising.kaufman_lnZ_torus(L, BETA_C) / (L * L)
    for b in (0.30, 0.35, 0.42, BETA_C, 0.55, 0.60):
        refs["onsager_lnZ_per_site"][f"{b:.17g}"] = ising.onsager_lnZ_per_site(b)
    with open(os.path.join(HERE, "exact_refs.json"), "w") as f:
        json.dump(refs, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
