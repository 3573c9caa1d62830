"""The oracle against Table I of the paper (Section IV): the per-sample
standard deviation of Z~ / Z for the Ising model with 128 spins on the
bonds of a periodic 8 x 8 tensor network (plaquette construction, Fig. 1),
zero field, six TRG steps with independent sampling of every tensor.

The exact Z is the direct contraction of the 8 x 8 network (row transfer
matrices of 256 x 256); the fixture tests/golden/table1_std.txt holds the
paper's three rows.  The first row (kept count 6, T = 1.5) is cheap enough
for the CPU oracle: its standard deviation must agree with the paper's
within the statistical spread of 300 samples (the paper does not state its
sample count), and the mean must be 1 within three standard errors."""
import math
import os

import numpy as np

from oracle import ising, lattice, trg

HERE = os.path.dirname(os.path.abspath(__file__))


def table1_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_std.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, T, sd = line.split()
                rows.append((int(k), float(T), float(sd)))
    return rows


def exact_lnZ_8x8_plaquette(T):
    A = ising.plaquette_tensor(1.0 / T)
    return math.log(lattice.network_Z([A] * 64, 8))


def test_table1_fixture_rows():
    assert table1_rows() == [(6, 1.5, 4.171e-02), (28, 2.34826, 5.017e-04), (40, 2.34826, 1.353e-05)]


def test_exact_Z_of_the_network_is_the_medial_ising_sum():
    # the same contraction on a 2 x 2 network equals the spin sum over its 8 bond spins
    for T in (1.5, 2.34826):
        A = ising.plaquette_tensor(1.0 / T)
        assert math.log(lattice.network_Z([A] * 4, 2)) == \
            __import__("pytest").approx(ising.brute_force_lnZ_medial(2, 1.0 / T), abs=1e-12)


def test_table1_first_row():
    k, T, paper_sd = table1_rows()[0]
    lnZ = exact_lnZ_8x8_plaquette(T)
    A = ising.plaquette_tensor(1.0 / T)
    v = []
    for s in range(300):
        r = trg.run_independent(A, 6, k, 0, s)
        v.append(r.sign * math.exp(r.ln_abs_Z - lnZ))
    v = np.array(v)
    sd = v.std(ddof=1)
    se = sd / math.sqrt(v.size)
    print(f"Table I row 1: std {sd:.4e} (paper {paper_sd:.4e}), mean {v.mean():.5f} +- {se:.5f}")
    assert abs(v.mean() - 1.0) < 3.0 * se
    # 300 samples fix the standard deviation to ~10 % for these near-Gaussian values
    assert 0.75 < sd / paper_sd < 1.33
