"""Plain FP64 CPU oracle for Monte Carlo tensor-network renormalization.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference against which the HIP library is checked.  Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  The product path (``paper_1710_03757_amd``) never imports,
links or calls anything here, and nothing here imports the product path:
the two share no code.  The only module both sides use is ``workloads``,
which generates seeded inputs and holds none of the method's arithmetic.

Modules
-------
ising     Ising tensors (site/vertex and plaquette constructions) and exact
          partition functions: brute force, transfer matrix, Kaufman's
          finite-torus formula, Onsager's free energy.
philox    Philox4x64-10 counter-based generator and the uniform-draw map.
esp       Sampling of kept subsets with p(e) proportional to the product of
          squared singular values, and the inclusion rates r(S_ii)
          (Section II, Eqs. for w(e), p(e), r(S_ii)).
trg       One TRG coarse-graining step with exact, stochastic or top-k
          truncation, and whole chains in shared and independent modes
          (Section III).
lattice   Plaquette bookkeeping for independent mode on an L x L torus.
estimate  Signed log-sum-exp estimate of ln Z with error bars (Section III,
          Eq. infiniteEnsemble; Section V, Eq. shrunkDev).

Parity status: every function is pinned by a CPU test (tests/test_oracle_*)
except where its docstring says "parity unpinned".
"""
