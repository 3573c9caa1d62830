"""Writes topk_refs.json: deterministic top-k TRG chains (Section II,
Eq. approxSVD: every step keeps the k largest singular values) of the FP64
oracle at the precision configurations - k = 48 at beta_c, h = 0, 24 steps
(2^24 sites) and k = 64 at beta = 0.42, h = 0.1, 20 steps (2^20 sites) -
with ln|Z| per site and ln c per step.  The GPU's contraction dtypes are
compared with these paired values.  Calls only the oracle.  Run from the
repository root:
    python tests/golden/make_topk_refs.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ising, trg  # noqa: E402
from workloads import BETA_C  # noqa: E402

CONFIGS = {"k48_betac_h0_24": (48, BETA_C, 0.0, 24), "k64_b042_h01_20": (64, 0.42, 0.1, 20)}


def main():
    out = {}
    for name, (k, beta, h, n) in CONFIGS.items():
        t0 = time.time()
        r = trg.run_shared(ising.site_tensor(beta, h), n, k, 0, 0, mode="topk")
        out[name] = {"k": k, "beta": beta, "h": h, "n_steps": n, "sign": r.sign,
                     "ln_abs_Z_per_site": r.ln_abs_Z / 2.0 ** n, "ln_c": r.ln_c,
                     "candidates": [[sp.c for sp in st.splits] for st in r.records]}
        print(f"{name}: ln|Z|/N = {r.ln_abs_Z / 2.0 ** n:.15f} in {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "topk_refs.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
