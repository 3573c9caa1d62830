"""Philox4x64-10 counter-based generator and the uniform draws of the sampler.

Test infrastructure only (see the package docstring).

The paper leaves the source of randomness open (Section II only requires
subsets e drawn with probability p(e)).  Both the oracle and the HIP path
draw every uniform from Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), addressed by a
counter that names the draw, so that a draw never depends on execution
order or batch composition.

Definition used here (from the SC'11 paper): state (x0,x1,x2,x3) of 64-bit
words, key (k0,k1).  One round:
    (hi0, lo0) = M0 * x0 (128-bit product),  (hi1, lo1) = M1 * x2,
    (x0,x1,x2,x3) <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0),
with M0 = 0xD2E7470EE14C6C93, M1 = 0xCA5A826395121157; between rounds the
key is bumped by the Weyl constants (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B).
Ten rounds.

Counter map of one selection uniform (this library's convention):
    key     = (seed, 0)
    counter = (sample_id, position_id, (purpose << 32) | (step << 1) | split,
               m >> 2)
    word    = m & 3 of the four output words
    u       = (word >> 11) * 2^-53            (in [0, 1))
with purpose 0 = subset selection, split 0 = A split ((l,u)|(r,d)),
1 = B split ((u,r)|(d,l)), step counted from 0, m the 0-based candidate
index, position_id 0 in shared mode.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block: four 64-bit counter words, two key words ->
    four 64-bit output words (Python ints)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for rnd in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0), lo1, (hi0 ^ x3 ^ k1), lo0
        if rnd != 9:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
    return x0, x1, x2, x3


def word_to_uniform(x: int) -> float:
    """Top 53 bits of a 64-bit word scaled to [0, 1)."""
    return float(x >> 11) * (2.0 ** -53)


def selection_uniforms(seed: int, sample_id: int, position_id: int, step: int,
                       split: int, count: int, purpose: int = 0) -> np.ndarray:
    """Uniforms u_0 .. u_{count-1} for the candidate indices m of one
    decomposition (see the counter map in the module docstring)."""
    w2 = ((purpose << 32) | (step << 1) | split) & MASK64
    out = np.empty(count, dtype=np.float64)
    for blk in range((count + 3) // 4):
        words = philox4x64_10((sample_id, position_id, w2, blk), (seed, 0))
        for j in range(4):
            m = 4 * blk + j
            if m < count:
                out[m] = word_to_uniform(words[j])
    return out
