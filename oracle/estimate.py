"""Monte Carlo estimate of ln Z from per-sample results (oracle).

Test infrastructure only (see the package docstring).

Section III, Eq. infiniteEnsemble: the sample mean of the traces converges
to Z.  Section V, Eq. shrunkDev: the error of the mean is the per-sample
error over sqrt(number of samples).  Samples may be negative (a truncated
tensor is not a nonnegative tensor), so the mean is taken with signs in the
log domain.  Also reported: mean(ln|Z~|)/N, a Jensen-biased but
well-conditioned summary used for very large N.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Estimate:
    ln_meanZ_per_site: float
    rel_stderr_Z: float
    mean_lnZ_per_site: float
    stderr_mean_lnZ: float
    n_used: int
    n_negative: int
    n_failed: int


def estimate_lnZ(sign: np.ndarray, ln_abs_Z: np.ndarray, n_sites: float) -> Estimate:
    sign = np.asarray(sign)
    ln_abs_Z = np.asarray(ln_abs_Z, dtype=np.float64)
    ok = (sign != 0) & np.isfinite(ln_abs_Z)
    n_failed = int(np.count_nonzero(~ok))
    s = sign[ok].astype(np.float64)
    l = ln_abs_Z[ok]
    n = int(l.size)
    if n == 0:
        return Estimate(math.nan, math.nan, math.nan, math.nan, 0, 0, n_failed)
    m = float(np.max(l))
    z = s * np.exp(l - m)               # Z~_i / e^m
    mean = float(np.mean(z))
    if mean > 0:
        ln_mean = (m + math.log(mean)) / n_sites
    else:
        ln_mean = math.nan
    if n > 1 and mean != 0:
        var = float(np.sum((z - mean) ** 2)) / (n - 1)
        rel = math.sqrt(var / n) / abs(mean)
        sd_l = float(np.std(l, ddof=1))
        se_l = sd_l / math.sqrt(n) / n_sites
    else:
        rel, se_l = math.nan, math.nan
    return Estimate(ln_mean, rel, float(np.mean(l)) / n_sites, se_l, n,
                    int(np.count_nonzero(s < 0)), n_failed)
