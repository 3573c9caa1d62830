"""The allocation-free sampling entry point (mctrg_sample_batched_noalloc)
against the allocating one (mctrg_sample_batched) and the oracle: two calls
in a row through the C ABI, the second with a smaller input, so that the
shared fixed scratch holds the first call's tables when the second runs.
Both run the same kernel, so the results must agree bit for bit; the kept
sets must also be the oracle's and the rates within 1e-12.  A request
beyond the fixed scratch is refused with ENOMEM."""
import numpy as np
import pytest

from oracle import esp
from oracle.philox import selection_uniforms

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


def _spectra(n, jobs, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(np.exp(rng.uniform(-30, 0, n)))[::-1] for _ in range(jobs)])


def _call(m, torch, S, k, seed, no_alloc):
    jobs = S.shape[0]
    rngw = np.array([[100 + i, i % 5, 3 + i % 7] for i in range(jobs)], dtype=np.int64)
    split = np.array([i % 2 for i in range(jobs)], dtype=np.int32)
    out = m.sample_batched(torch.tensor(S, device="cuda"), torch.tensor(rngw, device="cuda"),
                           torch.tensor(split, device="cuda"), k, seed=seed, no_alloc=no_alloc)
    return {key: v.cpu().numpy() for key, v in out.items()}, rngw, split


@pytest.mark.parametrize("first,second", [((1024, 32, 100), (256, 16, 9))])
def test_no_alloc_matches_allocating_entry_point(first, second):
    torch, m = need_gpu()
    for (n, k, jobs), seed in ((first, 5), (second, 6)):
        log(f"no-alloc sampler: n={n} k={k} jobs={jobs}")
        S = _spectra(n, jobs, seed)
        a, rngw, split = _call(m, torch, S, k, seed, no_alloc=False)
        b, _, _ = _call(m, torch, S, k, seed, no_alloc=True)
        for key in ("kept", "cand", "sel", "log_r", "weight"):
            assert np.array_equal(a[key], b[key]), key
        for i in (0, jobs // 2, jobs - 1):
            uf = lambda c, i=i: selection_uniforms(seed, int(rngw[i, 0]), int(rngw[i, 1]), int(rngw[i, 2]),
                                                     int(split[i]), c)
            tr = esp.truncate(S[i], k, "stochastic", uf, 1e-11)
            kk = len(tr.sel)
            assert b["cand"][i] == tr.c and b["kept"][i] == kk
            assert np.array_equal(b["sel"][i][:kk], tr.sel)
            assert np.allclose(b["log_r"][i][:kk], tr.log_r, rtol=0, atol=1e-12)


def test_no_alloc_refuses_beyond_its_scratch():
    torch, m = need_gpu()
    S = _spectra(1024, 200, 7)       # 200 jobs x 68,751 doubles > 8,388,608
    with pytest.raises(m.MctrgError) as e:
        _call(m, torch, S, 32, 7, no_alloc=True)
    assert e.value.status == m.ENOMEM
