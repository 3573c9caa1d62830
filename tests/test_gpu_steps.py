"""Step-level parity: the HIP decomposition, sampler and contraction against
the CPU oracle on identical inputs (paper Section II Eq. exactSVD, the
sampling/reweighting of Section II, and the Levin-Nave contraction of
Section III).  Inputs are seeded; sizes span several tiles and ragged tails."""
import math

import numpy as np
import pytest

from oracle import esp, ising, trg
from oracle.philox import selection_uniforms
from workloads import BETA_C, gaussian_tensor

from gpu_util import log, need_gpu

pytestmark = pytest.mark.gpu


def ising_unfoldings(k, steps, beta=BETA_C, h=0.0, seed=0, sample=0):
    """(M_A, M_B, col shapes) of the shared-chain tensors at each step."""
    T = ising.site_tensor(beta, h)
    out = []
    for step in range(steps):
        for split in (0, 1):
            M, rs, cs = trg.unfold(T, split)
            out.append((M.copy(), cs))
        r = trg.run_shared(T, 1, k, seed, sample + 1000 * step, keep_tensors=True)
        T = r.records[0].T_hat
    return out


@pytest.mark.parametrize("d1,d2,nm", [(2, 2, 3), (4, 4, 5), (5, 6, 4), (8, 8, 6), (16, 16, 3), (24, 24, 2),
                                      (33, 34, 2), (36, 36, 1), (48, 48, 1)])
def test_svd_random(d1, d2, nm):
    torch, m = need_gpu()
    log(f"svd_random d1={d1} d2={d2} nm={nm}")
    rng = np.random.default_rng(d1 * 100 + d2)
    n = d1 * d2
    # graded spectra: random orthogonal * geometric singular values * random orthogonal
    Ms = []
    for i in range(nm):
        U, _ = np.linalg.qr(rng.standard_normal((n, n)))
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        s = np.logspace(0, -8 * (i % 2 + 1), n)
        Ms.append((U * s) @ V.T)
    Ms = np.stack(Ms)
    sig, V, sw = m.svd_batched(torch.tensor(Ms, device="cuda"), d1, d2)
    sig, V, sw = sig.cpu().numpy(), V.cpu().numpy(), sw.cpu().numpy()
    assert np.all(sw > 0)
    for i in range(nm):
        U0, s0, Vt0 = trg.decompose(Ms[i], (d1, d2))
        assert np.max(np.abs(sig[i] - s0)) <= 1e-13 * s0[0] * math.sqrt(n)
        # vectors of well-separated values (relative gap > 1e-3) agree after the gauge
        gaps = np.minimum(np.abs(np.diff(np.r_[np.inf, s0])), np.abs(np.diff(np.r_[s0, -np.inf])))
        ok = (gaps > 1e-3 * s0) & (s0 > 1e-6 * s0[0])
        err = np.max(np.abs(V[i][ok] - Vt0[ok]))
        assert err < 1e-9, err


def test_svd_ising_unfoldings():
    torch, m = need_gpu()
    log("svd_ising_unfoldings")
    for (M, cs) in ising_unfoldings(8, 5):
        U0, s0, Vt0 = trg.decompose(M, cs)
        sig, V, sw = m.svd_batched(torch.tensor(M[None], device="cuda"), cs[0], cs[1])
        sig, V = sig.cpu().numpy()[0], V.cpu().numpy()[0]
        assert np.max(np.abs(sig - s0)) <= 1e-14 * s0[0] * M.shape[0]
        c = esp.n_candidates(s0, 1e-11)
        gaps = np.minimum(np.abs(np.diff(np.r_[np.inf, s0])), np.abs(np.diff(np.r_[s0, -np.inf])))
        ok = (np.arange(len(s0)) < c) & (gaps > 1e-6 * s0[0])
        assert np.max(np.abs(V[ok] - Vt0[ok])) < 1e-8


@pytest.mark.parametrize("k,mode", [(4, "shared"), (8, "shared"), (16, "shared"), (8, "topk"), (32, "shared")])
def test_sampler_matches_oracle(k, mode):
    torch, m = need_gpu()
    log(f"sampler k={k} mode={mode}")
    # spectra of real Ising unfoldings and of generic graded matrices
    sigmas = []
    for (M, cs) in ising_unfoldings(8, 5, beta=0.42, h=0.05):
        sigmas.append(np.linalg.svd(M, compute_uv=False))
    rng = np.random.default_rng(5)
    for n in (37, 64, 200, 256):
        sigmas.append(np.sort(np.exp(rng.uniform(-25, 0, n)))[::-1])
    sigmas.append(np.r_[1.0, 0.5, np.zeros(30)])           # fewer candidates than k
    nmax = max(s.size for s in sigmas)
    S = np.zeros((len(sigmas), nmax))
    for i, s in enumerate(sigmas):
        S[i, :s.size] = s
    jobs = len(sigmas)
    rngw = np.array([[7 + i, i % 3, 2 + i] for i in range(jobs)], dtype=np.int64)
    split = np.array([i % 2 for i in range(jobs)], dtype=np.int32)
    seed = 99
    out = m.sample_batched(torch.tensor(S, device="cuda"), torch.tensor(rngw, device="cuda"),
                           torch.tensor(split, device="cuda"), k, mode=mode, seed=seed)
    out = {key: v.cpu().numpy() for key, v in out.items()}
    for i in range(jobs):
        s = S[i]
        uf = lambda c, i=i: selection_uniforms(seed, int(rngw[i, 0]), int(rngw[i, 1]), int(rngw[i, 2]),
                                                 int(split[i]), c)
        tr = esp.truncate(s, k, "topk" if mode == "topk" else "stochastic", uf, 1e-11)
        kk = len(tr.sel)
        assert out["cand"][i] == tr.c
        assert out["kept"][i] == kk
        assert np.array_equal(out["sel"][i][:kk], tr.sel)
        assert np.all(out["sel"][i][kk:] == -1)
        assert np.allclose(out["log_r"][i][:kk], tr.log_r, rtol=0, atol=1e-12)
        assert np.allclose(out["weight"][i][:kk], tr.weights, rtol=1e-12, atol=0)


@pytest.mark.parametrize("D,kk,nj", [(2, 2, 3), (4, 4, 2), (4, 8, 2), (8, 8, 3), (8, 16, 2), (16, 16, 2),
                                     (6, 5, 2), (12, 12, 1)])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-5), ("bf16", 4e-2), ("fp8", 0.25)])
@pytest.mark.parametrize("tile", ["64", "128", "auto"])
def test_contract_matches_oracle(D, kk, nj, dtype, tol, tile, monkeypatch):
    """Both GEMM tile shapes (forced through the MCTRG_GEMM_TILE hook) and
    the autotuner's choice; shapes with and without whole 128 tiles."""
    torch, m = need_gpu()
    if tile != "auto":
        monkeypatch.setenv("MCTRG_GEMM_TILE", tile)
    log(f"contract D={D} kk={kk} nj={nj} {dtype} tile {tile}")
    rng = np.random.default_rng(D * 1000 + kk)
    GA = rng.standard_normal((nj, kk, D, D))
    GB = rng.standard_normal((nj, kk, D, D))
    FA = rng.standard_normal((nj, D, D, kk))
    FB = rng.standard_normal((nj, D, D, kk))
    out = m.contract_batched(*(torch.tensor(x, device="cuda") for x in (GA, GB, FA, FB)), dtype=dtype).cpu().numpy()
    for j in range(nj):
        ref = trg.contract(GA[j], GB[j], FA[j], FB[j])
        err = np.max(np.abs(out[j] - ref)) / np.max(np.abs(ref))
        assert err < tol, (dtype, err)
