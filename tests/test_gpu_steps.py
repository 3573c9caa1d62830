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


def approx_budget(tau):
    """Total Frobenius norm, relative to s_1, that the decomposition's
    approximations (early stop of the first QR, rank limit, deflation) may
    drop for the candidate cut tau (a tenth of the cut, at least 2^-48)."""
    return max(2.0 ** -48, tau / 10.0)


def check_svd(M, cs, sig, V, sw, tau, label):
    """The step's decomposition against the exact SVD (LAPACK through the
    oracle): every value within the Weyl bound of the dropped parts plus
    rounding (1e-13 sqrt(n) s_1); every vector whose value is isolated by a
    gap g within 4 eps / g of the exact one (the perturbation bound of
    singular subspaces, eps the same total perturbation), checked where that
    bound is below 1e-3; the rows of values above the budget orthonormal."""
    U0, s0, Vt0 = trg.decompose(M, cs)
    n = M.shape[0]
    eps = (approx_budget(tau) + 1e-13 * math.sqrt(n)) * s0[0]
    assert sw >= 1, (label, sw)
    verr = np.max(np.abs(sig - s0))
    assert verr <= eps, (label, verr, eps)
    assert np.all(np.diff(sig) <= 0)
    if V is None:
        return verr, 0.0, 0
    gaps = np.minimum(np.abs(np.diff(np.r_[np.inf, s0])), np.abs(np.diff(np.r_[s0, -np.inf])))
    bound = 4.0 * eps / np.maximum(gaps, 1e-300)
    ok = bound < 1e-3
    assert ok[0], (label, "the leading vector must be checked", gaps[0], eps)
    errs = np.max(np.abs(V[ok] - Vt0[ok]), axis=1)
    assert np.all(errs <= bound[ok]), (label, np.max(errs / bound[ok]))
    # zero values have zero rows; the rows above the budget are orthonormal
    assert np.all(V[sig == 0.0] == 0.0)
    top = sig > 10.0 * eps
    G = V[top] @ V[top].T
    assert np.max(np.abs(G - np.eye(int(top.sum())))) <= 1e-10 + 4.0 * eps / max(np.min(sig[top]), 1e-300)
    return verr, float(np.max(errs)), int(ok.sum())


@pytest.mark.parametrize("tau", [0.0, 1e-11, 1e-6])
@pytest.mark.parametrize("d1,d2,nm", [(2, 2, 3), (4, 4, 5), (5, 6, 4), (8, 8, 6), (16, 16, 3), (24, 24, 2),
                                      (33, 34, 2), (36, 36, 1), (48, 48, 1)])
def test_svd_random(d1, d2, nm, tau):
    """Graded spectra (random orthogonal x geometric values x random
    orthogonal, down to 1e-8 and 1e-16, and one of rank n/2), through every
    route of the decomposition: five or three QRs with the rank limit and
    deflation (n_pad <= 1024), three QRs (n_pad <= 4096)."""
    torch, m = need_gpu()
    log(f"svd_random d1={d1} d2={d2} nm={nm} tau={tau}")
    rng = np.random.default_rng(d1 * 100 + d2)
    n = d1 * d2
    Ms = []
    for i in range(nm):
        U, _ = np.linalg.qr(rng.standard_normal((n, n)))
        V, _ = np.linalg.qr(rng.standard_normal((n, n)))
        s = np.logspace(0, -8 * (i % 2 + 1), n)
        if i == 2:
            s[n // 2:] = 0.0
        Ms.append((U * s) @ V.T)
    Ms = np.stack(Ms)
    Md = torch.tensor(Ms, device="cuda")
    sig, V, sw = m.svd_batched(Md, d1, d2, tau_null=tau)
    sig2, V2, _ = m.svd_batched(Md, d1, d2, want_V=False, tau_null=tau)
    sig, V, sw, sig2 = sig.cpu().numpy(), V.cpu().numpy(), sw.cpu().numpy(), sig2.cpu().numpy()
    assert V2 is None
    # the values do not depend on whether the vectors are asked for
    assert np.array_equal(sig, sig2)
    for i in range(nm):
        verr, vecerr, nchk = check_svd(Ms[i], (d1, d2), sig[i], V[i], int(sw[i]), tau, f"{d1}x{d2}#{i}")
        log(f"  #{i}: |ds| {verr:.2e}  vectors checked {nchk} max err {vecerr:.2e}  sweeps {sw[i]}")


def test_svd_largest_size():
    """The largest decomposition the library takes, 64 x 64 = 4096 (the k =
    64 unfoldings): three QRs with 8-column panels, then 127 rounds per
    sweep; a graded spectrum down to 1e-12, across the candidate cut."""
    torch, m = need_gpu()
    d1 = d2 = 64
    tau = 1e-11
    log(f"svd_largest d1={d1} d2={d2} tau={tau}")
    rng = np.random.default_rng(6464)
    n = d1 * d2
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Ms = (U * np.logspace(0, -12, n)) @ V.T
    Ms = Ms[None]
    sig, V, sw = m.svd_batched(torch.tensor(Ms, device="cuda"), d1, d2, tau_null=tau)
    sig, V, sw = sig.cpu().numpy(), V.cpu().numpy(), sw.cpu().numpy()
    for i in range(1):
        verr, vecerr, nchk = check_svd(Ms[i], (d1, d2), sig[i], V[i], int(sw[i]), tau, f"{d1}x{d2}#{i}")
        log(f"  #{i}: |ds| {verr:.2e}  vectors checked {nchk} max err {vecerr:.2e}  sweeps {sw[i]}")


@pytest.mark.parametrize("tau", [0.0, 1e-11])
def test_svd_ising_unfoldings(tau):
    """The unfoldings of the shared chain's tensors at k = 8 (critical Ising,
    five steps, both splits): the values and the candidate vectors."""
    torch, m = need_gpu()
    log(f"svd_ising_unfoldings tau={tau}")
    for j, (M, cs) in enumerate(ising_unfoldings(8, 5)):
        sig, V, sw = m.svd_batched(torch.tensor(M[None], device="cuda"), cs[0], cs[1], tau_null=tau)
        check_svd(M, cs, sig.cpu().numpy()[0], V.cpu().numpy()[0], int(sw.cpu().numpy()[0]), tau, f"unfolding {j}")


def test_svd_rejects_bad_arguments():
    torch, m = need_gpu()
    M = torch.zeros((1, 4, 4), dtype=torch.float64, device="cuda")
    for tau in (-1e-3, 1.0, float("nan")):
        with pytest.raises(m.MctrgError):
            m.svd_batched(M, 2, 2, tau_null=tau)
    with pytest.raises(m.MctrgError):
        m.svd_batched(torch.zeros((1, 4225, 4225), dtype=torch.float64, device="cuda"), 65, 65)


def test_step_entries_empty_batches_and_zero_matrix():
    """Empty batches return at once through every step entry point (NULL
    pointers allowed); an all-zero matrix and a rank-one matrix decompose to
    their exact spectra (zero values with zero vector rows)."""
    import ctypes
    torch, m = need_gpu()
    lib = m._lib
    assert lib.mctrg_svd_batched(0, 4, 4, None, 1e-11, None, None, None, None) == 0
    assert lib.mctrg_sample_batched(0, 16, 4, 0, 0, 1e-11, None, None, None, None, None, None, None, None,
                                    None) == 0
    assert lib.mctrg_sample_batched_noalloc(0, 16, 4, 0, 0, 1e-11, None, None, None, None, None, None, None,
                                            None, None) == 0
    assert lib.mctrg_contract_batched(0, 4, 4, 0, None, None, None, None, None, None) == 0
    # sizes are still checked on an empty batch
    assert lib.mctrg_svd_batched(0, 65, 65, None, 1e-11, None, None, None, None) != 0
    sig, V, sw = m.svd_batched(torch.zeros((0, 16, 16), dtype=torch.float64, device="cuda"), 4, 4)
    assert sig.shape == (0, 16) and V.shape == (0, 16, 16) and sw.shape == (0,)
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal(36), rng.standard_normal(36)
    Ms = np.stack([np.zeros((36, 36)), 3.0 * np.outer(u, v)])
    sig, V, sw = m.svd_batched(torch.tensor(Ms, device="cuda"), 6, 6, tau_null=1e-11)
    sig, V = sig.cpu().numpy(), V.cpu().numpy()
    assert np.all(sig[0] == 0.0) and np.all(V[0] == 0.0)
    s1 = 3.0 * np.linalg.norm(u) * np.linalg.norm(v)
    assert abs(sig[1, 0] - s1) <= 1e-13 * s1 and np.all(np.abs(sig[1, 1:]) <= 1e-13 * s1)
    vh = v / np.linalg.norm(v)
    assert abs(abs(V[1, 0] @ vh) - 1.0) <= 1e-12


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
