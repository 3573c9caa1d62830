#!/usr/bin/env python3
"""Benchmark of the Monte Carlo TRG hot path on one MI355X.

Workload: the k = 32 form of the batched configuration - 2-D Ising site
tensors at beta_c, h = 0, 256 samples, a shared chain of warmup + steps
coarse-graining steps (default 5 + 20 = 25 steps, a 2^25-site lattice).  A
"step" is one full TRG step of the hot path (unfold, SVD of both splits,
subset sampling and reweighting, factors, contraction, normalisation) over
the whole batch.  The first ``--warmup`` steps (bond dimension 2 -> 4 ->
16 -> 32 and the first steps at 32) are untimed; the next ``--steps`` steps
are timed between device synchronisations, followed by the final trace and
the estimator.

Headline (``value``, ``dtype``): the paper's arithmetic, an FP64
contraction with the candidate cut tau_null = 1e-11.  Beside it
(``side_form``) the same window with an FP32 contraction (tau_null = 1e-6,
above that contraction's rounding floor), with its speedup over the FP64
form and both forms' |d ln Z|/site against the FP64 oracle.

``roofline``: the dominant kernel (larger busy time of the Jacobi rotation
kernel and the QR trailing update) against the FP64 MFMA peak, in the
method's algorithmic flops: the decomposition's (14/3) k^6 per
sample-step, attributed to the dominant kernel's dispatches of the window,
over their average duration (HIP events around every dispatch on the
library's own streams).  The kernel's own executed flops are reported
separately (``implementation_flops_per_launch``).  HBM traffic per dispatch
comes from the committed rocprofv3 counter summary when that was taken on
the same kernel source and workload window; with it, the kernel's HBM rate
over its busy time is set against a device copy timed live on the same GPU
(``hbm_probe``: the achievable rate for a read + write stream, well below the
8 TB/s nominal peak).  Also reported: the whole-step
roofline fraction, the MFMA rate of the coarse-graining GEMM, the same
window with the cheaper unbiased decomposition (``cheaper_decomposition``:
a QR-iteration basis instead of the SVD, its speedup and the spread of its
samples against the SVD form's) and the CPU oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import BETA_C  # noqa: E402

METRIC = "TRG sample-steps/s at χ=32 + MFMA util; |Δ ln Z|/site vs FP64 oracle"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
PEAK_HBM_TBS = 8.0
GEMM_ELT_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}
JACOBI_KERNEL = "jacobi_round64_kernel"
QR128_KERNEL = "qr_trailing128_kernel"
KERNEL_SRC = {JACOBI_KERNEL: os.path.join(ROOT, "paper_1710_03757_amd", "csrc", "k_jacobi.hip"),
              QR128_KERNEL: os.path.join(ROOT, "paper_1710_03757_amd", "csrc", "k_qr.hip")}
# Candidate cut tau_null (singular values <= tau_null * s_1 count as zero) per
# contraction dtype: about ten times the noise floor of the tensor the FP64
# decomposition sees.  For an FP64 contraction that floor is the SVD's own
# rounding (n eps), hence 1e-11; an FP32 contraction rounds T' at 2^-24 per
# operand, which gives singular values of 1e-8..1e-7 s_1 that carry no signal,
# hence 1e-6.  BF16 and FP8 keep the FP64 cut: ten times their rounding floor
# would cut most of the spectrum.
TAU_NULL = {"f64": 1e-11, "f32": 1e-6, "bf16": 1e-11, "fp8": 1e-11}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k32_batch256.json")


def window_key(k, batch, parts, tau, dtype, warmup, steps):
    return {"k": k, "batch": batch, "parts": parts, "tau_null": tau, "dtype": dtype, "warmup": warmup,
            "steps": steps}


def measured_traffic(kernel, key):
    """HBM bytes per dispatch of a kernel from the committed rocprofv3 --pmc
    FETCH_SIZE / WRITE_SIZE summary, if it was taken on the same kernel
    source and the same workload window (key); otherwise None."""
    try:
        rec = json.load(open(TRAFFIC_FILE))[kernel]
        sha = hashlib.sha256(open(KERNEL_SRC[kernel], "rb").read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source_sha256") != sha or rec.get("window") != key:
        return None
    return rec


def decomposition_flops(k: int) -> float:
    """Algorithmic FP64 flops of the decomposition per steady sample-step:
    two n x n splits (n = k^2), each n^3 (Gram) + 4/3 n^3 (reduction to
    tridiagonal form), i.e. (14/3) k^6."""
    return 14.0 / 3.0 * k ** 6


def gemm_flops(k: int) -> float:
    """Flops of the coarse-graining GEMM per steady sample-step: k^2 x k^2
    output, inner dimension D^2 = k^2, i.e. 2 k^6."""
    return 2.0 * k ** 6


def run_form(m, torch, args, dtype, tau, decomposition="svd"):
    """Runs the chains of one form over the window; returns its measurements."""
    k, B = args.k, args.batch
    n_chain = args.warmup + args.steps
    ts = m.init_tensor("site", [args.beta], [args.h])
    chain = m.Chain(ts, B, n_steps=n_chain, k=k, dtype=dtype, seed=0, profile=True, tau_null=tau,
                    decomposition=decomposition)
    for s in range(args.warmup):
        chain.step(1)
        print(f"[bench] {dtype}: warmup step {s} done, sweeps={chain.profile()['last_sweeps']}", flush=True)
    torch.cuda.synchronize()
    p0 = chain.profile()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    chain.step(args.steps)   # the timed steps in one call, as mctrg_run_samples advances a wave
    res = chain.finish()
    est = m.estimate_lnZ(res.sign, res.ln_abs_Z, 2.0 ** n_chain)
    ev1.record()
    torch.cuda.synchronize()
    p1 = chain.profile()
    ms_total = ev0.elapsed_time(ev1)
    print(f"[bench] {dtype}: timed {args.steps} steps in {ms_total:.1f} ms, sweeps "
          f"{p1['step_sweeps'][args.warmup:n_chain]}", flush=True)
    out = dict(ms_total=ms_total, value=B * args.steps / (ms_total / 1e3), ms_per_step=ms_total / args.steps,
               p0=p0, p1=p1, parts=p1["parts"], sweeps=p1["step_sweeps"][args.warmup:n_chain],
               pairs_last=p1["last_pairs"], ln=res.ln_abs_Z.cpu().numpy(), sign=res.sign.cpu().numpy(),
               est={k2: est[k2] for k2 in ("mean_lnZ_per_site", "stderr_mean_lnZ", "n_failed")})
    chain.close()
    ts.close()
    return out


def run_all_steps(m, torch, args, dtype, tau):
    """All steps 0..n-1 of a fresh chain of the headline form in one timed
    region (after the forms above, so that the GEMM tile autotuner has run:
    one-time setup - library load, autotuning, chain allocation and T0
    gather - stays outside)."""
    k, B = args.k, args.batch
    n_chain = args.warmup + args.steps
    ts = m.init_tensor("site", [args.beta], [args.h])
    chain = m.Chain(ts, B, n_steps=n_chain, k=k, dtype=dtype, seed=0, tau_null=tau)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    chain.step(n_chain)
    chain.finish()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    chain.close()
    ts.close()
    print(f"[bench] {dtype}: all {n_chain} steps in {ms:.1f} ms", flush=True)
    return {"value": B * n_chain / (ms / 1e3), "unit": "sample-steps/s", "steps": n_chain, "ms_total": ms,
            "note": f"steps 0..{n_chain - 1} of a fresh {B}-sample chain of the headline form (the small early "
                    "steps included); setup and tile autotuning outside the timed region"}


def gemm_floor(dt, k, batch):
    """(HBM bytes, MFMA ms, HBM ms) of one batched coarse-graining GEMM: the
    two k^2 x k^2 operands in the dtype, the k^2 x k^2 output in its
    accumulator type (8 bytes for FP64, else 4), the flops at the dtype's
    dense MFMA peak and the bytes at the nominal HBM peak."""
    nbytes = batch * k ** 4 * (2 * GEMM_ELT_BYTES[dt] + (8 if dt == "f64" else 4))
    t_mfma = gemm_flops(k) * batch / (PEAK_TFLOPS[dt] * 1e12) * 1e3
    t_hbm = nbytes / (PEAK_HBM_TBS * 1e12) * 1e3
    return nbytes, t_mfma, t_hbm


def contraction_alone(m, torch, args, dtypes):
    """The coarse-graining GEMM of each contraction dtype with nothing beside
    it: a one-part chain of the batch (one stream, so no other kernel runs
    during the GEMM) is advanced to the steady shape (D = k), and the GEMM of
    its next step is timed by the library's HIP events."""
    k, B = args.k, args.batch
    warm = 1
    while True:   # steps until the bond dimension reaches k
        D = 2
        for _ in range(warm):
            D = min(k, D * D)
        if D >= k:
            break
        warm += 1
    out = {}
    for dt in dtypes:
        ts = m.init_tensor("site", [args.beta], [args.h])
        chain = m.Chain(ts, B, n_steps=warm + 2, k=k, dtype=dt, seed=0, profile=True, tau_null=TAU_NULL[dt],
                        one_stream=True)
        chain.step(warm + 1)   # the first steady step also runs the tile autotuner for this shape
        p0 = chain.profile()
        chain.step(1)
        p1 = chain.profile()
        chain.close()
        ts.close()
        n = p1["gemm_launches"] - p0["gemm_launches"]
        ms = (p1["gemm_ms"] - p0["gemm_ms"]) / max(n, 1)
        ach = gemm_flops(k) * B / (ms / 1e3) / 1e12 if ms > 0 else None
        nbytes, t_mfma, t_hbm = gemm_floor(dt, k, B)
        out[dt] = {"kernel": f"gemm_tn_kernel<{dt}>", "achieved": ach, "peak": PEAK_TFLOPS[dt], "unit": "TFLOP/s",
                   "frac": ach / PEAK_TFLOPS[dt] if ach else None, "avg_launch_ms": ms, "launches": n,
                   "hbm_bytes_per_launch": nbytes, "bound": "mfma" if t_mfma >= t_hbm else "hbm",
                   "floor_ms": max(t_mfma, t_hbm), "frac_of_floor": max(t_mfma, t_hbm) / ms if ms > 0 else None}
        print(f"[bench] {dt}: GEMM alone {ms:.3f} ms ({ach:.1f} TF/s)", flush=True)
    return {"per_dtype": out, "batch": B, "shape": f"{k * k} x {k * k} x {k * k} per sample (k^2 x k^2 output, "
                                                  "inner dimension D^2 = k^2)",
            "flop_count": "2 k^6 per sample",
            "floor": "the larger of the flops at the dtype's MFMA peak and the operand and output bytes at 8 TB/s "
                     "(the narrow dtypes write a 4-byte accumulator per output element, so at this shape their "
                     "GEMM is bound by HBM)",
            "note": "one part (one stream): the GEMM dispatch has the GPU to itself; in the chains of the headline "
                    "three parts overlap"}


# The other configurations of the batched estimator, at reduced sample counts
# so that each runs in under a minute (throughput per sample-step; the full
# counts would only repeat the same waves).  (betas, hs) span the groups,
# ks are assigned round-robin over blocks of 64 samples.
CONFIGS = {
    "c1": dict(workload="Ising h=0 at beta_c, k=8, 16x16 lattice (8 steps), FP64", betas=[BETA_C], hs=[0.0],
               ks=[8], n_steps=8, samples=1000, full_samples=1000, dtype="f64"),
    "c2": dict(workload="Ising h=0, k=16, 2^20 sites (20 steps), 16 betas in [0.30, 0.60], FP64",
               betas=[0.30 + 0.02 * i for i in range(16)], hs=[0.0], ks=[16], n_steps=20, samples=16 * 256,
               full_samples=16 * 10000, dtype="f64"),
    "c3": dict(workload="batched: k in {16, 24, 32}, 32 betas in [0.35, 0.55] x h in {0, 0.05}, 30 steps, FP32 "
                        "contraction", betas=[0.35 + 0.2 * i / 31 for i in range(32)], hs=[0.0, 0.05],
               ks=[16, 24, 32], n_steps=30, samples=1536, full_samples=65536, dtype="f32"),
    "c4": dict(workload="Ising h=0 at beta_c, k=48, 24 steps, BF16 contraction", betas=[BETA_C], hs=[0.0], ks=[48],
               n_steps=24, samples=48, full_samples=8192, dtype="bf16"),
    "c5": dict(workload="Ising beta=0.42, h=0.1, k=64, 20 steps, FP8 e4m3 contraction", betas=[0.42], hs=[0.1],
               ks=[64], n_steps=20, samples=16, full_samples=256, dtype="fp8"),
}


def run_configs(m, torch, names):
    """Sample-steps/s of each named configuration through mctrg_run_samples
    (one call for the whole batch; a short call of the same shapes before it
    runs the tile autotuner)."""
    out = {}
    for name in names:
        c = CONFIGS[name]
        betas = [b for b in c["betas"] for _ in c["hs"]]
        hs = [h for _ in c["betas"] for h in c["hs"]]
        ts = m.init_tensor("site", betas, hs)
        ng, n = len(betas), c["samples"]
        groups = [i % ng for i in range(n)]
        ks = [c["ks"][(i // 64) % len(c["ks"])] for i in range(n)]
        kw = dict(n_steps=c["n_steps"], k=max(c["ks"]), dtype=c["dtype"], tau_null=TAU_NULL[c["dtype"]], seed=0)
        warm = sorted(set(ks))
        m.run_samples(ts, len(warm), groups=[0] * len(warm), ks=warm, **kw)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        r = m.run_samples(ts, n, groups=groups, ks=ks, **kw)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        est = m.estimate_lnZ(r.sign, r.ln_abs_Z, 2.0 ** c["n_steps"])
        ts.close()
        out[name] = {"workload": c["workload"], "value": n * c["n_steps"] / (ms / 1e3), "unit": "sample-steps/s",
                     "samples": n, "samples_in_config": c["full_samples"], "n_steps": c["n_steps"], "ks": c["ks"],
                     "groups": ng, "dtype": c["dtype"], "tau_null": TAU_NULL[c["dtype"]], "ms": ms,
                     "n_failed": est["n_failed"]}
        print(f"[bench] config {name}: {n} samples x {c['n_steps']} steps in {ms:.1f} ms", flush=True)
    return out


def kernel_records(r, args, dtype, tau):
    """Roofline records of the Jacobi and the 128-column QR update for one
    form (the dominant first)."""
    k, B = args.k, args.batch
    p0, p1 = r["p0"], r["p1"]
    d = lambda f: p1[f] - p0[f]  # noqa: E731
    dec_alg = decomposition_flops(k) * B * args.steps
    recs = {
        JACOBI_KERNEL: dict(launches=d("jacobi_launches"), ms=d("jacobi_ms"), busy=d("jacobi_busy_ms"),
                            impl=d("jacobi_flops"),
                            impl_count=f"rotated block pairs ({d('jacobi_rotated_pairs')}) x 3 * 64^2 * rotated row "
                                       "length (Gram + update; Grams of orthogonal pairs not counted)"),
        QR128_KERNEL: dict(launches=d("qr128_launches"), ms=d("qr128_ms"), busy=d("qr128_busy_ms"),
                           impl=d("qr128_flops"),
                           impl_count="dense C <- C - V (T^T (V^T C)): 4 m 128 c + 128^2 c per job and launch"),
    }
    key = window_key(k, B, r["parts"], tau, dtype, args.warmup, args.steps)

    def record(name):
        x = recs[name]
        n = max(x["launches"], 1)
        avg = x["ms"] / n
        alg = dec_alg / n
        ach = alg / (avg / 1e3) / 1e12 if avg > 0 else None
        tr = measured_traffic(name, key)
        traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"] if tr else None
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                "frac": ach / PEAK_TFLOPS["f64"] if ach else None, "traffic": traffic,
                "traffic_unit": "HBM bytes per dispatch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "hbm_rate_over_busy_time_TBps": (traffic * x["launches"] / (x["busy"] / 1e3) / 1e12
                                                 if traffic and x["busy"] > 0 else None),
                "algorithmic_flops_per_launch": alg,
                "flop_count": "the decomposition's (14/3) k^6 FP64 flops per sample-step over the window, divided "
                              "by this kernel's dispatches in the window",
                "avg_launch_ms": avg, "launches": x["launches"], "parts": r["parts"], "busy_ms": x["busy"],
                "achieved_over_busy_time": dec_alg / (x["busy"] / 1e3) / 1e12 if x["busy"] > 0 else None,
                "implementation_flops_per_launch": x["impl"] / n,
                "implementation_rate_TFLOPs": x["impl"] / (x["ms"] / 1e3) / 1e12 if x["ms"] > 0 else None,
                "implementation_flop_count": x["impl_count"],
                "share_of_step_time": x["busy"] / r["ms_total"] if r["ms_total"] else None}

    dom = max(recs, key=lambda nme: recs[nme]["busy"])
    other = QR128_KERNEL if dom == JACOBI_KERNEL else JACOBI_KERNEL
    return record(dom), record(other)


def gemm_record(r, args, dtype):
    k, B = args.k, args.batch
    p0, p1 = r["p0"], r["p1"]
    gl, gms, gbusy = (p1[f] - p0[f] for f in ("gemm_launches", "gemm_ms", "gemm_busy_ms"))
    galg = gemm_flops(k) * B * args.steps
    g = {"kernel": f"gemm_tn_kernel<{dtype}>", "achieved": galg / (gms / 1e3) / 1e12 if gms > 0 else None,
         "achieved_over_busy_time": galg / (gbusy / 1e3) / 1e12 if gbusy > 0 else None,
         "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s", "avg_launch_ms": gms / max(gl, 1), "launches": gl,
         "busy_ms": gbusy, "flop_count": "2 k^6 per sample-step (k^2 x k^2 output, inner dimension k^2)"}
    g["frac"] = g["achieved"] / g["peak"] if g["achieved"] else None
    return g


def t_ideal(k, dtype):
    """SURVEY-style ideal time per sample-step at the peaks: algorithmic
    decomposition flops at FP64, contraction flops at the GEMM dtype,
    compulsory tensor bytes (read T, write T', FP64) at HBM peak."""
    return (decomposition_flops(k) / (PEAK_TFLOPS["f64"] * 1e12) + gemm_flops(k) / (PEAK_TFLOPS[dtype] * 1e12)
            + 2.0 * k ** 4 * 8 / (PEAK_HBM_TBS * 1e12))


def cpu_baseline(args):
    """Times the CPU oracle (FP64, tau_null 1e-11) on the first chains of the
    batch; returns the rate over the timed window's steps and its results."""
    import numpy as np
    from oracle import ising, trg
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=None)
    except Exception:
        pass
    k = args.k
    T0 = ising.site_tensor(args.beta, args.h)
    t_steady, n_steady, results = 0.0, 0, []
    n = args.warmup + args.steps
    for sid in range(args.cpu_samples):
        T = T0.copy()
        ln_c = []
        for step in range(n):
            t0 = time.perf_counter()
            FA, GA, _ = trg.decompose_and_truncate(T, 0, k, "shared", 0, sid, 0, step, 1e-11)
            FB, GB, _ = trg.decompose_and_truncate(T, 1, k, "shared", 0, sid, 0, step, 1e-11)
            Tn = trg.contract(GA, GB, FA, FB)
            c = float(np.max(np.abs(Tn)))
            T = Tn / c
            ln_c.append(math.log(c))
            dt = time.perf_counter() - t0
            if step >= args.warmup:
                t_steady += dt
                n_steady += 1
        tr = trg.trace(T)
        N = 2.0 ** n
        ln = sum((N / 2.0 ** (s + 1)) * v for s, v in enumerate(ln_c)) + math.log(abs(tr))
        results.append((1 if tr > 0 else -1, ln))
        print(f"[bench] oracle chain {sid} done", flush=True)
    return {
        "value": n_steady / t_steady,
        "unit": "sample-steps/s",
        "cores": threads if threads else os.cpu_count(),
        "kind": "oracle",
        "sample": f"{args.cpu_samples} chains x {args.steps} timed steps (steps {args.warmup}..{n - 1}) at k={k} "
                  f"(n={k * k}); NumPy/LAPACK FP64 SVD and einsum contraction, tau_null 1e-11",
        "seconds": t_steady,
    }, results


def accuracy(r, ores, n_chain, dtype, tau):
    N = 2.0 ** n_chain
    diffs = [abs(float(r["ln"][i]) - o[1]) / N for i, o in enumerate(ores)]
    return {"abs_dlnZ_per_site_vs_f64_oracle": diffs, "max": max(diffs), "samples": len(ores),
            "signs_equal": bool(all(int(r["sign"][i]) == o[0] for i, o in enumerate(ores))), "lattice_sites": N,
            "note": f"same Philox draws; GPU contraction {dtype} with tau_null {tau:g}; oracle FP64, tau_null 1e-11"}


def hbm_probe(torch, mib=2048, reps=5):
    """Achievable HBM bandwidth on this GPU, measured live: a device-to-device
    copy (read + write) of ``mib`` MiB, the best of ``reps`` runs timed with
    events on the current stream."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms)

    nbytes = n * 4
    copy_ms = best(lambda: dst.copy_(src))
    del src, dst
    return {"bytes": nbytes, "copy_TBps": 2 * nbytes / (copy_ms / 1e3) / 1e12,
            "note": "bytes read + written by a device-to-device copy over its time"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16", "fp8"],
                    help="contraction dtype of the headline form")
    ap.add_argument("--side-dtype", default="f32", choices=["none", "f64", "f32", "bf16", "fp8"],
                    help="contraction dtype of the form run beside the headline")
    ap.add_argument("--cheap-decomposition", default="qr3", choices=["none", "qr3", "qr5"],
                    help="also run the headline dtype with the QR-iteration basis instead of the SVD")
    ap.add_argument("--beta", type=float, default=BETA_C)
    ap.add_argument("--h", type=float, default=0.0)
    ap.add_argument("--tau-null", type=float, default=None,
                    help="candidate cut of the headline form (default: per contraction dtype, see TAU_NULL)")
    ap.add_argument("--cpu-samples", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", default="",
                    help="comma-separated names of other configurations to time after the headline (" +
                         ", ".join(CONFIGS) + "), reported under 'configs'")
    ap.add_argument("--no-gemm-alone", action="store_true",
                    help="skip the GEMM of every contraction dtype timed on its own")
    ap.add_argument("--no-all-steps", action="store_true",
                    help="skip the all-steps rate (a fresh chain of the headline form timed over every step)")
    ap.add_argument("--no-hbm-probe", action="store_true",
                    help="skip the live copy bandwidth probe that the dominant kernel's HBM rate is set against")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, copy this many MiB device-to-device (a plain copy kernel of known "
                         "size whose counter readings calibrate FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): samples are independent, so a "
              "multi-GPU run would split sample ids across ranks and reduce the estimator partials once at "
              "the end; that path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_03757_amd as m

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    k, B = args.k, args.batch
    n_chain = args.warmup + args.steps
    tau = TAU_NULL[args.dtype] if args.tau_null is None else args.tau_null
    print(f"[bench] k={k} batch={B} dtype={args.dtype} warmup={args.warmup} steps={args.steps}", flush=True)
    r = run_form(m, torch, args, args.dtype, tau)
    roof, other = kernel_records(r, args, args.dtype, tau)
    dec_alg = decomposition_flops(k) * B * args.steps
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "sample-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"2-D Ising site tensors, beta={args.beta:.6f}, h={args.h}, k={k}, {B} samples, "
                               f"shared chain of {n_chain} steps (2^{n_chain} sites), steps "
                               f"{args.warmup}..{n_chain - 1} timed",
                   "k": k, "batch": B, "contract_dtype": args.dtype, "mode": "shared", "tau_null": tau,
                   "decomposition": "FP64 QR-preconditioned one-sided block Jacobi SVD",
                   "sampling_and_log_norm": "FP64"},
        "roofline": roof,
        "second_kernel": other,
        "decomposition": {"algorithmic_flops_per_sample_step": decomposition_flops(k),
                          "achieved_over_step_time": dec_alg / (r["ms_total"] / 1e3) / 1e12,
                          "frac_over_step_time": dec_alg / (r["ms_total"] / 1e3) / 1e12 / PEAK_TFLOPS["f64"],
                          "unit": "TFLOP/s", "peak": PEAK_TFLOPS["f64"]},
        "end_to_end_roofline_frac": t_ideal(k, args.dtype) / ((r["ms_total"] / 1e3) / (B * args.steps)),
        "mfma_contraction": gemm_record(r, args, args.dtype),
        "jacobi_sweeps_per_step": r["sweeps"],
        "jacobi_rotated_pairs_per_sweep_last_step": r["pairs_last"],
        "estimate_partial_chain": r["est"],
    }
    side = None
    if args.side_dtype != "none":
        stau = TAU_NULL[args.side_dtype]
        side = run_form(m, torch, args, args.side_dtype, stau)
        sroof, _ = kernel_records(side, args, args.side_dtype, stau)
        out["side_form"] = {
            "dtype": args.side_dtype, "tau_null": stau, "value": side["value"], "unit": "sample-steps/s",
            "ms_per_step": side["ms_per_step"], "speedup_vs_headline": side["value"] / r["value"],
            "end_to_end_roofline_frac": t_ideal(k, args.side_dtype) / ((side["ms_total"] / 1e3) / (B * args.steps)),
            "mfma_contraction": gemm_record(side, args, args.side_dtype),
            "dominant_kernel": {f: sroof[f] for f in ("kernel", "frac", "avg_launch_ms", "launches", "busy_ms",
                                                      "share_of_step_time")},
            "jacobi_sweeps_per_step": side["sweeps"], "estimate_partial_chain": side["est"]}
    if args.cheap_decomposition != "none":
        q = run_form(m, torch, args, args.dtype, tau, decomposition=args.cheap_decomposition)
        import numpy as np
        N = 2.0 ** n_chain
        phi_s, phi_q = r["ln"] / N, q["ln"] / N
        sd_s, sd_q = float(np.std(phi_s, ddof=1)), float(np.std(phi_q, ddof=1))
        out["cheaper_decomposition"] = {
            "decomposition": f"{args.cheap_decomposition}: orthonormal basis of "
                             f"{3 if args.cheap_decomposition == 'qr3' else 5} QR-iteration steps, terms (M v)(v^T) "
                             "drawn and reweighted like SVD terms (unbiased for any orthonormal basis), no Jacobi",
            "dtype": args.dtype, "value": q["value"], "unit": "sample-steps/s", "ms_per_step": q["ms_per_step"],
            "speedup_vs_headline": q["value"] / r["value"],
            "spread_ln_Z_per_site": sd_q, "spread_ln_Z_per_site_svd": sd_s,
            "variance_ratio_vs_svd": (sd_q / sd_s) ** 2 if sd_s > 0 else None,
            "mean_ln_Z_per_site": float(np.mean(phi_q)), "mean_ln_Z_per_site_svd": float(np.mean(phi_s)),
            "mean_difference_over_stderr": float((np.mean(phi_q) - np.mean(phi_s)) /
                                                 math.sqrt(sd_q ** 2 / len(phi_q) + sd_s ** 2 / len(phi_s))),
            "note": "same samples and draws addressing as the headline; shared chains (one tensor per level)"}
    if not args.no_all_steps:
        out["all_steps"] = run_all_steps(m, torch, args, args.dtype, tau)
    if args.configs:
        out["configs"] = run_configs(m, torch, [c for c in args.configs.split(",") if c])
    if not args.no_gemm_alone:
        out["mfma_contraction_alone"] = contraction_alone(m, torch, args, ("f64", "f32", "bf16", "fp8"))
    if not args.no_cpu_baseline:
        base, ores = cpu_baseline(args)
        out["cpu_baseline"] = base
        out["accuracy"] = {args.dtype: accuracy(r, ores, n_chain, args.dtype, tau)}
        if side is not None:
            out["accuracy"][args.side_dtype] = accuracy(side, ores, n_chain, args.side_dtype,
                                                        TAU_NULL[args.side_dtype])
    if not args.no_hbm_probe:
        hb = hbm_probe(torch)
        out["hbm_probe"] = hb
        for rec in (out["roofline"], out["second_kernel"]):
            rate = rec.get("hbm_rate_over_busy_time_TBps")
            rec["hbm_rate_over_copy_rate"] = rate / hb["copy_TBps"] if rate else None
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = args.copy_probe_mb * (1 << 20)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
