#!/usr/bin/env python3
"""Benchmark of the Monte Carlo TRG hot path on one MI355X.

Workload (default): the k = 32 form of the batched configuration - 2-D
Ising site tensors at beta_c, h = 0, a chain of 30 coarse-graining steps
(2^30 sites), FP32 coarse-graining GEMM, FP64 decomposition, sampling and
log-normalisation, candidate cut tau_null = 1e-6 s_1 (see TAU_NULL).  A "step" is one full TRG step of the hot path (unfold,
Jacobi SVD of both splits, subset sampling and reweighting, factors,
contraction, normalisation) over the whole batch of samples.  The first
``--warmup`` steps (the ramp-up of the bond dimension 2 -> 4 -> 16 -> 32 and
one steady step) are untimed; the next ``--steps`` steps are timed between
device synchronisations, followed by the final trace and the estimator.

Output: one JSON line with the throughput in sample-steps/s, a roofline
record of the dominant kernel (the 128-column trailing update of the QR
preconditioning, timed live with HIP events around every launch on the
library's streams; its HBM traffic per launch from the committed rocprofv3
counter summary when that was taken on the same kernel source and workload),
the same timing for the Jacobi rotation kernel, the whole-step roofline
fraction, the MFMA rate of the coarse-graining GEMM, the accuracy against the
CPU oracle on the first samples, and the oracle's own rate on the host
cores.
"""
from __future__ import annotations

import argparse
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
JACOBI_KERNEL = "jacobi_round64_kernel"
QR128_KERNEL = "qr_trailing128_kernel"
KERNEL_SRC = {JACOBI_KERNEL: os.path.join(ROOT, "paper_1710_03757_amd", "csrc", "k_jacobi.hip"),
              QR128_KERNEL: os.path.join(ROOT, "paper_1710_03757_amd", "csrc", "k_qr.hip")}
# Candidate cut tau_null (singular values <= tau_null * s_1 count as zero) per
# contraction dtype: about ten times the noise floor of the tensor the FP64
# decomposition sees.  For an FP64 contraction that floor is the SVD's own
# rounding (n eps), hence 1e-11; an FP32 contraction rounds T' at 2^-24 per
# operand, which gives singular values of 1e-8..1e-7 s_1 that carry no signal,
# hence 1e-6 (the library then also leaves rows below a tenth of the cut
# unrotated).  BF16 and FP8 keep the FP64 cut: ten times their rounding floor
# would cut most of the spectrum.
TAU_NULL = {"f64": 1e-11, "f32": 1e-6, "bf16": 1e-11, "fp8": 1e-11}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k32_batch256.json")


def measured_traffic(kernel, k, batch, parts, tau):
    """HBM bytes per dispatch of a kernel from the committed rocprofv3 --pmc
    FETCH_SIZE / WRITE_SIZE summary, if it was taken on the same kernel
    source and workload shape (batch split in the same number of parts, same
    candidate cut); otherwise None."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))[kernel]
        sha = hashlib.sha256(open(KERNEL_SRC[kernel], "rb").read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("source_sha256") != sha or rec.get("k") != k or rec.get("batch") != batch or \
            rec.get("parts", 1) != parts or rec.get("tau_null") != tau:
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


def cpu_baseline(k, beta, h, n_chain_steps, warmup, steps, samples, dtype):
    """Times the CPU oracle on the same chains (steady steps only)."""
    import numpy as np
    from oracle import ising, trg
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=None)
    except Exception:
        pass
    T0 = ising.site_tensor(beta, h)
    t_steady = 0.0
    n_steady = 0
    results = []
    for sid in range(samples):
        T = T0.copy()
        ln_c = []
        for step in range(warmup + steps):
            t0 = time.perf_counter()
            FA, GA, _ = trg.decompose_and_truncate(T, 0, k, "shared", 0, sid, 0, step, 1e-11)
            FB, GB, _ = trg.decompose_and_truncate(T, 1, k, "shared", 0, sid, 0, step, 1e-11)
            Tn = trg.contract(GA, GB, FA, FB)
            c = float(np.max(np.abs(Tn)))
            T = Tn / c
            ln_c.append(math.log(c))
            dt = time.perf_counter() - t0
            if step >= warmup:
                t_steady += dt
                n_steady += 1
        n = warmup + steps
        tr = trg.trace(T)
        N = 2.0 ** n
        ln = sum((N / 2.0 ** (s + 1)) * v for s, v in enumerate(ln_c)) + math.log(abs(tr))
        results.append((1 if tr > 0 else -1, ln))
    return {
        "value": n_steady / t_steady,
        "unit": "sample-steps/s",
        "cores": threads if threads else os.cpu_count(),
        "kind": "oracle",
        "sample": f"{samples} chains x {steps} steady steps at k={k} (n={k * k}), after {warmup} untimed "
                  f"ramp-up steps; NumPy/LAPACK FP64, contraction FP64",
        "seconds": t_steady,
    }, results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=7)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--dtype", default="f32", choices=["f64", "f32", "bf16", "fp8"])
    ap.add_argument("--beta", type=float, default=BETA_C)
    ap.add_argument("--h", type=float, default=0.0)
    ap.add_argument("--chain-steps", type=int, default=30)
    ap.add_argument("--tau-null", type=float, default=None,
                    help="candidate cut (default: per contraction dtype, see TAU_NULL)")
    ap.add_argument("--cpu-samples", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the timed region, copy this many MiB device-to-device (a plain copy kernel of known "
                         "size whose counter readings calibrate FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): samples are independent, so a "
              "multi-GPU run would split sample ids across ranks and reduce the estimator partials once at "
              "the end; that path is not built.", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > args.chain_steps:
        print("warmup + steps must not exceed the chain length", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_03757_amd as m

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    k, B = args.k, args.batch
    print(f"[bench] k={k} batch={B} dtype={args.dtype} warmup={args.warmup} steps={args.steps}", flush=True)
    ts = m.init_tensor("site", [args.beta], [args.h])
    tau = TAU_NULL[args.dtype] if args.tau_null is None else args.tau_null
    chain = m.Chain(ts, B, n_steps=args.chain_steps, k=k, dtype=args.dtype, seed=0, profile=True, tau_null=tau)
    for s in range(args.warmup):
        chain.step(1)
        print(f"[bench] warmup step {s} done, sweeps={chain.profile()['last_sweeps']}", flush=True)
    torch.cuda.synchronize()
    p0 = chain.profile()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    # the timed steps in one call, as mctrg_run_samples advances a wave: the
    # two parts of the batch run free instead of joining after every step
    chain.step(args.steps)
    res = chain.finish()
    est = m.estimate_lnZ(res.sign, res.ln_abs_Z, 2.0 ** (args.warmup + args.steps))
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = chain.profile()
    sweeps = p1["step_sweeps"][args.warmup:args.warmup + args.steps]
    pair_hist = p1["last_pairs"]
    ms_total = ev0.elapsed_time(ev1)
    wall = t1 - t0
    print(f"[bench] timed {args.steps} steps: {ms_total:.1f} ms (events), {wall * 1e3:.1f} ms (wall), "
          f"sweeps {sweeps}", flush=True)
    ms_per_step = ms_total / args.steps
    value = B * args.steps / (ms_total / 1e3)

    parts = p1["parts"]
    jl = p1["jacobi_launches"] - p0["jacobi_launches"]
    jms = p1["jacobi_ms"] - p0["jacobi_ms"]
    jbusy = p1["jacobi_busy_ms"] - p0["jacobi_busy_ms"]
    gl = p1["gemm_launches"] - p0["gemm_launches"]
    gms = p1["gemm_ms"] - p0["gemm_ms"]
    gbusy = p1["gemm_busy_ms"] - p0["gemm_busy_ms"]
    ql = p1["qr128_launches"] - p0["qr128_launches"]
    qms = p1["qr128_ms"] - p0["qr128_ms"]
    qbusy = p1["qr128_busy_ms"] - p0["qr128_busy_ms"]
    qflops = p1["qr128_flops"] - p0["qr128_flops"]

    def traffic_of(kernel, launches, busy):
        tr = measured_traffic(kernel, k, B, parts, tau)
        t = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"] if tr else None
        return t, (t * launches / (busy / 1e3) / 1e12) if (t and busy > 0) else None

    # The roofline record is the dominant kernel's: of the two FP64 MFMA
    # kernels that take most of the step, the one with the larger busy time
    # (union of its launch intervals over both parts, whose launches run
    # concurrently).  achieved = its algorithmic flops over that busy time;
    # avg_launch_ms is the mean duration of one dispatch (what rocprofv3
    # reports per dispatch).
    # * qr_trailing128_kernel (the 128-column trailing update of the second to
    #   fifth QR): the dense count of C <- C - V (T^T (V^T C)), summed by the
    #   library over the timed launches.
    # * jacobi_round64_kernel: per rotated pair of 32-row blocks the 64 x 64
    #   Gram over the rotated row length (64^2 len, symmetric) and the update
    #   W <- Q^T W (2 64^2 len), summed by the library (len = the columns up
    #   to the rank limit of the QRs); the Grams of pairs found orthogonal are
    #   not counted, so this is a lower bound of the kernel's work.
    jpairs = p1["jacobi_rotated_pairs"] - p0["jacobi_rotated_pairs"]
    jflops = p1["jacobi_flops"] - p0["jacobi_flops"]
    recs = {
        QR128_KERNEL: dict(launches=ql, ms=qms, busy=qbusy, flops=qflops,
                           count="dense C <- C - V (T^T (V^T C)): 4 m 128 c + 128^2 c per job and launch"),
        JACOBI_KERNEL: dict(launches=jl, ms=jms, busy=jbusy, flops=jflops,
                            count=f"rotated block pairs ({jpairs}) x 3 * 64^2 * rotated row length (Gram + "
                                  "update; Grams of orthogonal pairs not counted)"),
    }

    def record(name):
        r = recs[name]
        ach = r["flops"] / (r["busy"] / 1e3) / 1e12 if r["busy"] > 0 else None
        traffic, rate = traffic_of(name, r["launches"], r["busy"])
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                "frac": (ach / PEAK_TFLOPS["f64"]) if ach else None, "traffic": traffic,
                "traffic_unit": "bytes per dispatch (HBM, FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_rate_TBs": rate, "avg_launch_ms": r["ms"] / max(r["launches"], 1),
                "launches": r["launches"], "parts": parts, "flops_per_launch": r["flops"] / max(r["launches"], 1),
                "flop_count": r["count"], "busy_ms": r["busy"],
                "share_of_step_time": r["busy"] / ms_total if ms_total else None}

    dom = max(recs, key=lambda n: recs[n]["busy"])
    roofline = record(dom)
    other = record(QR128_KERNEL if dom == JACOBI_KERNEL else JACOBI_KERNEL)
    # the whole FP64 decomposition against the algorithmic count of the
    # method ((14/3) k^6 per sample-step), over the step time
    decomposition = {"algorithmic_flops_per_sample_step": decomposition_flops(k),
                     "achieved_over_step_time": decomposition_flops(k) * B * args.steps / (ms_total / 1e3) / 1e12,
                     "unit": "TFLOP/s", "peak": PEAK_TFLOPS["f64"]}
    galg = gemm_flops(k) * B * args.steps
    gemm = {"kernel": f"gemm_tn_kernel<{args.dtype}>", "achieved": galg / (gbusy / 1e3) / 1e12 if gbusy > 0 else None,
            "peak": PEAK_TFLOPS[args.dtype], "unit": "TFLOP/s", "avg_launch_ms": gms / max(gl, 1), "launches": gl,
            "busy_ms": gbusy}
    gemm["frac"] = gemm["achieved"] / gemm["peak"] if gemm["achieved"] else None

    # whole-step roofline fraction: ideal time per sample-step at the peaks
    # (algorithmic decomposition flops at FP64, contraction flops at the GEMM
    # dtype, compulsory tensor bytes at HBM peak) over the measured time
    t_ideal = (decomposition_flops(k) / (PEAK_TFLOPS["f64"] * 1e12) + gemm_flops(k) / (PEAK_TFLOPS[args.dtype] * 1e12)
               + 2.0 * k ** 4 * 8 / (PEAK_HBM_TBS * 1e12))
    t_meas = (ms_total / 1e3) / (B * args.steps)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "sample-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2-D Ising site tensors, beta={args.beta:.6f}, h={args.h}, k={k}, chain of "
                               f"{args.chain_steps} steps (2^{args.chain_steps} sites), shared chain, "
                               f"steady-state steps {args.warmup}..{args.warmup + args.steps - 1}",
                   "k": k, "batch": B, "contract_dtype": args.dtype, "mode": "shared", "tau_null": tau,
                   "decomposition": "FP64 one-sided block Jacobi"},
        "roofline": roofline,
        "second_kernel": other,
        "decomposition": decomposition,
        "end_to_end_roofline_frac": t_ideal / t_meas,
        "mfma_contraction": gemm,
        "jacobi_sweeps_per_step": sweeps,
        "jacobi_rotated_pairs_per_sweep_last_step": pair_hist,
        "estimate_partial_chain": {k2: est[k2] for k2 in ("mean_lnZ_per_site", "stderr_mean_lnZ", "n_failed")},
    }

    if not args.no_cpu_baseline:
        base, ores = cpu_baseline(k, args.beta, args.h, args.chain_steps, args.warmup, args.steps,
                                  args.cpu_samples, args.dtype)
        out["cpu_baseline"] = base
        ln = res.ln_abs_Z.cpu().numpy()
        sg = res.sign.cpu().numpy()
        N = 2.0 ** (args.warmup + args.steps)
        diffs = [abs(float(ln[i]) - o[1]) / N for i, o in enumerate(ores)]
        out["accuracy"] = {"abs_dlnZ_per_site_vs_f64_oracle": diffs, "samples": len(ores),
                           "signs_equal": bool(all(int(sg[i]) == o[0] for i, o in enumerate(ores))),
                           "lattice_sites": N, "note": "same Philox draws; GPU contraction in "
                                                       f"{args.dtype} with tau_null {tau:g}, oracle FP64 "
                                                       "with tau_null 1e-11"}
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = args.copy_probe_mb * (1 << 20)
    print(json.dumps(out), flush=True)
    chain.close()


if __name__ == "__main__":
    main()
