#!/usr/bin/env python3
"""Throughput of the ChiSao per-cycle population update on one MI355X.

Workload (the paper's Gaussian-mixture objective, anisotropic, at d=64): 128
components with centres in [-20,20]^64 and covariances Q diag(lam) Q^T
(lam log-uniform in [0.05,1]), N=65536 samples, L-BFGS memory 10, 18 L-BFGS
iterations, 3 smoothing steps of 16 probes at sigma=0.1, 5 anti-convergence
steps.  A step is one (non-final) oscillation cycle: all six phases.

The metric counts sample-iterations nominally: N * (n_conv + n_cloud + n_anti)
per cycle, masked samples included.  `value` is the adjoint-gradient
throughput; the finite-difference throughput on the same schedule and the
ratio between the two are reported beside it, together with the roofline
position of the dominant kernel (HIP events around its launches during the
timed cycles) and the FP64 CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = "sample-iterations/s at d=64,N=65536 (adjoint vs FD grad); mode recall vs oracle"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def eval_flops_per_point(d: int, K: int) -> int:
    """Algorithmic flops of one objective (+adjoint) evaluation: per component
    the contraction u = P (x - mu) (2 d^2), the quadratic form delta . u (2 d)
    and the gradient accumulation (2 d)."""
    return K * (2 * d * d + 4 * d)


def lbfgs_bytes_per_step(d: int, m: int) -> int:
    """Algorithmic HBM bytes of one L-BFGS direction + pair update for one
    sample with a full history: read x, x_prev, g, g_prev, S, Y (m d each), rho;
    write the new pair and the direction."""
    return lbfgs_bytes(d, 1, m)


def lbfgs_bytes(d: int, steps: int, pairs: int) -> int:
    """Algorithmic HBM bytes of `steps` L-BFGS sample-steps whose two-loops read
    `pairs` history pairs in total: per step x, x_prev, g, g_prev read (4d), the
    new pair written (2d + 1) and the direction written (d); per pair s, y and
    rho read (2d + 1)."""
    return 4 * (steps * (7 * d + 1) + pairs * (2 * d + 1))


HERE = os.path.dirname(os.path.abspath(__file__))
COUNTERS = os.path.join(HERE, "profiles", "eval_kernel_gauss128_d64_counters.md")


def eval_source_digest() -> str:
    """Digest of the evaluation kernel's sources, comments and blank space
    removed: hardware-counter figures are only used while the kernel is the
    one they were taken from."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("eval.hip", "common.h", "kernels.h"):
        with open(os.path.join(HERE, "paper_2606_26164_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update("\n".join(ln.strip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when absent or taken from a different kernel source."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    vals = dict(ln.split(": ", 1) for ln in text.splitlines() if ln.startswith(("traffic_bytes", "eval_source")))
    if vals.get("eval_source_sha256", "").strip() != eval_source_digest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(prob, cfg, x0, warmup, steps, profile=True):
    import torch

    from paper_2606_26164_amd.api import Optimizer

    opt = Optimizer(prob, cfg, x0)
    per_cycle = []
    for i in range(warmup):
        torch.cuda.synchronize()
        t = time.perf_counter()
        opt.cycle(1)
        torch.cuda.synchronize()
        per_cycle.append(time.perf_counter() - t)
        log(f"  warmup cycle {i + 1}: {per_cycle[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    if profile:
        opt.profile_begin()
    t0 = time.perf_counter()
    stats = opt.cycle(steps, stats=True) if steps > 0 else []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = opt.profile_end() if profile else {}
    opt.close()
    return dict(seconds=t1 - t0, warmup_seconds=per_cycle, stats=stats, profile=prof)


def cpu_baseline(prob, cfg, n_samples):
    from oracle import oracle as O

    x0 = __import__("workloads").uniform_population(2, n_samples, prob.lo, prob.hi)
    c = cfg.with_(N=n_samples)
    run = O.OracleRun(prob, c, x0)
    t = time.perf_counter()
    run.cycle()
    dt = time.perf_counter() - t
    si = n_samples * (c.n_conv + c.n_cloud + c.n_anti)
    return dict(value=si / dt, unit="sample-iterations/s", cores=O.num_threads(), kind="oracle",
                sample=f"d=64, K=128 Gaussian mixture, {n_samples} samples from a uniform start, one non-final "
                       f"cycle with the analytic gradient, FP64: {si} sample-iterations in {dt:.1f} s")


def closed_form_leg(W, steps):
    """The paper's value-only setting on one of its Appendix D functions:
    Michalewicz at d=64 with central-difference gradients (129 evaluations per
    gradient), default schedule.  Throughput at N=65536, and the wall-clock
    of a whole default run (N=200, 3 cycles) as in the paper's timing table."""
    import torch

    from paper_2606_26164_amd.api import Optimizer

    prob = W.closed_form_problem("michalewicz", 64)
    N = 65536
    cfg = W.RunConfig(N=N, m=10, n_osc=1000, n_conv=0, M=10, grad_mode=0, eps_grad=1e-2, seed=11)
    n_conv = max(10, math.ceil(3 * math.log2(prob.d)))  # the default schedule (n_conv=0)
    x0 = W.uniform_population(11, N, prob.lo, prob.hi)
    log(f"closed form: Michalewicz d=64, N={N}, central differences, {steps} cycle(s)")
    r = run_gpu(prob, cfg, x0, 1, steps)
    si = N * (n_conv + cfg.n_cloud + cfg.n_anti) * steps
    prof = r["profile"]
    fdp = prof.get("eval_fd", {})
    out = dict(workload="Michalewicz (Appendix D), d=64, N=65536, central differences (value-only), m=10, "
                        "n_conv=18, n_cloud=3 x M=10 probes, n_anti=5; one step = one cycle",
               ms_per_step=r["seconds"] / steps * 1e3, value=si / r["seconds"], unit="sample-iterations/s",
               cycles=steps,
               fd_eval_points_per_s=(fdp["points"] / (fdp["ms"] * 1e-3)) if fdp.get("ms") else None,
               kernel_ms_per_step={k: round(v["ms"] / steps, 3) for k, v in prof.items() if v["launches"]})
    # a whole run at the paper's defaults: N=200, 3 cycles, handle creation included
    small = cfg.with_(N=200, n_osc=3)
    xs = W.uniform_population(12, 200, prob.lo, prob.hi)
    times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        with Optimizer(prob, small, xs) as opt:
            opt.cycle(3)
            opt.modes()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    out["paper_setting_run"] = dict(N=200, n_osc=3, seconds_median=sorted(times)[2],
                                    note="handle creation, 3 cycles and mode export; the paper's own timing "
                                         "table gives 23.8 s on an RTX 3080 for this function at d=64 (context)")
    log(f"closed form: {out['ms_per_step']:.1f} ms/cycle; N=200 run {out['paper_setting_run']['seconds_median']:.3f} s")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fd-steps", type=int, default=1, help="finite-difference cycles timed (0: skip)")
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--cpu-samples", type=int, default=2048, help="oracle baseline sample size (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=3, help="64-problem batch cycles timed (0: skip)")
    ap.add_argument("--cf-steps", type=int, default=2,
                    help="closed-form (Michalewicz d=64, value-only) cycles timed (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed cycles, copy a buffer of this size once (a reference kernel of known "
                         "traffic for hardware-counter scaling)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2
    import torch

    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"reference copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst
    prob, cfg, x0 = W.gauss128_d64(N=args.N)
    si_per_cycle = cfg.N * (cfg.n_conv + cfg.n_cloud + cfg.n_anti)
    log(f"adjoint: N={cfg.N} d={prob.d} K={prob.K} warmup={args.warmup} steps={args.steps}")
    adj = run_gpu(prob, cfg, x0, args.warmup, args.steps)
    value = si_per_cycle * args.steps / adj["seconds"]
    ms_per_step = adj["seconds"] / args.steps * 1e3
    log(f"adjoint: {ms_per_step:.1f} ms/cycle, {value:.4g} sample-iterations/s")

    fd = None
    if args.fd_steps > 0:
        log(f"finite differences: {args.fd_steps} cycle(s) from the same start")
        r = run_gpu(prob, cfg.with_(grad_mode=0), x0, 0, args.fd_steps, profile=False)
        fd_value = si_per_cycle * args.fd_steps / r["seconds"]
        # adjoint cycle 1 from the same start, for a like-for-like ratio
        adj_first = adj["warmup_seconds"][0] if adj["warmup_seconds"] else None
        fd = dict(value=fd_value, unit="sample-iterations/s", cycles=args.fd_steps,
                  ms_per_step=r["seconds"] / args.fd_steps * 1e3,
                  adjoint_over_fd_first_cycles=(r["seconds"] / args.fd_steps) / adj_first if adj_first else None)
        log(f"fd: {fd['ms_per_step']:.1f} ms/cycle, {fd_value:.4g} sample-iterations/s")

    # roofline of the dominant kernel over the timed cycles
    prof = adj["profile"]
    dom = max((k for k in prof if k.startswith("eval")), key=lambda k: prof[k]["ms"])
    p = prof[dom]
    fpp = eval_flops_per_point(prob.d, prob.K)
    achieved = p["points"] * fpp / (p["ms"] * 1e-3) / 1e12
    traffic = measured_traffic() if dom == "eval_probe" else None
    roof = dict(bound="mfma", achieved=achieved, peak=PEAK_FP32_MFMA_TFLOPS, unit="TFLOP/s",
                frac=achieved / PEAK_FP32_MFMA_TFLOPS, traffic=traffic, traffic_unit="bytes per launch",
                kernel=f"eval_kernel ({dom})",
                launches=p["launches"], avg_launch_ms=p["ms"] / max(p["launches"], 1),
                flops_per_point=fpp, points=p["points"])
    lb = prof.get("lbfgs")
    roof_lbfgs = None
    if lb and lb["ms"] > 0:
        pairs = prof.get("lbfgs_pairs", {}).get("points", 0)
        nbytes = lbfgs_bytes(prob.d, lb["points"], pairs)
        gbs = nbytes / (lb["ms"] * 1e-3) / 1e9
        roof_lbfgs = dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s", frac=gbs / PEAK_HBM_GBS,
                          traffic=None, kernel="lbfgs_step_kernel", bytes_per_launch=nbytes / max(lb["launches"], 1),
                          sample_steps=lb["points"], history_pairs_read=pairs,
                          bytes_per_sample_step_full_history=lbfgs_bytes_per_step(prob.d, cfg.m),
                          launches=lb["launches"], avg_launch_ms=lb["ms"] / max(lb["launches"], 1))
    kernel_ms = {k: round(v["ms"] / args.steps, 3) for k, v in prof.items() if v["launches"]}

    batch = None
    if args.batch_steps > 0:
        items = W.batch64()
        si = sum(c.N * (c.n_conv + c.n_cloud + c.n_anti) for _, c, _ in items)
        from paper_2606_26164_amd.api import Optimizer

        with Optimizer.batched(items) as opt:
            opt.cycle(1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            opt.cycle(args.batch_steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / args.batch_steps
        batch = dict(workload=f"{len(items)} independent problems in one handle (d in 2..64, K in 4..64, "
                              f"N in 1024..16384, {sum(c.N for _, c, _ in items)} samples), adjoint, graph replay",
                     ms_per_step=dt * 1e3, value=si / dt, unit="sample-iterations/s", cycles=args.batch_steps)
        log(f"batch: {dt * 1e3:.1f} ms/cycle, {si / dt:.4g} sample-iterations/s")

    closed = None
    if args.cf_steps > 0:
        closed = closed_form_leg(W, args.cf_steps)

    cpu = None
    if args.cpu_samples > 0:
        log(f"cpu baseline: oracle on {args.cpu_samples} samples")
        cpu = cpu_baseline(prob, cfg, args.cpu_samples)
        log(f"cpu: {cpu['value']:.4g} sample-iterations/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "sample-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"d=64 anisotropic Gaussian mixture, K=128, N={cfg.N}; m=10, n_conv=18, "
                        f"n_cloud=3 x M=16 probes (sigma=0.1), n_anti=5; adjoint gradient; one step = one cycle",
            "N": cfg.N, "d": prob.d, "K": prob.K, "grad": "adjoint",
            "parallelism": "single GPU",
        },
        "fd": fd,
        "batched": batch,
        "closed_form": closed,
        "adjoint_over_fd": (value / fd["value"]) if fd else None,
        "roofline": roof,
        "roofline_lbfgs": roof_lbfgs,
        "kernel_ms_per_step": kernel_ms,
        "cycle_stats_last": adj["stats"][-1] if adj["stats"] else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
