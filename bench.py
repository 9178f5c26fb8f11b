#!/usr/bin/env python3
"""Throughput of the ChiSao per-cycle population update on one MI355X.

Workload (the paper's Gaussian-mixture objective, anisotropic, at d=64): 128
components with centres in [-20,20]^64 and covariances Q diag(lam) Q^T
(lam log-uniform in [0.05,1]), N=65536 samples, L-BFGS memory 10, 18 L-BFGS
iterations, 3 smoothing steps of 16 probes at sigma=0.1, 5 anti-convergence
steps.  A step is one (non-final) oscillation cycle: all six phases.

The metric counts sample-iterations nominally: N * (n_conv + n_cloud + n_anti)
per cycle, masked samples included; the active count (samples that actually
took each step) is reported beside it.  `value` is the adjoint-gradient
throughput; the finite-difference throughput on the same schedule and the
ratio between the two are reported beside it.  The timed cycles run as the
library runs them by default, one captured hipGraph replayed per cycle; a few
further cycles are then launched one by one with HIP events around every
launch, which give the roofline position of the dominant kernel (priced
against the published and the measured peaks), the kernel time breakdown and
the active share of the sample-iterations.  Also reported: the
other workloads' throughput (d=16 finite differences, the 64-problem batch,
the noisy Student-t mixture, a closed form), the mode recall of a full run
against the FP64 reference, and the FP64 CPU oracle's throughput on bounded
samples.
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
PEAK_FP32_VECTOR_TFLOPS = 157.3  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_HBM_GBS = 8000.0
ALU_DP = 8  # mixtures with d <= 8 are evaluated on the VALU, one point per lane


def padded_width(d: int) -> int:
    """The launch class's width: 8 for the VALU path, else d padded to 16, 32 or 64."""
    return ALU_DP if d <= ALU_DP else (16 if d <= 16 else (32 if d <= 32 else 64))


def executed_width(d: int) -> int:
    """Coordinates a point's arithmetic runs over: 2, 4 or 8 on the VALU path,
    the padded tile width otherwise."""
    return (2 if d <= 2 else (4 if d <= 4 else 8)) if d <= ALU_DP else padded_width(d)

HERE = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(HERE, "profiles")
COUNTER_SUMMARIES = {
    # kernel -> (summary file, sources its figures were taken from)
    "eval_probe": ("eval_kernel_gauss128_d64_counters.md", ("eval.hip", "common.h", "kernels.h")),
    "lbfgs": ("lbfgs_step_kernel_gauss128_d64_counters.md", ("cycle.hip", "common.h", "kernels.h")),
}


def eval_flops_per_point(d: int, K: int) -> int:
    """Algorithmic flops of one objective (+adjoint) evaluation: per component
    the contraction u = P (x - mu) (2 d^2), the quadratic form delta . u (2 d)
    and the gradient accumulation (2 d)."""
    return K * (2 * d * d + 4 * d)


def lbfgs_bytes_per_step(d: int, m: int) -> int:
    """Algorithmic HBM bytes of one L-BFGS direction + pair update for one
    sample with a full history."""
    return lbfgs_bytes(d, 1, m)


def lbfgs_bytes(d: int, steps: int, pairs: int) -> int:
    """Algorithmic HBM bytes of `steps` L-BFGS sample-steps whose two-loops read
    `pairs` history pairs in total: per step x, x_prev, g, g_prev read (4d), the
    new pair written (2d + 1) and the direction written (d); per pair s, y and
    rho read (2d + 1)."""
    return 4 * (steps * (7 * d + 1) + pairs * (2 * d + 1))


def source_digest(files) -> str:
    """Digest of kernel sources, comments and blank space removed: hardware
    counter figures are only used while the kernel is the one they were
    taken from."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "paper_2606_26164_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update("\n".join(ln.strip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of a kernel from its committed counter summary, or
    None when absent or taken from a different kernel source."""
    if kernel not in COUNTER_SUMMARIES:
        return None
    name, files = COUNTER_SUMMARIES[kernel]
    try:
        text = open(os.path.join(PROFILES, name)).read()
    except OSError:
        return None
    vals = dict(ln.split(": ", 1) for ln in text.splitlines() if ln.startswith(("traffic_bytes", "source_sha256")))
    if vals.get("source_sha256", "").strip() != source_digest(files):
        return None
    return int(vals["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(model=model, nproc=usable, cpu_count=os.cpu_count())


def measure_peaks(copy_gib: int = 4):
    import ctypes as C

    import torch

    from paper_2606_26164_amd import _lib as L

    lib = L.load()
    out = L.Peaks()
    L.check(lib.chisao_measure_peaks(C.byref(out), copy_gib << 30, torch.cuda.current_stream().cuda_stream),
            "chisao_measure_peaks")
    return dict(fp32_mfma_tflops=out.fp32_mfma_tflops, hbm_copy_gbs=out.hbm_copy_gbs,
                mfma_kernel_ms=out.mfma_ms, copy_kernel_ms=out.copy_ms, copy_bytes=out.copy_bytes,
                note="v_mfma_f32_16x16x4f32 on independent accumulators over a full grid; a streaming copy of "
                     f"{copy_gib} GiB (read + write bytes over time); best of several repetitions")


def run_gpu(items, warmup, steps, profile_steps=0):
    """Warm-up cycles, then `steps` timed cycles as the library runs them by
    default (one captured hipGraph replayed per cycle), then `profile_steps`
    further cycles launched one by one with HIP events around every launch
    (kernel times, evaluation counts, cycle statistics).  items: [(problem,
    config, x0)]; one handle for all of them."""
    import torch

    from paper_2606_26164_amd.api import Optimizer

    opt = Optimizer.batched(items)
    per_cycle = []
    for i in range(warmup):
        torch.cuda.synchronize()
        t = time.perf_counter()
        opt.cycle(1)
        torch.cuda.synchronize()
        per_cycle.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if steps > 0:
        opt.cycle(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats, prof, tp = [], {}, 0.0
    if profile_steps > 0:
        opt.profile_begin()
        t2 = time.perf_counter()
        stats = opt.cycle(profile_steps, stats=True)
        tp = time.perf_counter() - t2
        prof = opt.profile_end()
    opt.close()
    if len(items) == 1:
        stats = [[s] for s in stats]
    return dict(seconds=t1 - t0, warmup_seconds=per_cycle, stats=stats, profile=prof, profile_seconds=tp,
                profile_steps=profile_steps)


def nominal_si(items, last=False):
    return sum(c.N * (c.n_conv + (0 if last else c.n_cloud + c.n_anti)) for _, c, _ in items)


def active_fraction(items, r):
    """Share of the nominal sample-iterations of the profiled cycles that the
    samples actually took: L-BFGS steppers (counted on the device) plus the
    unfrozen samples of every smoothing and anti-convergence step."""
    lb = r["profile"].get("lbfgs", {}).get("points", 0)
    expl = 0
    for cyc in r["stats"]:
        for (_, c, _), s in zip(items, cyc):
            expl += s["n_unfrozen"] * (c.n_cloud + c.n_anti)
    return (lb + expl) / (nominal_si(items) * max(r["profile_steps"], 1))


def eval_roofline(items, r, peaks, dominant_only=True):
    """Roofline of the evaluation launches over the profiled cycles.  With one
    problem the dominant launch kind (by time); otherwise all evaluation
    launches of the handle, with the problems' own evaluation counts."""
    prof = r["profile"]
    if dominant_only:
        prob = items[0][0]
        dom = max((k for k in prof if k.startswith("eval") and prof[k]["ms"] > 0), key=lambda k: prof[k]["ms"])
        p = prof[dom]
        fpp = eval_flops_per_point(prob.d, prob.K)
        flops, ms, launches = p["points"] * fpp, p["ms"], p["launches"]
        kernel, traffic = f"eval_kernel ({dom})", (measured_traffic(dom) if prob.d == 64 and prob.K == 128 else None)
        extra = dict(flops_per_point=fpp, points=p["points"])
    else:
        flops = padded = 0
        for cyc in r["stats"]:
            for (prob, _, _), s in zip(items, cyc):
                flops += s["evals"] * eval_flops_per_point(prob.d, prob.K)
                padded += s["evals"] * eval_flops_per_point(executed_width(prob.d), prob.K)
        ev = [k for k in prof if k.startswith("eval")]
        ms = sum(prof[k]["ms"] for k in ev)
        launches = sum(prof[k]["launches"] for k in ev)
        kernel, traffic = "eval_kernel (all launch kinds)", None
        extra = dict(achieved_padded=padded / (ms * 1e-3) / 1e12,
                     note="achieved counts each problem's own d; achieved_padded the work at the width the "
                          "kernel executes (tiles padded to 16, 32 or 64; 2, 4 or 8 on the VALU path)")
    achieved = flops / (ms * 1e-3) / 1e12
    # mixtures with d <= 8 run on the VALU, the rest on the FP32 matrix cores
    alu = all(padded_width(prob.d) == ALU_DP for prob, _, _ in items)
    peak = PEAK_FP32_VECTOR_TFLOPS if alu else PEAK_FP32_MFMA_TFLOPS
    out = dict(bound="alu" if alu else "mfma", achieved=achieved, peak=peak, unit="TFLOP/s",
               frac=achieved / peak, traffic=traffic, traffic_unit="bytes per launch",
               kernel=kernel, launches=launches, avg_launch_ms=ms / max(launches, 1))
    if peaks and not alu:
        out.update(peak_measured=peaks["fp32_mfma_tflops"], frac_measured=achieved / peaks["fp32_mfma_tflops"])
    if alu:
        # the vector peak counts packed FP32 (two lanes' worth per instruction);
        # the kernels are compiled without packed FP32, so one FMA per lane per
        # instruction is the reachable rate
        out.update(peak_nonpacked=PEAK_FP32_VECTOR_TFLOPS / 2, frac_nonpacked=achieved / (PEAK_FP32_VECTOR_TFLOPS / 2))
    out.update(extra)
    return out


def cycle_roofline(prob, r, peaks):
    """Every objective evaluation of the profiled cycles (their evaluation
    counts times the algorithmic flops per point) over those cycles' wall time
    (launched one by one with events, a little slower than graph replay)."""
    n = r["profile_steps"]
    if n <= 0 or r["profile_seconds"] <= 0:
        return None
    evals = sum(s["evals"] for cyc in r["stats"] for s in cyc)
    flops = evals * eval_flops_per_point(prob.d, prob.K)
    achieved = flops / r["profile_seconds"] / 1e12
    out = dict(bound="mfma", achieved=achieved, peak=PEAK_FP32_MFMA_TFLOPS, unit="TFLOP/s",
               frac=achieved / PEAK_FP32_MFMA_TFLOPS, evaluations_per_cycle=evals / n,
               ms_per_cycle=r["profile_seconds"] / n * 1e3,
               note="every objective evaluation a cycle performs (samples, line-search trials including the "
                    "speculative ones, smoothing probes) at K(2d^2+4d) flops each, over the whole cycle's time")
    if peaks:
        out.update(peak_measured=peaks["fp32_mfma_tflops"], frac_measured=achieved / peaks["fp32_mfma_tflops"])
    return out


def lbfgs_roofline(prob, cfg, r, peaks):
    lb = r["profile"].get("lbfgs")
    if not lb or lb["ms"] <= 0:
        return None
    pairs = r["profile"].get("lbfgs_pairs", {}).get("points", 0)
    nbytes = lbfgs_bytes(prob.d, lb["points"], pairs)
    gbs = nbytes / (lb["ms"] * 1e-3) / 1e9
    out = dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s", frac=gbs / PEAK_HBM_GBS,
               traffic=measured_traffic("lbfgs"), traffic_unit="bytes per launch", kernel="lbfgs_step_kernel",
               bytes_per_launch=nbytes / max(lb["launches"], 1), sample_steps=lb["points"],
               history_pairs_read=pairs, bytes_per_sample_step_full_history=lbfgs_bytes_per_step(prob.d, cfg.m),
               launches=lb["launches"], avg_launch_ms=lb["ms"] / max(lb["launches"], 1))
    if peaks:
        out.update(peak_measured=peaks["hbm_copy_gbs"], frac_measured=gbs / peaks["hbm_copy_gbs"])
    return out


def workload_line(name, items, warmup, steps, peaks, roofline=True):
    log(f"{name}: {len(items)} problem(s), {sum(c.N for _, c, _ in items)} samples, {steps} timed cycle(s)")
    r = run_gpu(items, warmup, steps, profile_steps=steps)
    si = nominal_si(items) * steps
    out = dict(workload=name, ms_per_step=r["seconds"] / steps * 1e3, value=si / r["seconds"],
               active_value=si / r["seconds"] * active_fraction(items, r), unit="sample-iterations/s", cycles=steps,
               kernel_ms_per_step={k: round(v["ms"] / steps, 3) for k, v in r["profile"].items() if v["launches"]})
    if roofline:
        out["roofline"] = eval_roofline(items, r, peaks, dominant_only=len(items) == 1)
    log(f"{name}: {out['ms_per_step']:.1f} ms/cycle, {out['value']:.4g} sample-iterations/s")
    return out


def batch_class_lines(W, peaks, steps):
    """The 64-problem batch by evaluation launch class (width 8 on the VALU,
    16, 32, 64 on the matrix cores): each class's problems in a handle of their
    own (a class's launches are the same launches in the full batch), so each
    class gets its own roofline."""
    items = W.batch64()
    out = {}
    for dp in (ALU_DP, 16, 32, 64):
        sub = [it for it in items if padded_width(it[0].d) == dp]
        if sub:
            out[f"padded_d{dp}"] = workload_line(f"batch class padded d={dp} ({len(sub)} problems)", sub, 1, steps,
                                                 peaks)
    return out


# ---------------------------------------------------------------------------
# The oracle leg: CPU baseline and the recall scoring against the FP64
# reference.  The only part of this script that uses the oracle.
# ---------------------------------------------------------------------------
def _match(X, Xref, radius):
    """One-to-one L-inf matching within `radius` (greedy by distance)."""
    import numpy as np

    if len(X) == 0 or len(Xref) == 0:
        return 0
    D = np.abs(X[:, None, :] - Xref[None, :, :]).max(2)
    used_a, used_b, n = set(), set(), 0
    for flat in np.argsort(D, axis=None):
        a, b = divmod(int(flat), D.shape[1])
        if D[a, b] >= radius:
            break
        if a not in used_a and b not in used_b:
            used_a.add(a)
            used_b.add(b)
            n += 1
    return n


def oracle_leg(prob, cfg, W, args, full_modes):
    import numpy as np

    from oracle import oracle as O
    from oracle.modes import newton_modes, value_grad_hess

    out = {}
    cpu = host_cpu()
    n_all = O.num_threads()

    def timed_cycle(c, x0, threads):
        O.set_num_threads(threads)
        run = O.OracleRun(prob, c, x0)
        t = time.perf_counter()
        run.cycle()
        return time.perf_counter() - t

    si_per = cfg.n_conv + cfg.n_cloud + cfg.n_anti
    n = args.cpu_samples
    x0 = W.uniform_population(2, n, prob.lo, prob.hi)
    dt = timed_cycle(cfg.with_(N=n), x0, n_all)
    log(f"cpu baseline: {n} samples, {n_all} threads, {dt:.1f} s")
    base = dict(value=n * si_per / dt, unit="sample-iterations/s", cores=n_all, kind="oracle",
                sample=f"d=64, K=128 Gaussian mixture, {n} samples from a uniform start, one non-final cycle with "
                       f"the analytic gradient, FP64: {n * si_per} sample-iterations in {dt:.1f} s",
                host=cpu)
    n1 = max(16, n // 8)
    dt1 = timed_cycle(cfg.with_(N=n1), x0[:n1], 1)
    base["one_thread"] = dict(value=n1 * si_per / dt1, samples=n1, seconds=dt1)
    nf = args.cpu_fd_samples
    if nf > 0:
        dtf = timed_cycle(cfg.with_(N=nf, grad_mode=0), x0[:nf], n_all)
        base["fd"] = dict(value=nf * si_per / dtf, samples=nf, seconds=dtf, threads=n_all,
                          note="central differences (129 evaluations per gradient), one non-final cycle")
    O.set_num_threads(n_all)
    out["cpu_baseline"] = base

    if full_modes is None:
        return out
    # recall of the full run against the Newton-refined reference set (FP64)
    t = time.perf_counter()
    Xall, Fall = newton_modes(prob, log_delta=None)
    keep = Fall >= Fall.max() + cfg.log_delta
    X = full_modes.X.astype(np.float64)
    tol = []
    for x in Xall:
        _, _, H = value_grad_hess(prob, x)
        tol.append(max(1e-4, 2.0 * np.abs(np.linalg.inv(H)).sum(1).max() * cfg.eps_grad))
    tol = np.array(tol)
    owner = [int(np.argmin(np.abs(Xall - x).max(1))) for x in X]
    is_max = [np.abs(Xall[j] - x).max() < tol[j] for j, x in zip(owner, X)]
    hit_sig = {j for j, ok in zip(owner, is_max) if ok and keep[j]}
    f_best = float(full_modes.F.max()) if len(full_modes.F) else -np.inf
    band = (Fall >= f_best + cfg.log_delta - 1e-4) & (Fall <= f_best + 1e-4)
    hit_band = {j for j, ok in zip(owner, is_max) if ok and band[j]}
    rec = dict(value=len(hit_sig) / max(int(keep.sum()), 1), significant_modes=int(keep.sum()),
               significant_recovered=len(hit_sig), recovered_points=len(X), points_not_a_maximum=int(sum(
                   not v for v in is_max)), maxima_in_gate_of_best_found=int(band.sum()),
               maxima_in_gate_recovered=len(hit_band), cycles=cfg.n_osc, N=cfg.N,
               note="significant set: Newton ascent from every centre, negative-definite Hessian, gate "
                    "f >= max f + log delta over all local maxima (Sec. 3.1, eq. 1)")
    log(f"recall: {rec['significant_recovered']}/{rec['significant_modes']} significant, "
        f"{rec['maxima_in_gate_recovered']}/{rec['maxima_in_gate_of_best_found']} in the gate of the best found "
        f"({time.perf_counter() - t:.1f} s)")
    out["recall"] = rec

    # GPU against the oracle cycle by cycle at a population the host affords
    from paper_2606_26164_amd.api import Optimizer

    Nr, nc = args.recall_oracle_N, args.recall_oracle_cycles
    if Nr > 0 and nc > 0:
        p2, c2, xr = W.gauss128_d64(N=Nr, n_osc=nc)
        run = O.OracleRun(p2, c2, xr)
        per = []
        with Optimizer(p2, c2, xr) as opt:
            for k in range(nc):
                run.cycle()
                opt.cycle(1)
                Xo, _, _ = run.modes()
                mg = opt.modes().X.astype(np.float64)
                per.append(dict(cycle=k + 1, gpu=len(mg), oracle=len(Xo), matched=_match(mg, Xo, 1e-3)))
        out["oracle_mode_sets"] = dict(N=Nr, per_cycle=per,
                                       note="GPU run and FP64 oracle run from the same start and random "
                                            "streams; modes matched one-to-one within L-inf 1e-3")
        log(f"oracle mode sets at N={Nr}: {per}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--profile-steps", type=int, default=5,
                    help="cycles after the timed ones, launched one by one with HIP events (kernel times, rooflines)")
    ap.add_argument("--fd-steps", type=int, default=1, help="finite-difference cycles timed (0: skip)")
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--cpu-samples", type=int, default=2048, help="oracle baseline sample size (0: skip the oracle leg)")
    ap.add_argument("--cpu-fd-samples", type=int, default=48, help="oracle finite-difference sample size (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=3, help="64-problem batch cycles timed (0: skip)")
    ap.add_argument("--other-steps", type=int, default=3,
                    help="cycles timed for the d=16 finite-difference, Student-t and closed-form workloads (0: skip)")
    ap.add_argument("--recall-cycles", type=int, default=300, help="cycles of the full run scored for recall (0: skip)")
    ap.add_argument("--recall-oracle-N", type=int, default=2048)
    ap.add_argument("--recall-oracle-cycles", type=int, default=4)
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured-peak kernels")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the timed cycles, copy a buffer of this size once (a reference kernel of known "
                         "traffic for hardware-counter scaling)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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
    peaks = None if args.no_peaks else measure_peaks()
    if peaks:
        log(f"measured peaks: {peaks['fp32_mfma_tflops']:.1f} TFLOP/s FP32 MFMA, {peaks['hbm_copy_gbs']:.0f} GB/s copy")

    prob, cfg, x0 = W.gauss128_d64(N=args.N)
    items = [(prob, cfg, x0)]
    si_per_cycle = nominal_si(items)
    log(f"adjoint: N={cfg.N} d={prob.d} K={prob.K} warmup={args.warmup} steps={args.steps}")
    adj = run_gpu(items, args.warmup, args.steps, profile_steps=args.profile_steps)
    value = si_per_cycle * args.steps / adj["seconds"]
    ms_per_step = adj["seconds"] / args.steps * 1e3
    active = value * active_fraction(items, adj)
    log(f"adjoint: {ms_per_step:.1f} ms/cycle, {value:.4g} sample-iterations/s ({active:.4g} active)")

    fd = None
    if args.fd_steps > 0:
        log(f"finite differences: {args.fd_steps} cycle(s) from the same start")
        fitems = [(prob, cfg.with_(grad_mode=0), x0)]
        r = run_gpu(fitems, 0, args.fd_steps)
        fd_value = si_per_cycle * args.fd_steps / r["seconds"]
        adj_first = adj["warmup_seconds"][0] if adj["warmup_seconds"] else None
        fd = dict(value=fd_value, unit="sample-iterations/s", cycles=args.fd_steps,
                  ms_per_step=r["seconds"] / args.fd_steps * 1e3,
                  adjoint_over_fd_first_cycles=(r["seconds"] / args.fd_steps) / adj_first if adj_first else None)
        log(f"fd: {fd['ms_per_step']:.1f} ms/cycle, {fd_value:.4g} sample-iterations/s")

    roof = eval_roofline(items, adj, peaks)
    roof_lbfgs = lbfgs_roofline(prob, cfg, adj, peaks)
    cycle_roof = cycle_roofline(prob, adj, peaks)
    kernel_ms = {k: round(v["ms"] / args.profile_steps, 3) for k, v in adj["profile"].items() if v["launches"]}

    others = {}
    if args.batch_steps > 0:
        from paper_2606_26164_amd.api import Optimizer

        bitems = W.batch64()
        si = nominal_si(bitems)
        with Optimizer.batched(bitems) as opt:
            opt.cycle(1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            opt.cycle(args.batch_steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / args.batch_steps
        others["batched"] = dict(
            workload=f"{len(bitems)} independent problems in one handle (d in 2..64, K in 4..64, N in "
                     f"1024..16384, {sum(c.N for _, c, _ in bitems)} samples), adjoint, graph replay",
            ms_per_step=dt * 1e3, value=si / dt, unit="sample-iterations/s", cycles=args.batch_steps)
        log(f"batch: {dt * 1e3:.1f} ms/cycle, {si / dt:.4g} sample-iterations/s")
        others["batched"]["classes"] = batch_class_lines(W, peaks, args.batch_steps)
    if args.other_steps > 0:
        p2, c2, x2 = W.gauss32_d16()
        others["gauss32_d16_fd"] = workload_line(
            "d=16 anisotropic Gaussian mixture, K=32, N=16384, central differences (33 evaluations per gradient), "
            "m=8, n_conv=12", [(p2, c2, x2)], 1, args.other_steps, peaks)
        p5, c5, x5 = W.student48_d32()
        others["student48_d32_noisy"] = workload_line(
            "d=32 Student-t mixture (nu=3), K=48, N=131072, unit evaluation noise, M=32 probes at sigma=0.2, gate "
            "over 32 draws, adjoint gradient", [(p5, c5, x5)], 1, args.other_steps, peaks)
        pc = W.closed_form_problem("michalewicz", 64)
        cc = W.RunConfig(N=65536, m=10, n_osc=1000, n_conv=0, M=10, grad_mode=0, eps_grad=1e-2, seed=11)
        cc = cc.with_(n_conv=max(10, math.ceil(3 * math.log2(pc.d))))
        others["closed_form"] = workload_line(
            "Michalewicz (Appendix D), d=64, N=65536, central differences (value-only), m=10, n_conv=18, n_cloud=3 "
            "x M=10 probes, n_anti=5", [(pc, cc, W.uniform_population(11, 65536, pc.lo, pc.hi))], 1,
            args.other_steps, peaks, roofline=False)

    full_modes = None
    if args.recall_cycles > 0 and args.cpu_samples > 0:
        from paper_2606_26164_amd.api import Optimizer

        rc = cfg.with_(n_osc=args.recall_cycles)
        t = time.perf_counter()
        with Optimizer(prob, rc, x0) as opt:
            opt.cycle(rc.n_osc)
            full_modes = opt.modes()
        log(f"full run: {rc.n_osc} cycles in {time.perf_counter() - t:.1f} s, {len(full_modes.F)} modes")
        cfg_full = rc
    else:
        cfg_full = cfg
    ol = oracle_leg(prob, cfg_full, W, args, full_modes) if args.cpu_samples > 0 else {}

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
        "active_value": active,
        "fd": fd,
        "adjoint_over_fd": (value / fd["value"]) if fd else None,
        "roofline": roof,
        "roofline_lbfgs": roof_lbfgs,
        "roofline_cycle": cycle_roof,
        "peaks_measured": peaks,
        "kernel_ms_per_step": kernel_ms,
        "recall": ol.get("recall"),
        "oracle_mode_sets": ol.get("oracle_mode_sets"),
        "cycle_stats_last": adj["stats"][-1][0] if adj["stats"] else None,
        "cpu_baseline": ol.get("cpu_baseline"),
    }
    out.update(others)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
