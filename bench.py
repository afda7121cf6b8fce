#!/usr/bin/env python3
"""Benchmark of the explicit 3-D heat-diffusion step on one MI355X.

A bench step is one call of the library's time loop: nt = 100 steps of the
512^3 FP64 bump workload (T0 = Gaussian bump + 0.01*U[0,1], Ci = 0.5*(1+0.5u),
dt by the 6.1 rule; the grid and precision of the paper's Fig. 1 listing).
The headline value is the effective memory throughput
    T_eff = 3 * sizeof(dtype) * nx*ny*nz / t_step      (GB/s, 1e9 bytes)
(read T, read Ci, write T2 per step), with t_step the time of one diffusion
step.  Printed as one JSON line, with the roofline of the step kernel, the
measured copy bandwidth, the reduced-precision forms, the adjoint/forward
time ratio and the oracle timed on the host (CPU baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_step_tbs4_bump512_f64.json")
PASS = 4                        # steps per launch of the FP64 time loop (S-step kernel)
METRIC = "T_eff GB/s (% HBM peak) per 3-D diffusion step; adjoint/forward time ratio"


def kernel_source_hash() -> str:
    csrc = os.path.join(ROOT, "paper_2211_15634_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "diff3d.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def median_ci(xs):
    """Median and an approximate 95% confidence interval of the median
    (order statistics of the binomial(n, 1/2) around n/2)."""
    xs = sorted(xs)
    n = len(xs)
    med = statistics.median(xs)
    if n < 6:
        return med, xs[0], xs[-1]
    k = int(math.floor(n / 2 - 1.96 * math.sqrt(n) / 2))
    j = int(math.ceil(n / 2 + 1.96 * math.sqrt(n) / 2))
    return med, xs[max(k, 0)], xs[min(j, n - 1)]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def large_form(d3, workloads, torch, np, dev, stream, n=1024, nt=500, C=32):
    """1024^3 FP32: T0 ~ U[0,1] (seed 0), Ci = 0.5, T_target ~ U[0,1] (seed 2);
    forward with a checkpoint every C steps, FP64 loss on the GPU, reverse
    sweep.  Returns timings and T_eff of the forward and reverse sweeps."""
    N = n ** 3
    esz = 4
    T0 = torch.from_numpy(workloads.uniform(n, n, n, workloads.SEED_T0).astype(np.float32)).to(dev)
    Ci = torch.full((n, n, n), 0.5, dtype=torch.float32, device=dev)
    s = d3.problem_scalars(Ci)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    ws_bytes = d3.adjoint_workspace_bytes(T0.shape, nt, C, torch.float32)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    T = T0.clone()
    T2 = torch.empty_like(T0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    d3.run(T, T2, Ci, *sc, nt, ckpt=ws, ckpt_every=C)
    ev[1].record(stream)
    Tt = torch.from_numpy(workloads.target(n, n, n).astype(np.float32)).to(dev)
    loss = d3.loss(T, Tt, T2)          # T2 now holds the seed dL/dT_nt
    del Tt
    gT0 = torch.empty_like(T0)
    gCi = torch.empty_like(T0)
    ev[2].record(stream)
    d3.adjoint_run(T0, Ci, T2, gT0, gCi, ws, True, *sc, nt, C)
    ev[3].record(stream)
    torch.cuda.synchronize()
    tf = ev[0].elapsed_time(ev[1]) / 1e3
    tb = ev[2].elapsed_time(ev[3]) / 1e3
    # the same forward in single-step launches (the paper's step)
    d3.set_kernel(d3.KERNEL_ZMARCH)
    T.copy_(T0)
    ev[0].record(stream)
    d3.run(T, T2, Ci, *sc, nt, ckpt=ws, ckpt_every=C)
    ev[1].record(stream)
    torch.cuda.synchronize()
    d3.set_kernel(d3.KERNEL_AUTO)
    tf1 = ev[0].elapsed_time(ev[1]) / 1e3
    nck = (nt + C - 1) // C
    recompute = nt - nck
    gnorm = float(d3.norm2(gT0)) ** 0.5
    finite = bool(torch.isfinite(gT0).all() and torch.isfinite(gCi).all())
    out = {"large_workload": "1024^3 FP32, nt=%d, checkpoint every %d (%d checkpoints), workspace %.1f GB"
                             % (nt, C, nck, ws_bytes / 1e9),
           "large_fwd_s": round(tf, 4), "large_bwd_s": round(tb, 4), "large_ratio": round(tb / tf, 3),
           "large_fwd_single_step_s": round(tf1, 4), "large_ratio_vs_single_step": round(tb / tf1, 3),
           "large_teff_fwd_GBps": round(3 * esz * N * nt / tf / 1e9, 1),
           "large_teff_bwd_GBps": round((3 * recompute + 6 * nt) * esz * N / tb / 1e9, 1),
           "large_loss": float(loss), "large_gradnorm_T0": gnorm, "large_finite": finite}
    del T0, Ci, ws, T, T2, gT0, gCi
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nt", type=int, default=100)
    ap.add_argument("--quick", action="store_true", help="headline only: no precision, adjoint or CPU legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--large", action="store_true",
                    help="also run the 1024^3 FP32 forward + checkpointed adjoint form (nt=500, C=32, ~240 GB)")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only run the 256^3 adjoint form (FP64 and FP32: forward with checkpoints, loss, "
                         "reverse sweep), twice each (for kernel traces)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only launch a 1 GiB copy, the four-step, two-step and single-step kernels, 3 times "
                         "each (for counter runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the 3-D diffusion step on a single MI355X "
              "(no multi-GPU halo exchange); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2211_15634_amd as d3
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, nt = args.n, args.nt
    N = n * n * n

    if args.adjoint_probe:
        m, ntg, C = 256, 200, 14
        for tdt in (torch.float64, torch.float32):
            x, cc = workloads.uniform_const(m, m, m)
            X0 = torch.from_numpy(x).to(dev, tdt)
            Cg = torch.from_numpy(cc).to(dev, tdt)
            Tt = torch.from_numpy(workloads.target(m, m, m)).to(dev, tdt)
            sg = d3.problem_scalars(Cg)
            scg = (sg["lam"], sg["dt"], sg["rdx"], sg["rdy"], sg["rdz"])
            ws = torch.empty(d3.adjoint_workspace_bytes(X0.shape, ntg, C, tdt), dtype=torch.uint8, device=dev)
            Tg, T2g = X0.clone(), torch.empty_like(X0)
            seed, gT0, gCi = torch.empty_like(X0), torch.empty_like(X0), torch.empty_like(X0)
            for _ in range(2):
                Tg.copy_(X0)
                d3.run(Tg, T2g, Cg, *scg, ntg, ckpt=ws, ckpt_every=C)
                d3.loss(Tg, Tt, seed)
                d3.adjoint_run(X0, Cg, seed, gT0, gCi, ws, True, *scg, ntg, C)
            torch.cuda.synchronize()
            del X0, Cg, Tt, ws, Tg, T2g, seed, gT0, gCi
            torch.cuda.empty_cache()
        log("adjoint probe done: 256^3 FP64 and FP32, nt=%d, C=%d, forward + reverse sweep twice each" % (ntg, C))
        return
    if args.traffic_probe:
        # A copy of known size calibrates the FETCH_SIZE / WRITE_SIZE counters;
        # then the forward step kernel on the benchmark workload.
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            d3.copy_(dst, src)
        torch.cuda.synchronize()
        del src, dst
        T0h, Cih = workloads.bump(n, n, n)
        T = torch.from_numpy(T0h).to(dev)
        Ci = torch.from_numpy(Cih).to(dev)
        s = d3.problem_scalars(Ci)
        T2 = T.clone()
        for _ in range(3):
            d3.stepn(T2, T, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"], PASS)
        for _ in range(3):
            d3.step2(T2, T, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
        for _ in range(3):
            d3.step(T2, T, Ci, s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
        torch.cuda.synchronize()
        log("traffic probe done: 3 copies of 1 GiB, 3 %d-step, 3 two-step and 3 single-step launches on bump%d FP64"
            % (PASS, n))
        return
    log("bench: generating bump%d inputs" % n)
    T0h, Cih = workloads.bump(n, n, n)
    T0 = torch.from_numpy(T0h).to(dev)
    Ci = torch.from_numpy(Cih).to(dev)
    s = d3.problem_scalars(Ci)
    T = T0.clone()
    T2 = torch.empty_like(T)
    sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
    stream = torch.cuda.current_stream(dev)

    # ---------------------------------------------------------- headline
    log("bench: warmup %d x run(nt=%d)" % (args.warmup, nt))
    for _ in range(args.warmup):
        d3.run(T, T2, Ci, *sc, nt)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        d3.run(T, T2, Ci, *sc, nt)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_run_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    t_step = ms_per_step / 1e3 / nt
    bytes_step = 3 * 8 * N
    teff = bytes_step / t_step / 1e9
    med, lo, hi = median_ci(per_run_ms)
    if not torch.isfinite(T).all():
        raise RuntimeError("non-finite values after the timed runs")
    log("bench: %.3f ms per run of %d steps, T_eff %.1f GB/s (wall %.3f s)" % (ms_per_step, nt, teff, wall))

    # ---------------------------------------------------------- kernel durations
    # one launch between two events, on the stream it runs on: the S-step
    # kernel (what the time loop runs for FP64), the two-step and the
    # single-step kernels
    def kernel_ms(fn, reps=100, warm=30):
        # the clocks settle over the first tens of launches after an idle gap:
        # launch `warm` unrecorded ones first
        kev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        a, b = T, T2
        for i in range(warm):
            fn(b, a)
            a, b = b, a
        for i in range(reps):
            kev[2 * i].record(stream)
            fn(b, a)
            kev[2 * i + 1].record(stream)
            a, b = b, a
        torch.cuda.synchronize()
        return sum(kev[2 * i].elapsed_time(kev[2 * i + 1]) for i in range(reps)) / reps

    kS_ms = kernel_ms(lambda b, a: d3.stepn(b, a, Ci, *sc, PASS))
    k2_ms = kernel_ms(lambda b, a: d3.step2(b, a, Ci, *sc))
    k1_ms = kernel_ms(lambda b, a: d3.step(b, a, Ci, *sc))
    achieved = PASS * bytes_step / (kS_ms / 1e3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("source_hash") == kernel_source_hash() and tr.get("workload") == "bump%d_f64" % n:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "step_tbs (%d steps per launch)" % PASS, "kernel_avg_us": round(kS_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": PASS * bytes_step,
                "hbm_GBps": round(traffic / (kS_ms / 1e3) / 1e9, 1) if traffic else None}
    single = {"kernel": "step_zmarch (one step per launch)", "kernel_avg_us": round(k1_ms * 1e3, 2),
              "teff_GBps": round(bytes_step / (k1_ms / 1e3) / 1e9, 1)}
    two = {"kernel": "step_tb2 (two steps per launch)", "kernel_avg_us": round(k2_ms * 1e3, 2),
           "teff_GBps": round(2 * bytes_step / (k2_ms / 1e3) / 1e9, 1)}
    log("bench: %d-step kernel %.1f us (%.1f GB/s algorithmic), two-step %.1f us (%.1f GB/s), single-step "
        "kernel %.1f us (%.1f GB/s)" % (PASS, kS_ms * 1e3, achieved, k2_ms * 1e3, two["teff_GBps"], k1_ms * 1e3,
                                        single["teff_GBps"]))

    # ---------------------------------------------------------- copy bandwidth
    del T2
    torch.cuda.empty_cache()
    cb = 4 << 30
    src = torch.empty(cb, dtype=torch.uint8, device=dev)
    dst = torch.empty(cb, dtype=torch.uint8, device=dev)
    src.fill_(1)
    for _ in range(2):
        d3.copy_(dst, src)
    cev = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
    cev[0].record(stream)
    for i in range(10):
        d3.copy_(dst, src)
        cev[i + 1].record(stream)
    torch.cuda.synchronize()
    cms = sorted(cev[i].elapsed_time(cev[i + 1]) for i in range(10))
    copy_gbps = 2 * cb / (statistics.median(cms) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log("bench: copy %.1f GB/s" % copy_gbps)

    extra = {}
    if not args.quick:
        # ------------------------------------------------------ precision forms
        T2 = torch.empty_like(T)
        for name, tdt, rounding in (("f32", torch.float32, "sr"), ("bf16_sr", torch.bfloat16, "sr"),
                                    ("bf16_rne", torch.bfloat16, "rne")):
            Tl = T0.to(tdt)
            T2l = torch.empty_like(Tl)
            Cl = Ci.to(tdt)
            d3.run(Tl, T2l, Cl, *sc, nt, rounding=rounding)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                d3.run(Tl, T2l, Cl, *sc, nt, rounding=rounding)
            e1.record(stream)
            torch.cuda.synchronize()
            ts = e0.elapsed_time(e1) / 3 / 1e3 / nt
            esz = Tl.element_size()
            extra["teff_%s_GBps" % name] = round(3 * esz * N / ts / 1e9, 1)
            extra["t_step_%s_us" % name] = round(ts * 1e6, 2)
            extra["speedup_%s_vs_f64" % name] = round(t_step / ts, 3)
            del Tl, T2l, Cl
        del T2
        torch.cuda.empty_cache()
        log("bench: precision forms", extra)

        # ------------------------------------------------------ 64^3 FP64, nt = 100
        # (the small parity workload: cache-resident and launch-bound, reported,
        # not gated)
        x, cc = workloads.uniform_const(64, 64, 64)
        Ts = torch.from_numpy(x).to(dev, torch.float64)
        Cs = torch.from_numpy(cc).to(dev, torch.float64)
        ss = d3.problem_scalars(Cs)
        scs = (ss["lam"], ss["dt"], ss["rdx"], ss["rdy"], ss["rdz"])
        T2s = torch.empty_like(Ts)
        for _ in range(3):
            d3.run(Ts, T2s, Cs, *scs, 100)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            d3.run(Ts, T2s, Cs, *scs, 100)
        e1.record(stream)
        torch.cuda.synchronize()
        ts = e0.elapsed_time(e1) / 20 / 1e3 / 100
        extra["t_step_uniform64_f64_us"] = round(ts * 1e6, 2)
        extra["teff_uniform64_f64_GBps"] = round(3 * 8 * 64 ** 3 / ts / 1e9, 1)
        del Ts, Cs, T2s
        log("bench: 64^3 FP64 time loop %.2f us per step" % (ts * 1e6))

        # ------------------------------------------------------ 2-D form, 8192^2 FP64, nt = 100
        n2 = 8192
        x2 = np.random.default_rng(0).random((n2, n2))
        T2d = torch.from_numpy(x2).to(dev)
        C2d = torch.full_like(T2d, 0.5)
        dx2 = 1.0 / (n2 - 1)
        sc2 = (1.0, dx2 * dx2 / 1.0 / 0.5 / 4.1, 1.0 / dx2, 1.0 / dx2)
        S2d = torch.empty_like(T2d)
        d3.run2d(T2d, S2d, C2d, *sc2, 10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            d3.run2d(T2d, S2d, C2d, *sc2, 100)
        e1.record(stream)
        torch.cuda.synchronize()
        ts = e0.elapsed_time(e1) / 3 / 1e3 / 100
        extra["t_step_2d_8192_f64_us"] = round(ts * 1e6, 2)
        extra["teff_2d_8192_f64_GBps"] = round(3 * 8 * n2 * n2 / ts / 1e9, 1)
        del T2d, C2d, S2d, x2
        torch.cuda.empty_cache()
        log("bench: 2-D 8192^2 FP64 %.1f us per step" % (ts * 1e6))

        # ------------------------------------------------------ adjoint ratio
        for tdt, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
            m, ntg, C = 256, 200, 14
            x, cc = workloads.uniform_const(m, m, m)
            tt = workloads.target(m, m, m)
            X0 = torch.from_numpy(x).to(dev, tdt)
            Cg = torch.from_numpy(cc).to(dev, tdt)
            Tt = torch.from_numpy(tt).to(dev, tdt)
            sg = d3.problem_scalars(Cg)
            scg = (sg["lam"], sg["dt"], sg["rdx"], sg["rdy"], sg["rdz"])
            ws = torch.empty(d3.adjoint_workspace_bytes(X0.shape, ntg, C, tdt), dtype=torch.uint8, device=dev)
            Tg, T2g = X0.clone(), torch.empty_like(X0)
            seed, gT0, gCi = torch.empty_like(X0), torch.empty_like(X0), torch.empty_like(X0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            for rep in range(2):   # the first repetition warms up
                Tg.copy_(X0)
                ev[0].record(stream)
                d3.run(Tg, T2g, Cg, *scg, ntg, ckpt=ws, ckpt_every=C)
                ev[1].record(stream)
                d3.loss(Tg, Tt, seed)
                ev[2].record(stream)
                d3.adjoint_run(X0, Cg, seed, gT0, gCi, ws, True, *scg, ntg, C)
                ev[3].record(stream)
                torch.cuda.synchronize()
            tf = ev[0].elapsed_time(ev[1])
            tb = ev[2].elapsed_time(ev[3])
            # the same forward with single-step launches (the paper's step)
            d3.set_kernel(d3.KERNEL_ZMARCH)
            Tg.copy_(X0)
            ev[0].record(stream)
            d3.run(Tg, T2g, Cg, *scg, ntg, ckpt=ws, ckpt_every=C)
            ev[1].record(stream)
            torch.cuda.synchronize()
            d3.set_kernel(d3.KERNEL_AUTO)
            tf1 = ev[0].elapsed_time(ev[1])
            extra["adjoint_%s_256_fwd_ms" % tag] = round(tf, 3)
            extra["adjoint_%s_256_fwd_single_step_ms" % tag] = round(tf1, 3)
            extra["adjoint_%s_256_bwd_ms" % tag] = round(tb, 3)
            extra["adjoint_%s_256_ratio" % tag] = round(tb / tf, 3)
            extra["adjoint_%s_256_ratio_vs_single_step" % tag] = round(tb / tf1, 3)
            extra["adjoint_%s_256_gradnorm" % tag] = float(d3.norm2(gT0)) ** 0.5
            del X0, Cg, Tt, ws, Tg, T2g, seed, gT0, gCi
            torch.cuda.empty_cache()
        log("bench: adjoint", {k: v for k, v in extra.items() if k.startswith("adjoint")})

    # ---------------------------------------------------------- large adjoint form
    if args.large:
        del T
        torch.cuda.empty_cache()
        extra.update(large_form(d3, workloads, torch, np, dev, stream))
        log("bench: large form", {k: v for k, v in extra.items() if k.startswith("large")})

    # ---------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu and not args.quick:
        import oracle
        threads = oracle.max_threads()
        # a bounded sample: the oracle on the same 512^3 inputs, k steps, sized
        # from a one-step probe to about --cpu-seconds of work
        # per-step time from two short runs (each also copies its two fields)
        t1 = time.perf_counter()
        oracle.forward(T0h, Cih, *sc, 1)
        t_one = time.perf_counter() - t1
        t1 = time.perf_counter()
        oracle.forward(T0h, Cih, *sc, 3)
        t_three = time.perf_counter() - t1
        per_step = max((t_three - t_one) / 2, 1e-4)
        k = max(1, min(10 * nt, int((args.cpu_seconds - (t_one - per_step)) / per_step)))
        t1 = time.perf_counter()
        oracle.forward(T0h, Cih, *sc, k)
        tc = time.perf_counter() - t1
        cpu_teff = bytes_step * k / tc / 1e9
        # one thread: per-step time from runs of 1 and 2 steps
        t1 = time.perf_counter()
        oracle.forward(T0h, Cih, *sc, 1, threads=1)
        s_one = time.perf_counter() - t1
        t1 = time.perf_counter()
        oracle.forward(T0h, Cih, *sc, 2, threads=1)
        s_step = max(time.perf_counter() - t1 - s_one, 1e-4)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": round(cpu_teff, 2), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": "oracle FP64 forward on the same bump 512^3 inputs, %d step(s) (plus its two "
                         "initial field copies), %.1f s" % (k, tc),
               "t_step_s": round(tc / k, 4), "cpu_model": model,
               "single_thread": {"value": round(bytes_step / s_step / 1e9, 2), "unit": "GB/s",
                                 "t_step_s": round(s_step, 3), "sample": "steps 1 and 2 of the same run"}}
        log("bench: cpu oracle", cpu)

    out = {
        "metric": METRIC,
        "value": round(teff, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "bump%d FP64: 3-D heat diffusion %d^3, nt=%d per step, Gaussian bump + 0.01 U[0,1] "
                               "noise, Ci=0.5(1+0.5u), lam=1, dt=min(dx^2)/lam/max(Ci)/6.1" % (n, n, nt),
                   "nx": n, "ny": n, "nz": n, "nt": nt, "kernel": "four-step passes (temporal blocking over 4 steps)",
                   "parallelism": "single GPU"},
        "t_step_us": round(t_step * 1e6, 3),
        "teff_frac_hbm_peak": round(teff / HBM_PEAK_GBPS, 4),
        "copy_GBps": round(copy_gbps, 1),
        "teff_frac_copy": round(teff / copy_gbps, 4),
        "run_ms_median": round(med, 4),
        "run_ms_ci95": [round(lo, 4), round(hi, 4)],
        "roofline": roofline,
        "two_step": two,
        "single_step": single,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
