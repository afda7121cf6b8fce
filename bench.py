#!/usr/bin/env python3
"""Benchmark of the explicit 3-D heat-diffusion step on one MI355X.

A bench step is one call of the library's time loop: nt = 100 steps of the
512^3 FP64 bump workload (T0 = Gaussian bump + 0.01*U[0,1], Ci = 0.5*(1+0.5u),
dt by the 6.1 rule; the grid and precision of the paper's Fig. 1 listing).
The headline value is the effective memory throughput
    T_eff = 3 * sizeof(dtype) * nx*ny*nz / t_step      (GB/s, 1e9 bytes)
(read T, read Ci, write T2 per step), with t_step the time of one diffusion
step.  Printed as one JSON line, with the roofline of the time loop's kernel,
the measured copy bandwidth, the reduced-precision forms with their errors,
the adjoint/forward time ratio at 256^3 and 1024^3, and the oracle timed on
the host (CPU baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick] [--no-large]

Profiling helpers (rocprofv3 runs them; see the files under profiles/):
    --traffic-probe {f64,bf16_sr}   launch a 1 GiB copy and the time loop's kernels three times each
    --adjoint-probe                 the 256^3 forward + reverse sweep, twice per dtype
    --summarize-traffic / --summarize-trace   turn rocprofv3 output into the profiles/ summaries
"""
from __future__ import annotations

import argparse
import glob
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
FP64_VECTOR_OPS_PEAK = 39.3     # Top/s: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz (add or multiply)
ALU_OPS_PER_POINT_STEP = 18     # the step's FP operations per interior point: Laplacian 14, update 4
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "traffic_step_tbs4_bump512_f64.json")
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


# ------------------------------------------------------------------ profiles
# rocprofv3 writes its results as an SQLite database (<dir>/<name>_results.db);
# these helpers read the per-dispatch counters and the kernel statistics
# from it and write the short summaries kept under profiles/.
def _db_rows(d, query):
    import sqlite3
    out = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)):
        con = sqlite3.connect(path)
        try:
            out += list(con.execute(query))
        finally:
            con.close()
    return out


def _counters(d):
    """{counter: [(dispatch id, kernel name, value), ...]} in dispatch order."""
    out = {}
    for disp, name, counter, value in _db_rows(
            d, "select dispatch_id, kernel_name, counter_name, value from counters_collection order by dispatch_id"):
        out.setdefault(counter, []).append((disp, name, float(value)))
    return out


def summarize_traffic(fetch_dir, write_dir, kernel, steps, workload, nbytes_alg, out_prefix, command,
                      calibration=None, note="read T and Ci, write T2 once", max_rows=8):
    """FETCH_SIZE / WRITE_SIZE per dispatch (KiB) from two rocprofv3 --pmc runs
    of --traffic-probe, scaled by what each counter reads for the 1 GiB copy
    launched first (or in the runs named by `calibration`); writes
    <out_prefix>.json and .md."""
    fetch = _counters(fetch_dir)["FETCH_SIZE"]
    write = _counters(write_dir)["WRITE_SIZE"]
    cfd, cwd = calibration or (fetch_dir, write_dir)
    cf = [v for _, n, v in _counters(cfd)["FETCH_SIZE"] if "copy16" in n]
    cw = [v for _, n, v in _counters(cwd)["WRITE_SIZE"] if "copy16" in n]
    kf = [v for _, n, v in fetch if kernel in n]
    kw = [v for _, n, v in write if kernel in n]
    kname = next(n for _, n, _ in fetch if kernel in n).split("(")[0]
    gib_kib = 1024.0 * 1024.0
    fs = statistics.median(cf) / gib_kib
    ws = statistics.median(cw) / gib_kib
    fb = statistics.median(kf) * 1024 / fs
    wb = statistics.median(kw) * 1024 / ws
    rec = {"kernel": kname, "workload": workload, "steps_per_launch": steps, "source_hash": kernel_source_hash(),
           "fetch_size_kib_per_dispatch": kf, "write_size_kib_per_dispatch": kw,
           "copy_1GiB_fetch_size_kib": cf, "copy_1GiB_write_size_kib": cw,
           "fetch_scale": round(fs, 5), "write_scale": round(ws, 5),
           "fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
           "bytes_per_launch": int(fb + wb), "compulsory_bytes_per_launch": int(nbytes_alg),
           "hbm_bytes_per_step": int((fb + wb) / steps)}
    with open(out_prefix + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# HBM traffic of `%s`, %s" % (kname, workload), "",
             "One launch advances %d time step(s).  Compulsory bytes per launch (%s): "
             "%d B." % (steps, note, nbytes_alg), "", "Commands (repository root, one MI355X):", "", "```", command,
             "```", "", "| dispatch | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) |", "|---|---|---|"]
    for i, (x, y) in enumerate(zip(cf, cw)):
        lines.append("| copy16, 1 GiB, #%d | %.1f | %.1f |" % (i + 1, x, y))
    for i, (x, y) in enumerate(zip(kf, kw)):
        if i == max_rows:
            lines.append("| ... %d more dispatches | | |" % (len(kf) - max_rows))
            break
        lines.append("| kernel #%d | %.1f | %.1f |" % (i + 1, x, y))
    lines += ["", "Calibration with the copy of known size (1 GiB read and written): FETCH_SIZE reports %.5f of "
              "the bytes read, WRITE_SIZE %.5f of the bytes written.  Scaled, per launch (median):" % (fs, ws), "",
              "- fetched %.4f GB, written %.4f GB, total %.4f GB (%.3f x the compulsory bytes)" %
              (fb / 1e9, wb / 1e9, (fb + wb) / 1e9, (fb + wb) / nbytes_alg),
              "- per time step %.4f GB" % ((fb + wb) / steps / 1e9), ""]
    with open(out_prefix + ".md", "w") as f:
        f.write("\n".join(lines))
    print(json.dumps(rec))


def summarize_trace(trace_dir, out_md, command, top=14, title="", note=""):
    rows = _db_rows(trace_dir, "select name, total_calls, total_duration, average, percentage from top_kernels")
    lines = ["# rocprofv3 kernel trace summary" + (": " + title if title else ""), ""]
    if note:
        lines += [note, ""]
    lines += ["Command (repository root, one MI355X):", "", "```", command,
              "```", "", "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    rows.sort(key=lambda r: -float(r[2]))
    for name, calls, total, avg, pct in rows[:top]:
        lines.append("| `%s` | %s | %.1f | %.2f | %.2f |" % (name.split("(")[0][:120], calls, float(total),
                                                            float(avg), float(pct)))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_sq(dir1, dir2, kernel, title, out_md, command):
    """Shader-sequencer counters of the third dispatch of `kernel` from two
    rocprofv3 --pmc runs, with the derived issue and wait fractions."""
    vals = {}
    for d in (dir1, dir2):
        for counter, rows in _counters(d).items():
            ks = [v for _, n, v in rows if kernel in n]
            if ks:
                vals[counter] = ks[min(2, len(ks) - 1)]
    g = lambda c: vals.get(c, float("nan"))
    lines = ["# Shader-sequencer counters, %s" % title, "", "Commands (repository root, one MI355X):", "", "```",
             command, "```", "", "| counter | value |", "|---|---|"]
    for c in sorted(vals):
        lines.append("| %s | %.4g |" % (c, vals[c]))
    lines += ["| SQ_WAIT_ANY / SQ_WAVE_CYCLES | %.3f |" % (g("SQ_WAIT_ANY") / g("SQ_WAVE_CYCLES")),
              "| SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES | %.3f |" % (g("SQ_ACTIVE_INST_ANY") / g("SQ_WAVE_CYCLES")),
              "| SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES | %.3f |" % (g("SQ_ACTIVE_INST_VALU") / g("SQ_WAVE_CYCLES")),
              "| SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES | %.3f |" % (g("SQ_WAIT_INST_LDS") / g("SQ_WAVE_CYCLES")),
              "| SQ_INSTS_SALU / SQ_INSTS_VALU | %.3f |" % (g("SQ_INSTS_SALU") / g("SQ_INSTS_VALU")), ""]
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


# ------------------------------------------------------------------ legs
def max_rel_dev(a, b, torch):
    """max_i |a_i - b_i| / |b_i| over the whole grid, computed on the GPU."""
    a = a.to(torch.float64)
    return float(((a - b).abs() / b.abs().clamp_min(1e-300)).max())


def large_form(d3, workloads, torch, np, dev, stream, n=1024, nt=500, C=32):
    """1024^3 FP32: T0 ~ U[0,1] (seed 0), Ci = 0.5, T_target ~ U[0,1] (seed 2);
    forward with a checkpoint every C steps, FP64 loss on the GPU, reverse
    sweep.  Returns timings, T_eff of both sweeps and their ratio."""
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
    Tt = torch.from_numpy(workloads.target(n, n, n).astype(np.float32)).to(dev)
    gT0 = torch.empty_like(T0)
    gCi = torch.empty_like(T0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    tfs, tbs = [], []
    for rep in range(4):   # the first repetition warms up; the median of the other three
        T.copy_(T0)
        torch.cuda.synchronize()
        ev[0].record(stream)
        d3.run(T, T2, Ci, *sc, nt, ckpt=ws, ckpt_every=C)
        ev[1].record(stream)
        loss = d3.loss(T, Tt, T2)          # T2 now holds the seed dL/dT_nt
        ev[2].record(stream)
        d3.adjoint_run(T0, Ci, T2, gT0, gCi, ws, True, *sc, nt, C)
        ev[3].record(stream)
        torch.cuda.synchronize()
        log("bench: large form repetition %d: forward %.3f s, reverse %.3f s" %
            (rep, ev[0].elapsed_time(ev[1]) / 1e3, ev[2].elapsed_time(ev[3]) / 1e3))
        if rep:
            tfs.append(ev[0].elapsed_time(ev[1]) / 1e3)
            tbs.append(ev[2].elapsed_time(ev[3]) / 1e3)
    tf = statistics.median(tfs)
    tb = statistics.median(tbs)
    nck = (nt + C - 1) // C
    gnorm = float(d3.norm2(gT0)) ** 0.5
    finite = bool(torch.isfinite(gT0).all() and torch.isfinite(gCi).all())
    out = {"large_workload": "1024^3 FP32, nt=%d, checkpoint every %d (%d checkpoints), workspace %.1f GB"
                             % (nt, C, nck, ws_bytes / 1e9),
           "large_fwd_s": round(tf, 4), "large_bwd_s": round(tb, 4), "large_ratio": round(tb / tf, 3),
           "large_teff_fwd_GBps": round(3 * esz * N * nt / tf / 1e9, 1),
           "large_teff_bwd_GBps": round(6 * esz * N * nt / tb / 1e9, 1),
           "large_loss": float(loss), "large_gradnorm_T0": gnorm, "large_finite": finite}
    del T0, Ci, ws, T, T2, gT0, gCi, Tt
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--nt", type=int, default=100)
    ap.add_argument("--quick", action="store_true", help="headline only: no precision, adjoint, large or CPU legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 FP32 forward + adjoint form")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only run the 256^3 adjoint form (FP64 and FP32: forward with checkpoints, loss, "
                         "reverse sweep), twice each (for kernel traces)")
    ap.add_argument("--traffic-probe", choices=["f64", "bf16_sr"], default=None,
                    help="only launch a 1 GiB copy, then the time loop's kernels for this form, 3 times each "
                         "(for counter runs)")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("SQ1_DIR", "SQ2_DIR"))
    ap.add_argument("--title", default="")
    ap.add_argument("--kernel", default="step_tbs<0, 4")
    ap.add_argument("--workload", default="bump512_f64")
    ap.add_argument("--steps-per-launch", type=int, default=4)
    ap.add_argument("--compulsory-bytes", type=float, default=3 * 8 * 512 ** 3)
    ap.add_argument("--calibration", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="counter runs holding the 1 GiB copy (default: the summarized runs)")
    ap.add_argument("--compulsory-note", default="read T and Ci, write T2 once")
    ap.add_argument("--note", default="", help="a paragraph under the title of a trace summary")
    ap.add_argument("--out", default=None)
    ap.add_argument("--command", default="")
    args = ap.parse_args()

    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1], args.kernel, args.steps_per_launch,
                          args.workload, int(args.compulsory_bytes), args.out, args.command,
                          calibration=args.calibration, note=args.compulsory_note)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.out, args.command, title=args.title, note=args.note)
        return
    if args.summarize_sq:
        summarize_sq(args.summarize_sq[0], args.summarize_sq[1], args.kernel, args.title, args.out, args.command)
        return

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
        # then the forward kernels on the benchmark workload.
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            d3.copy_(dst, src)
        torch.cuda.synchronize()
        del src, dst
        T0h, Cih = workloads.bump(n, n, n)
        tdt = torch.float64 if args.traffic_probe == "f64" else torch.bfloat16
        T = torch.from_numpy(T0h).to(tdt).to(dev)
        Ci = torch.from_numpy(Cih).to(tdt).to(dev)
        s = d3.problem_scalars(Ci)
        sc = (s["lam"], s["dt"], s["rdx"], s["rdy"], s["rdz"])
        T2 = T.clone()
        S = d3.pass_plan(T.shape, 100, tdt)[0]
        for _ in range(3):
            d3.stepn(T2, T, Ci, *sc, S)
        if tdt == torch.float64:
            for _ in range(3):
                d3.step2(T2, T, Ci, *sc)
        for _ in range(3):
            d3.step(T2, T, Ci, *sc)
        torch.cuda.synchronize()
        log("traffic probe done: 3 copies of 1 GiB, 3 %d-step launches%s and 3 single-step launches on bump%d %s"
            % (S, ", 3 two-step launches" if tdt == torch.float64 else "", n, args.traffic_probe))
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
    plan = d3.pass_plan(T.shape, nt, torch.float64)
    PASS = plan[0]

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
    # A pass of S steps must read T and Ci and write T2 once: 3*8*N
    # compulsory bytes per launch, the roofline's algorithmic bytes (T_eff
    # counts them once per step, i.e. S times per launch).
    compulsory = 3 * 8 * N
    achieved = compulsory / (kS_ms / 1e3) / 1e9
    traffic = None
    tr_hash = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        tr_hash = tr.get("source_hash")
        if tr_hash == kernel_source_hash() and tr.get("workload") == "bump%d_f64" % n and \
                tr.get("steps_per_launch") == PASS:
            traffic = tr.get("bytes_per_launch")
    hbm = traffic / (kS_ms / 1e3) / 1e9 if traffic else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "step_tbs (%d steps per launch)" % PASS, "kernel_avg_us": round(kS_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": compulsory,
                "algorithmic_bytes_note": "compulsory bytes of one pass: read T and Ci, write T2 once",
                "hbm_GBps": round(hbm, 1) if hbm else None,
                "frac_physical": round(hbm / HBM_PEAK_GBPS, 4) if hbm else None,
                "teff_over_peak": round(PASS * compulsory / (kS_ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                "traffic_source_hash": tr_hash,
                # the FP64 vector-arithmetic roof beside the bandwidth one: the
                # step's 18 operations per point (no fused multiply-add), S
                # steps per launch, against 256 CUs x 4 SIMDs x 16 FP64 lanes x
                # 2.4 GHz = 39.3 Top/s (78.6 TFLOP/s counts an FMA as two)
                "alu": {"ops_per_point_step": ALU_OPS_PER_POINT_STEP,
                        "achieved": round(ALU_OPS_PER_POINT_STEP * (n - 2) ** 3 * PASS / (kS_ms / 1e3) / 1e12, 2),
                        "peak": FP64_VECTOR_OPS_PEAK, "unit": "Top/s",
                        "frac": round(ALU_OPS_PER_POINT_STEP * (n - 2) ** 3 * PASS / (kS_ms / 1e3) / 1e12
                                      / FP64_VECTOR_OPS_PEAK, 4)}}
    single = {"kernel": "step_zmarch (one step per launch)", "kernel_avg_us": round(k1_ms * 1e3, 2),
              "teff_GBps": round(bytes_step / (k1_ms / 1e3) / 1e9, 1)}
    two = {"kernel": "step_tb2 (two steps per launch)", "kernel_avg_us": round(k2_ms * 1e3, 2),
           "teff_GBps": round(2 * bytes_step / (k2_ms / 1e3) / 1e9, 1)}
    log("bench: %d-step kernel %.1f us (%.1f GB/s compulsory), two-step %.1f us, single-step %.1f us (%.1f GB/s)"
        % (PASS, kS_ms * 1e3, achieved, k2_ms * 1e3, k1_ms * 1e3, single["teff_GBps"]))

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
        # timed at 512^3; errors over the whole grid against the FP64 result
        # of the same time loop, which equals the FP64 oracle bit for bit
        # (tests/test_gpu_headline.py), at 512^3 and at the 256^3 instance
        ref = T0.clone()
        T2 = torch.empty_like(ref)
        d3.run(ref, T2, Ci, *sc, nt)
        del T2
        forms = (("f32", torch.float32, "sr"), ("bf16_sr", torch.bfloat16, "sr"), ("bf16_rne", torch.bfloat16, "rne"))
        for name, tdt, rounding in forms:
            Tl = T0.cpu().to(tdt).to(dev)
            T2l = torch.empty_like(Tl)
            Cl = Ci.cpu().to(tdt).to(dev)
            X0 = Tl.clone()
            d3.run(Tl, T2l, Cl, *sc, nt, rounding=rounding)
            extra["maxrel_%s_512" % name] = max_rel_dev(Tl, ref, torch)
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
            extra["passes_%s" % name] = d3.pass_plan(Tl.shape, nt, tdt, rounding=rounding)[0]
            del Tl, T2l, Cl, X0
        del ref
        torch.cuda.empty_cache()
        m = 256
        a0, c0 = workloads.bump(m, m, m)
        a0d, c0d = torch.from_numpy(a0).to(dev), torch.from_numpy(c0).to(dev)
        s256 = d3.problem_scalars(c0d)
        sc256 = (s256["lam"], s256["dt"], s256["rdx"], s256["rdy"], s256["rdz"])
        r256 = a0d.clone()
        d3.run(r256, torch.empty_like(r256), c0d, *sc256, nt)
        for name, tdt, rounding in forms:
            Tl = torch.from_numpy(a0).to(tdt).to(dev)
            d3.run(Tl, torch.empty_like(Tl), torch.from_numpy(c0).to(tdt).to(dev), *sc256, nt, rounding=rounding)
            extra["maxrel_%s_256" % name] = max_rel_dev(Tl, r256, torch)
        extra["precision_gates"] = {"f32": 1e-5, "bf16_sr": 2e-2, "bf16_rne": None,
                                    "reference": "FP64 time loop (bit-identical to the FP64 oracle)"}
        del a0d, c0d, r256
        torch.cuda.empty_cache()
        log("bench: precision forms", {k: v for k, v in extra.items() if "rel" in k or "speedup" in k})

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
        # the same call captured once into a graph and replayed: the launches
        # of a call go to the device together
        side = torch.cuda.Stream(dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            d3.run(Ts, T2s, Cs, *scs, 100)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            d3.run(Ts, T2s, Cs, *scs, 100)
        for _ in range(3):
            graph.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(20):
            graph.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        tg = e0.elapsed_time(e1) / 20 / 1e3 / 100
        extra["t_step_uniform64_f64_graph_us"] = round(tg * 1e6, 2)
        extra["teff_uniform64_f64_graph_GBps"] = round(3 * 8 * 64 ** 3 / tg / 1e9, 1)
        del graph, Ts, Cs, T2s
        log("bench: 64^3 FP64 time loop %.2f us per step (%.2f replayed from a graph)" % (ts * 1e6, tg * 1e6))

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
        # the same field and time loop in the other storage forms
        for tdt, rnd, tag, esz in ((torch.float32, "sr", "f32", 4), (torch.bfloat16, "sr", "bf16_sr", 2),
                                   (torch.bfloat16, "rne", "bf16_rne", 2)):
            Tq = torch.from_numpy(x2).to(dev, tdt)
            Cq = torch.full_like(Tq, 0.5)
            Sq = torch.empty_like(Tq)
            d3.run2d(Tq, Sq, Cq, *sc2, 10, rounding=rnd)
            e0.record(stream)
            for _ in range(3):
                d3.run2d(Tq, Sq, Cq, *sc2, 100, rounding=rnd)
            e1.record(stream)
            torch.cuda.synchronize()
            tq = e0.elapsed_time(e1) / 3 / 1e3 / 100
            extra["t_step_2d_8192_%s_us" % tag] = round(tq * 1e6, 2)
            extra["teff_2d_8192_%s_GBps" % tag] = round(3 * esz * n2 * n2 / tq / 1e9, 1)
            del Tq, Cq, Sq
        del T2d, C2d, S2d, x2
        torch.cuda.empty_cache()
        log("bench: 2-D 8192^2 us per step: FP64 %.1f, FP32 %.1f, BF16-SR %.1f, BF16-RNE %.1f"
            % (ts * 1e6, extra["t_step_2d_8192_f32_us"], extra["t_step_2d_8192_bf16_sr_us"],
               extra["t_step_2d_8192_bf16_rne_us"]))

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
            tfs, tbs = [], []
            for rep in range(4):   # the first repetition warms up
                Tg.copy_(X0)
                ev[0].record(stream)
                d3.run(Tg, T2g, Cg, *scg, ntg, ckpt=ws, ckpt_every=C)
                ev[1].record(stream)
                d3.loss(Tg, Tt, seed)
                ev[2].record(stream)
                d3.adjoint_run(X0, Cg, seed, gT0, gCi, ws, True, *scg, ntg, C)
                ev[3].record(stream)
                torch.cuda.synchronize()
                if rep:
                    tfs.append(ev[0].elapsed_time(ev[1]))
                    tbs.append(ev[2].elapsed_time(ev[3]))
            tf, tb = statistics.median(tfs), statistics.median(tbs)
            extra["adjoint_%s_256_fwd_ms" % tag] = round(tf, 3)
            extra["adjoint_%s_256_bwd_ms" % tag] = round(tb, 3)
            extra["adjoint_%s_256_ratio" % tag] = round(tb / tf, 3)
            extra["adjoint_%s_256_gradnorm" % tag] = float(d3.norm2(gT0)) ** 0.5
            del X0, Cg, Tt, ws, Tg, T2g, seed, gT0, gCi
            torch.cuda.empty_cache()
        log("bench: adjoint", {k: v for k, v in extra.items() if k.startswith("adjoint")})

        # ------------------------------------------------------ large adjoint form
        if not args.no_large:
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
                   "nx": n, "ny": n, "nz": n, "nt": nt,
                   "kernel": "passes of %s steps (temporal blocking)" % ",".join(str(p) for p in sorted(set(plan))),
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
