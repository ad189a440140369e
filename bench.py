#!/usr/bin/env python3
"""Benchmark: ground-state solves per second of the rotating SOC spin-1 PCG
solver on one MI355X, mixed FP32->FP64 against plain FP64.

Headline (`value`): a continuous stream of solves of the 2D workload 256x256 on
[-12,12]^2, harmonic trap, Omega = 0.6, SOC strength 1.0, c0 = 500, c1 = -2,
initial guess ((x+iy) phi_a, phi_a, phi_a) + 1e-3 complex noise with seeds
2602, 2603, ..., each to the energy criterion at the paper's default tolerance
1e-14 (Algorithm 1 with the line search of Algorithm 2). `--inflight` requests
(default 32) are on the device at all times: a new one is submitted as soon as
one completes, and requests are admitted into freed slots at chunk boundaries
(continuous batching). A step is `--inflight` completions; `--warmup` steps
fill the pipeline untimed, then the clock runs over `--steps` steps. The same
seeds are streamed in plain FP64 first: a mixed solve counts only when its
energy agrees with the FP64 solve of the same seed to |dE| / max(|E|, 1) <
1e-10, and the FP64 stream's rate gives the mixed-vs-FP64 factor. The guesses
are resident in device memory before the clock starts.

Other sections of the same JSON line: per-kernel timing at full slot
occupancy (the roofline), the headline workload one solve at a time
(latency), the 64^2 workload, the 3D 128^3 cascadic-multigrid solve, Example
7's anisotropic cases at 256^3 on the elongated domain, the
96-solve parameter sweep, Table 2 by enumeration, a served stream with Poisson
arrivals, and the CPU oracle on the host cores. Run only when named: `gaps`
(the sweep's three grid classes together and alone at a fixed iteration count,
to be read under a kernel trace) and `c4oracle` (the oracle on the sweep's
128^2 solves, host only).

Prints one JSON line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ground-state solves/s at |dE|<1e-10 (mixed vs FP64 PCG); p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure
DE_GATE = 1e-10
TOL = 1e-14               # energy criterion (3.11), the paper's default tolerance (Sec. 4)
KERNEL_SOURCES = ("paper_2602_17950_amd/csrc/fft_core.h", "paper_2602_17950_amd/csrc/fft_launch.h",
                  "paper_2602_17950_amd/csrc/fft_fwd.hip", "paper_2602_17950_amd/csrc/fft_inv.hip",
                  "paper_2602_17950_amd/csrc/fft_mid.hip", "paper_2602_17950_amd/csrc/pw_kernels.hip",
                  "paper_2602_17950_amd/csrc/device_common.h", "paper_2602_17950_amd/csrc/control.h",
                  "paper_2602_17950_amd/csrc/gs_internal.h")
TRAFFIC_SUMMARY = "profiles/hbm_traffic_kernels256.md"
SECTIONS = ("headline", "kernels", "tuner", "single", "c1", "cm3d", "ex7", "sweep", "table2", "serve")
# host-only sections, run only when named (the oracle on the sweep's 128^2 solves
# takes about an hour of host time)
EXTRA_SECTIONS = ("c3oracle", "c4oracle")
# GPU sections run only when named: `gaps` exists to be run under a kernel trace
GPU_EXTRA_SECTIONS = ("gaps",)
GAP_PAUSE_S = 0.25        # host pause between the `gaps` batches: marks them apart in a trace
KINDS = ("hl_fwd", "hl_mid", "hl_inv", "pre_fwd", "pre_mid", "pre_inv", "resid", "lsred", "ctrl", "eval")
# Table 2 (Example 3): lowest energy over the 1000 guess combinations of Sec. 4, and the
# paper's CM-PCG CPU seconds for that one solve (a Xeon Gold 6248R, threads not stated;
# context only)
TABLE2 = {0.6: (2.2833, 7.0), 0.7: (2.0437, 116.0), 0.8: (1.6806, 46.0), 0.9: (1.0492, 1340.0)}
GUESS_KINDS = ("a", "b", "bbar", "c", "cbar", "d", "dbar", "e", "ebar", "f")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(label):
    """HBM bytes per launch of kernel `label` from the committed counter summary,
    or None when the summary is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"traffic_bytes_per_launch\[{re.escape(label)}\]:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * len(xs) + 0.5)) - 1))
    return xs[k]


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def oracle_objects(O, pb):
    return (O.Grid(pb.dim, pb.n, pb.L), O.Trap(pb.g, pb.q2, pb.q4), O.Params(pb.omega, pb.gamma, pb.c0, pb.c1))


def oracle_rate(pb, psi0, threads, seconds, iters_per_solve):
    """The oracle's PCG from psi0 for about `seconds` of host time on `threads`
    threads: (seconds per iteration, iterations run, wall seconds)."""
    import oracle as O
    O.set_threads(threads)
    g, t, p = oracle_objects(O, pb)
    probe = 3
    t0 = time.perf_counter()
    O.pcg(g, t, p, psi0, O.Options(tol=1e-12, max_iter=probe))
    t_probe = time.perf_counter() - t0
    k = int(max(probe + 2, min(iters_per_solve, seconds / max(t_probe / probe, 1e-6))))
    t0 = time.perf_counter()
    r = O.pcg(g, t, p, psi0, O.Options(tol=1e-12, max_iter=k))
    dt = time.perf_counter() - t0
    done = max(1, r.iters)
    return dt / done, done, dt


def cpu_baseline(pb, psi0, iters_per_solve, seconds):
    """The FP64 CPU oracle on the same input, timed on all host cores for a
    bounded number of PCG iterations of the headline solve and scaled to
    solves/s by the mean iteration count of the GPU's FP64 solves of the
    workload; the same on one thread."""
    cores = os.cpu_count() or 1
    per_all, done_all, dt_all = oracle_rate(pb, psi0, cores, seconds, iters_per_solve)
    per_one, done_one, dt_one = oracle_rate(pb, psi0, 1, seconds / 2, iters_per_solve)
    return {
        "value": 1.0 / (per_all * iters_per_solve),
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"first {done_all} PCG iterations of the seed-2602 256^2 solve on the host "
                   f"({dt_all:.1f} s, {per_all * 1e3:.1f} ms/iteration on {cores} threads), scaled by the "
                   f"mean {iters_per_solve:.0f} iterations of the GPU's FP64 solves of the workload"),
        "one_thread": {"value": 1.0 / (per_one * iters_per_solve), "ms_per_iteration": per_one * 1e3,
                       "iterations": done_one},
        "ms_per_iteration": per_all * 1e3,
    }


def run_stream(ctx, torch, probs, guesses, outs, opt, inflight, nwarm, ntimed):
    """Continuous stream over probs in order with `inflight` requests on the
    device at all times: nwarm + ntimed + inflight requests are submitted, one
    as each earlier one completes. The clock runs from the nwarm-th completion
    (after a device synchronisation) to the (nwarm + ntimed)-th, so the window
    sees a full pipeline at both ends; the last requests then drain untimed.
    Every submitted request completes, so both streams over the same seeds
    hold results for every index. Returns (results by index, timed seconds,
    indices completed in the timed window)."""
    total = nwarm + ntimed + inflight
    assert len(probs) >= total
    tickets, done, order = {}, {}, []
    nxt = 0
    t0 = t1 = None

    def fill():
        nonlocal nxt
        while len(tickets) < inflight and nxt < total:
            tickets[nxt] = ctx.submit(probs[nxt], guesses[nxt], outs[nxt], opt)
            nxt += 1

    fill()
    if nwarm == 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    while len(done) < total:
        ctx.progress(block=True)
        for i in list(tickets):
            r = ctx.poll(tickets[i])
            if r is None:
                continue
            done[i] = r
            del tickets[i]
            order.append(i)
            if t0 is None and len(order) == nwarm:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if t1 is None and len(order) == nwarm + ntimed:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
        fill()
    torch.cuda.synchronize()
    return done, t1 - t0, order[nwarm:nwarm + ntimed]


def kernel_table(ctx, torch, probs, guesses, outs, opt, iters):
    """Average duration and algorithmic bytes per launch of every kernel kind
    with all slots running every iteration (tol 0, `iters` iterations)."""
    reqs = [(pb, g, o, opt, None) for pb, g, o in zip(probs, guesses, outs)]
    ctx.batch_solve(reqs)   # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.batch_solve(reqs)
    torch.cuda.synchronize()
    row = {"ms_per_iteration": (time.perf_counter() - t) / iters * 1e3, "kinds": {}}
    for kind in KINDS:
        ctx.kernel_timer_start(kind)
        ctx.batch_solve(reqs)
        torch.cuda.synchronize()
        k = ctx.kernel_timer_read()
        ctx.kernel_timer_start(None)
        if k["launches"]:
            avg_s = k["ms"] * 1e-3 / k["launches"]
            bpl = k["bytes"] / k["launches"]
            row["kinds"][kind] = {"avg_us": avg_s * 1e6, "launches": k["launches"], "bytes_per_launch": bpl,
                                  "GBs": bpl / avg_s / 1e9, "per_iteration_us": k["ms"] * 1e3 / iters}
    return row


def roofline_of(row, kind, label, where):
    k = row["kinds"][kind]
    return {"bound": "hbm", "achieved": k["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": k["GBs"] / HBM_PEAK_GBS, "traffic": measured_traffic(label), "kernel": label,
            "kind": kind, "launches": k["launches"], "avg_us": k["avg_us"],
            "bytes_per_launch": k["bytes_per_launch"], "timed_in": where}


class Batch:
    """Device-resident guesses and outputs for a list of (Problem, guess)."""

    def __init__(self, torch, probs):
        self.probs = [pb for pb, _ in probs]
        self.guess = [None if g is None else torch.from_numpy(g).to("cuda") for _, g in probs]
        self.out = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device="cuda") for pb in self.probs]

    def requests(self, opt):
        return [(pb, g, o, opt, None) for pb, g, o in zip(self.probs, self.guess, self.out)]


def host_sections(sections, args):
    """Sections that run on the host only: `c3oracle`, the FP64 oracle on the
    128^3 cascadic-multigrid solve of `cm3d`, level by level to completion, and
    `c4oracle`, the FP64 oracle on the
    solves of the 96-solve sweep on one grid size (--c4-n, default 128^2;
    --c4-count of them after skipping --c4-start), energy criterion 1e-12, all
    host cores, each solve to completion."""
    import numpy as np
    from paper_2602_17950_amd import inputs
    import oracle as O
    line = {"metric": METRIC, "data": "synthetic", "n_gpus": 0}
    if "c3oracle" in sections:
        # the 128^3 cascadic-multigrid solve of the cm3d section on the oracle, level by level
        cores = os.cpu_count() or 1
        O.set_threads(cores)
        pb, _ = inputs.workload_aniso_3d(n=128)
        levels = [inputs.Problem(dim=3, n=(m, m, m), L=pb.L, g=pb.g, omega=pb.omega, gamma=pb.gamma, c0=pb.c0,
                                 c1=pb.c1) for m in (32, 64, 128)]
        psi = inputs.initial_guess(levels[0], ("a", "a", "a"))
        rows, prev = [], None
        t_all = time.perf_counter()
        for q in levels:
            g, t, p = oracle_objects(O, q)
            t0 = time.perf_counter()
            if prev is not None:
                psi = O.interp(prev, psi, g)
            r = O.pcg(g, t, p, psi, O.Options(tol=1e-12))
            dt = time.perf_counter() - t0
            psi, prev = r.psi, g
            rows.append({"n": q.n[0], "s": dt, "iters": r.iters, "status": r.status})
            log(f"c3oracle {q.n[0]}^3: {dt:.1f}s, {r.iters} iterations")
        ev = O.evaluate(prev, t, p, psi)
        line["c3oracle"] = {"s": time.perf_counter() - t_all, "threads": cores, "levels": rows, "E": ev["E"],
                            "mu": ev["mu"], "resid_inf": ev["resid_inf"],
                            "workload": "the cm3d section's solve: 3D 128^3 on [-8,8]^3, V=(x^2+y^2+4z^2)/2, "
                                        "Omega=0.5, SOC 1.0, c0=800, c1=5; cascadic multigrid 32^3->64^3->128^3 "
                                        "from (a,a,a); FP64 oracle, energy criterion 1e-12 per level"}
    if "c4oracle" in sections:
        cores = os.cpu_count() or 1
        O.set_threads(cores)
        spec = inputs.workload_sweep_2d()
        idx = [i for i, (pb, _) in enumerate(spec) if pb.n[0] == args.c4_n][args.c4_start:]
        if args.c4_count > 0:
            idx = idx[:args.c4_count]
        rows = []
        t_all = time.perf_counter()
        for k, i in enumerate(idx):
            pb, kinds = spec[i]
            g, t, p = oracle_objects(O, pb)
            t0 = time.perf_counter()
            r = O.pcg(g, t, p, inputs.initial_guess(pb, kinds), O.Options(tol=1e-12))
            dt = time.perf_counter() - t0
            rows.append({"index": i, "s": dt, "iters": r.iters, "status": r.status,
                         "E": O.evaluate(g, t, p, r.psi)["E"]})
            log(f"c4oracle {k + 1}/{len(idx)}: solve {i} {dt:.1f}s, {r.iters} iterations")
        T = time.perf_counter() - t_all
        line["c4oracle"] = {"solves": len(rows), "s": T, "solves_per_s": len(rows) / T, "threads": cores,
                            "iters_mean": float(np.mean([r["iters"] for r in rows])), "rows": rows,
                            "workload": f"the {args.c4_n}^2 solves of the 96-solve sweep (seed 17950) after "
                                        f"skipping {args.c4_start}, FP64 oracle, energy criterion 1e-12, one after "
                                        "another on all host cores"}
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="timed steps of --inflight completions")
    ap.add_argument("--warmup", type=int, default=1, help="untimed steps that fill the pipeline")
    ap.add_argument("--inflight", type=int, default=32, help="requests on the device at once (headline)")
    ap.add_argument("--n", type=int, default=256, help="grid points per axis of the headline workload")
    ap.add_argument("--kernel-iters", type=int, default=128, help="iterations per kernel-table run")
    ap.add_argument("--mixed-dir", choices=("fp32", "fp64"), default="fp32",
                    help="direction precision of the double phase of mixed solves")
    ap.add_argument("--sections", default=",".join(SECTIONS))
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-capacity-requests", type=int, default=48)
    ap.add_argument("--serve-loads", default="0.5,0.8", help="arrival rates / measured capacity of the served mix")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--c4-start", type=int, default=0,
                    help="c4oracle: skip this many of the sweep's solves of the chosen size (resume a run)")
    ap.add_argument("--c4-n", type=int, default=128, choices=(128, 256, 512),
                    help="c4oracle: grid size of the sweep's solves to run")
    ap.add_argument("--c4-count", type=int, default=0, help="c4oracle: at most this many solves (0: all)")
    ap.add_argument("--gap-iters", type=int, default=256, help="gaps: iterations of every solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every solve of these workloads fits one MI355X, and the "
              "path shards over independent solves (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    sections = [s for s in args.sections.split(",") if s]
    for s in sections:
        if s not in SECTIONS + EXTRA_SECTIONS + GPU_EXTRA_SECTIONS:
            sys.exit(f"unknown section {s!r}; choose from {SECTIONS + EXTRA_SECTIONS + GPU_EXTRA_SECTIONS}")
    if all(s in EXTRA_SECTIONS for s in sections):
        print(json.dumps(host_sections(sections, args)), flush=True)
        return

    import numpy as np
    import torch
    from paper_2602_17950_amd import gs, inputs

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB")
        return

    ctx = gs.Context(0)
    mdir = gs.GS_FP32 if args.mixed_dir == "fp32" else gs.GS_FP64
    o64 = gs.default_options(precision=gs.GS_FP64, tol=TOL)
    omx = gs.default_options(precision=gs.GS_MIXED, tol=TOL, dir_precision=mdir)
    line = {"metric": METRIC, "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "fp32->fp64", "data": "synthetic"}
    B = args.inflight

    # ------------------------------------------------------------------ headline
    total = B * (args.warmup + args.steps + 1)   # one more step drains after the clock stops
    iters64 = None
    if "headline" in sections:
        seeds = [2602 + i for i in range(total)]
        work = [inputs.workload_vortex_2d(n=args.n, seed=s) for s in seeds]
        probs = [pb for pb, _ in work]
        guesses = [torch.from_numpy(g).to("cuda") for _, g in work]
        outs = [torch.empty_like(g) for g in guesses]
        # a short warm run of both paths (class creation, first-launch costs)
        for opt in (o64, omx):
            ctx.batch_solve([(probs[i], guesses[i], outs[i], opt, None) for i in range(min(B, 4))])
        torch.cuda.synchronize()
        r64, T64, win64 = run_stream(ctx, torch, probs, guesses, outs, o64, B, B * args.warmup, B * args.steps)
        log(f"fp64 stream: {len(win64)} solves in {T64:.2f}s ({len(win64) / T64:.2f}/s)")
        rmx, Tmx, winmx = run_stream(ctx, torch, probs, guesses, outs, omx, B, B * args.warmup, B * args.steps)
        dEs = {i: rel(rmx[i]["E"], r64[i]["E"]) for i in rmx}
        counted = sum(1 for i in winmx if dEs[i] < DE_GATE)
        lat = [rmx[i]["wall_s"] for i in winmx]
        itmx = [rmx[i]["iters"] for i in winmx]
        iters64 = float(np.mean([r64[i]["iters"] for i in win64]))
        log(f"mixed stream: {len(winmx)} solves in {Tmx:.2f}s; counted {counted}; iters mean {np.mean(itmx):.0f}")
        line["value"] = counted / Tmx
        line["ms_per_step"] = Tmx / args.steps * 1e3
        line["p50_ms"] = percentile(lat, 50) * 1e3
        line["p99_ms"] = percentile(lat, 99) * 1e3
        line["iters_per_s"] = sum(itmx) / Tmx
        fp64_rate = len(win64) / T64
        line["headline"] = {
            "inflight": B, "solves_timed": len(winmx), "counted": counted,
            "solves_per_s_all": len(winmx) / Tmx,
            "dE_rel_max": max(dEs[i] for i in winmx), "dE_rel_median": float(np.median([dEs[i] for i in winmx])),
            "mixed_iters_mean": float(np.mean(itmx)),
            "mixed_iters_fp32_mean": float(np.mean([rmx[i]["iters_fp32"] for i in winmx])),
            "fp64_solves_per_s": fp64_rate, "fp64_iters_mean": iters64,
            "fp64_iters_per_s": sum(r64[i]["iters"] for i in win64) / T64,
            "fp64_p50_ms": percentile([r64[i]["wall_s"] for i in win64], 50) * 1e3,
            "fp64_p99_ms": percentile([r64[i]["wall_s"] for i in win64], 99) * 1e3,
            "speedup_counted": (counted / Tmx) / fp64_rate,
            "speedup_all": (len(winmx) / Tmx) / fp64_rate,
            "seeds": f"2602..{2601 + total} ({B} more than the warm-up and timed steps: the pipeline stays "
                     "full until the clock stops)",
            "latency_note": "p50/p99: submission to completion, over the timed window",
        }
        del guesses, outs

    # ---------------------------------------------------------- kernels at full occupancy
    if "kernels" in sections:
        kw = [inputs.workload_vortex_2d(n=args.n, seed=2602 + i) for i in range(B)]
        kb = Batch(torch, kw)
        tab = {}
        for name, opt in (("fp64", gs.default_options(precision=gs.GS_FP64, tol=0.0, max_iter=args.kernel_iters)),
                          ("fp32", gs.default_options(precision=gs.GS_FP32, tol=0.0, max_iter=args.kernel_iters)),
                          ("fp64_state_fp32_dir", gs.default_options(precision=gs.GS_FP64, tol=0.0,
                                                                     max_iter=args.kernel_iters,
                                                                     dir_precision=gs.GS_FP32))):
            tab[name] = kernel_table(ctx, torch, kb.probs, kb.guess, kb.out, opt, args.kernel_iters)
            log(f"kernels {name}: {tab[name]['ms_per_iteration']:.3f} ms/iteration; " + ", ".join(
                f"{k} {v['avg_us']:.1f}us {v['GBs'] / 1e3:.2f}TB/s" for k, v in tab[name]["kinds"].items()))
        line["kernels"] = {"slots": B, "iterations": args.kernel_iters, "grid": args.n, "table": tab,
                           "note": ("every slot runs every iteration (tol 0): launches at full occupancy; "
                                    "GBs = algorithmic bytes / average launch duration")}
        # the headline's mixed solves spend almost all iterations in the double phase
        # (double state, direction in the --mixed-dir precision): its dominant kernel
        hx = "fp64_state_fp32_dir" if mdir == gs.GS_FP32 else "fp64"
        dom = max(tab[hx]["kinds"], key=lambda k: tab[hx]["kinds"][k]["avg_us"])
        line["roofline"] = roofline_of(tab[hx], dom, f"{hx}:{dom}",
                                       f"double phase of the mixed path, {B} slots of {args.n}^2 at full occupancy")
        d64 = max(tab["fp64"]["kinds"], key=lambda k: tab["fp64"]["kinds"][k]["avg_us"])
        line["roofline_fp64"] = roofline_of(tab["fp64"], d64, f"fp64:{d64}",
                                            f"plain FP64 path, {B} slots of {args.n}^2 at full occupancy")
        del kb
        # achievable streaming bandwidth in the same run: the better of a 1 GiB
        # device-to-device copy and a 1 GiB float scale b = 2a (torch's kernels),
        # bytes read + written over the time of 10 repetitions
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        a32, b32 = a.view(torch.float32), b.view(torch.float32)
        stream = {}
        for name, f in (("copy", lambda: b.copy_(a)), ("scale_f32", lambda: torch.mul(a32, 2.0, out=b32))):
            f()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                f()
            e1.record()
            torch.cuda.synchronize()
            stream[name] = 10 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        best = max(stream.values())
        for key in ("roofline", "roofline_fp64"):
            line[key]["stream_GBs"] = stream
            line[key]["frac_of_stream"] = line[key]["achieved"] / best
        log("stream: " + ", ".join(f"{k} {v:.0f} GB/s" for k, v in stream.items()))
        del a, b, a32, b32

    # ------------------------------------------- FFT schedules: fixed table vs tuned
    if "tuner" in sections:
        tun = {}
        for label, nslots, make in (("128^2", B, lambda i: inputs.workload_vortex_2d(n=128, seed=2602 + i)),
                                    ("256^2", B, lambda i: inputs.workload_vortex_2d(n=256, seed=2602 + i)),
                                    ("512^2", 16, lambda i: inputs.workload_vortex_2d(n=512, seed=2602 + i)),
                                    ("1024^2", 8, lambda i: inputs.workload_vortex_2d(n=1024, seed=2602 + i)),
                                    ("128^3", 4, lambda i: inputs.workload_aniso_3d(n=128))):
            tb = Batch(torch, [make(i) for i in range(nslots)])
            row = {"slots": nslots}
            for name, opt in (("fp64_state_fp32_dir", gs.default_options(precision=gs.GS_FP64, tol=0.0, max_iter=64,
                                                                         dir_precision=gs.GS_FP32)),
                              ("fp64", gs.default_options(precision=gs.GS_FP64, tol=0.0, max_iter=64))):
                ms = {}
                for tune in (0, 1):
                    with gs.Context(0) as tctx:
                        tctx.set_autotune(tune)
                        tctx.batch_solve(tb.requests(opt))   # warm-up; with tuning on, its first chunk tunes
                        torch.cuda.synchronize()
                        t = time.perf_counter()
                        tctx.batch_solve(tb.requests(opt))
                        torch.cuda.synchronize()
                        ms[tune] = (time.perf_counter() - t) / 64 * 1e3
                        if tune:
                            rep = [r for r in tctx.autotune_report() if r["decided"]]
                            chosen = {k: v["chosen"] for r in rep for k, v in r["passes"].items()}
                row[name] = {"ms_per_iteration_fixed": ms[0], "ms_per_iteration_tuned": ms[1],
                             "gain": ms[0] / ms[1], "chosen": chosen}
            log(f"tuner {label}: " + ", ".join(f"{k} {v['ms_per_iteration_fixed']:.3f} -> "
                                               f"{v['ms_per_iteration_tuned']:.3f} ms"
                                               for k, v in row.items() if k != "slots"))
            tun[label] = row
            del tb
        tun["note"] = ("ms per batched iteration of the given number of solves (tol 0, every slot running), fixed "
                       "table against the schedules the autotuner chose in the warm-up's first chunk; candidates are "
                       "(lines x threads) per block, the same bits for every choice")
        line["tuner"] = tun

    # ------------------------------------------------------------ single solve
    if "single" in sections:
        pb, g0 = inputs.workload_vortex_2d(n=args.n, seed=2602)
        one = Batch(torch, [(pb, g0)])
        single = {}
        for name, opt in (("fp64", o64), ("mixed", omx)):
            ctx.solve_device(pb, one.guess[0], one.out[0], opt)   # warm
            lat, r = [], None
            for k in range(3):
                t = time.perf_counter()
                r = ctx.solve_device(pb, one.guess[0], one.out[0], opt)
                lat.append(time.perf_counter() - t)
            single[name] = {"solves_per_s": len(lat) / sum(lat), "p50_ms": percentile(lat, 50) * 1e3,
                            "iters": r["iters"], "iters_fp32": r["iters_fp32"], "E": r["E"],
                            "ms_per_iteration": percentile(lat, 50) * 1e3 / r["iters"]}
            log(f"single {name}: {single[name]['p50_ms']:.1f} ms, iters {r['iters']}")
        single["dE_rel"] = rel(single["mixed"]["E"], single["fp64"]["E"])
        single["speedup_mixed_vs_fp64"] = single["mixed"]["solves_per_s"] / single["fp64"]["solves_per_s"]
        line["single"] = single
        if line["value"] is None:   # headline section skipped
            line["value"] = single["mixed"]["solves_per_s"] if single["dE_rel"] < DE_GATE else 0.0
            line["ms_per_step"] = single["mixed"]["p50_ms"]

    # --------------------------------------------------- 64^2 workload, GPU and oracle
    if "c1" in sections:
        pb, g0 = inputs.workload_small_2d()
        one = Batch(torch, [(pb, g0)])
        opt = gs.default_options(precision=gs.GS_FP64, tol=1e-12)
        ctx.solve_device(pb, one.guess[0], one.out[0], opt)
        lat = []
        for k in range(5):
            t = time.perf_counter()
            r = ctx.solve_device(pb, one.guess[0], one.out[0], opt)
            lat.append(time.perf_counter() - t)
        c1 = {"gpu": {"solves_per_s": len(lat) / sum(lat), "p50_ms": percentile(lat, 50) * 1e3,
                      "iters": r["iters"], "E": r["E"]},
              "workload": ("2D 64x64 on [-8,8]^2, harmonic, Omega 0, SOC 0.5, c0 100, c1 -0.5, Gaussian "
                           "guess, plain FP64, energy criterion 1e-12")}
        if not args.no_cpu_baseline:
            import oracle as O
            g, t, p = oracle_objects(O, pb)
            for name, th in (("oracle_all_cores", os.cpu_count() or 1), ("oracle_1_thread", 1)):
                O.set_threads(th)
                t0 = time.perf_counter()
                ro = O.pcg(g, t, p, g0, O.Options(tol=1e-12))
                dt = time.perf_counter() - t0
                E = O.evaluate(g, t, p, ro.psi)["E"]
                c1[name] = {"s": dt, "solves_per_s": 1.0 / dt, "iters": ro.iters, "threads": th, "E": E,
                            "dE_rel_gpu": rel(r["E"], E)}
            c1["gpu_vs_oracle_all_cores"] = c1["gpu"]["solves_per_s"] / c1["oracle_all_cores"]["solves_per_s"]
        log(f"c1: gpu {c1['gpu']['p50_ms']:.1f} ms/solve")
        line["c1"] = c1

    # ------------------------------------------------------- 3D multigrid solve
    if "cm3d" in sections:
        pb3, _ = inputs.workload_aniso_3d(n=128)
        pc = inputs.Problem(dim=3, n=(32, 32, 32), L=pb3.L, g=pb3.g, omega=pb3.omega, gamma=pb3.gamma,
                            c0=pb3.c0, c1=pb3.c1)
        g3 = torch.from_numpy(inputs.initial_guess(pc, ("a", "a", "a"))).to("cuda")
        out3 = torch.empty((3,) + pb3.shape, dtype=torch.complex128, device="cuda")
        cm = {}
        for name, prec in (("fp64", gs.GS_FP64), ("mixed", gs.GS_MIXED)):
            opt = gs.default_options(precision=prec, tol=1e-12, cm_levels=3,
                                     dir_precision=mdir if prec == gs.GS_MIXED else gs.GS_FP64)
            ctx.solve_device(pb3, g3, out3, opt)   # warm
            t = time.perf_counter()
            r = ctx.solve_device(pb3, g3, out3, opt)
            cm[name] = {"s": time.perf_counter() - t, "E": r["E"], "mu": r["mu"], "iters_fine": r["iters"],
                        "iters_coarse": r["iters_coarse"], "iters_fp32": r["iters_fp32"],
                        "resid_inf": r["resid_inf"], "virial": r["virial"], "status": r["rc"]}
            log(f"cm3d {name}: {cm[name]['s']:.2f}s E={r['E']:.15f} iters {r['iters']}+{r['iters_coarse']}")
        cm["dE_rel"] = rel(cm["mixed"]["E"], cm["fp64"]["E"])
        cm["workload"] = ("3D 128^3 on [-8,8]^3, V=(x^2+y^2+4z^2)/2, Omega=0.5, SOC 1.0, c0=800, c1=5; "
                          "cascadic multigrid 32^3->64^3->128^3 from (a,a,a); energy criterion 1e-12 per level")
        line["cm3d"] = cm
        del g3, out3

    # ------------------------------------------------------------------- ex7
    if "ex7" in sections:
        # Example 7's anisotropic cases on the elongated domain, as the paper runs
        # them: cascadic multigrid 64^3 -> 128^3 -> 256^3
        def ex7_problem(n, omega, gamma):
            return inputs.Problem(dim=3, n=(n, n, n), L=(10.0, 10.0, 80.0), g=(0.97, 1.03, 0.05), omega=omega,
                                  gamma=gamma, c0=3000.0, c1=1.0)
        out7 = torch.empty((3,) + ex7_problem(256, 0.5, 0.4).shape, dtype=torch.complex128, device="cuda")
        ex = {}
        for case, (omega, gamma) in ((4, (0.5, 0.4)), (5, (0.5, 0.8)), (6, (0.7, 0.4))):
            pb7, pc7 = ex7_problem(256, omega, gamma), ex7_problem(64, omega, gamma)
            g7 = torch.from_numpy(inputs.initial_guess(pc7, ("f", "f", "f"))).to("cuda")
            row = {}
            for name, prec in (("fp64", gs.GS_FP64), ("mixed", gs.GS_MIXED)):
                opt = gs.default_options(precision=prec, tol=1e-12, cm_levels=3,
                                         dir_precision=mdir if prec == gs.GS_MIXED else gs.GS_FP64)
                ctx.solve_device(pb7, g7, out7, opt)   # warm
                t = time.perf_counter()
                r = ctx.solve_device(pb7, g7, out7, opt)
                row[name] = {"s": time.perf_counter() - t, "E": r["E"], "mu": r["mu"], "iters_fine": r["iters"],
                             "iters_coarse": r["iters_coarse"], "iters_fp32": r["iters_fp32"],
                             "resid_inf": r["resid_inf"], "virial": r["virial"], "status": r["rc"]}
                log(f"ex7 case {case} {name}: {row[name]['s']:.2f}s E={r['E']:.15f} "
                    f"iters {r['iters']}+{r['iters_coarse']}")
            row["dE_rel"] = rel(row["mixed"]["E"], row["fp64"]["E"])
            ex[f"case{case}"] = row
            del g7
        ex["workload"] = ("Example 7, Cases 4-6: 3D 256^3 on [-10,10]^2 x [-80,80], gamma = (0.97, 1.03, 0.05), "
                          "c0=3000, c1=1, (Omega, SOC) = (0.5, 0.4), (0.5, 0.8), (0.7, 0.4); cascadic multigrid "
                          "64^3->128^3->256^3 from the Thomas-Fermi guess (f,f,f); energy criterion 1e-12 per level")
        line["ex7"] = ex
        del out7

    # ------------------------------------------------------------------- sweep
    cap = None
    if "sweep" in sections:
        spec = inputs.workload_sweep_2d()
        sw = Batch(torch, [(pb, inputs.initial_guess(pb, k)) for pb, k in spec])
        out = {}
        E = {}
        for name, prec, dirp in (("fp64", gs.GS_FP64, gs.GS_FP64), ("mixed", gs.GS_MIXED, mdir),
                                 ("fp64_state_fp32_dir", gs.GS_FP64, gs.GS_FP32)):
            opt = gs.default_options(precision=prec, tol=1e-12, dir_precision=dirp)
            t = time.perf_counter()
            rs = ctx.batch_solve(sw.requests(opt))
            dt = time.perf_counter() - t
            E[name] = [r["E"] for r in rs]
            out[name] = {"s": dt, "solves_per_s": len(rs) / dt, "iters_mean": float(np.mean([r["iters"] for r in rs])),
                         "p50_ms": percentile([r["wall_s"] for r in rs], 50) * 1e3,
                         "p99_ms": percentile([r["wall_s"] for r in rs], 99) * 1e3,
                         "warnings": sum(1 for r in rs if r["rc"] > 0), "errors": sum(1 for r in rs if r["rc"] < 0)}
            log(f"sweep {name}: {dt:.2f}s ({out[name]['solves_per_s']:.2f} solves/s)")
        d = [rel(a, b) for a, b in zip(E["mixed"], E["fp64"])]
        out["counted"] = sum(1 for x in d if x < DE_GATE)
        out["counted_solves_per_s"] = out["counted"] / out["mixed"]["s"]
        out["speedup_counted"] = out["counted_solves_per_s"] / out["fp64"]["solves_per_s"]
        # where the other solves end: a lower or a higher local minimum than the FP64 run's
        for name in ("mixed", "fp64_state_fp32_dir"):
            sgn = [(a - b) / max(abs(b), 1.0) for a, b in zip(E[name], E["fp64"])]
            out[name]["same_minimum"] = sum(1 for x in sgn if abs(x) < DE_GATE)
            out[name]["lower_energy"] = sum(1 for x in sgn if x <= -DE_GATE)
            out[name]["higher_energy"] = sum(1 for x in sgn if x >= DE_GATE)
            out[name]["log10_dE_histogram"] = {
                "edges": [-17, -12, -10, -8, -6, -4, -2, 1],
                "counts": np.histogram(np.log10(np.maximum(np.abs(sgn), 1e-17)),
                                       bins=[-17, -12, -10, -8, -6, -4, -2, 1])[0].tolist()}
        # the same sweep with the stop stated as a residual: float to max ||r||_inf < 1e-6,
        # then the double finish to ||r||_inf < 1e-10 (criterion (3.10)); FP64 to the same
        rr = {}
        Er = {}
        for name, prec, dirp in (("fp64", gs.GS_FP64, gs.GS_FP64), ("mixed", gs.GS_MIXED, mdir)):
            opt = gs.default_options(precision=prec, stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-10, switch_resid=1e-6,
                                     dir_precision=dirp)
            t = time.perf_counter()
            rs = ctx.batch_solve(sw.requests(opt))
            dt = time.perf_counter() - t
            Er[name] = [r["E"] for r in rs]
            rr[name] = {"s": dt, "solves_per_s": len(rs) / dt,
                        "iters_mean": float(np.mean([r["iters"] for r in rs])),
                        "resid_max": max(r["resid_inf"] for r in rs),
                        "warnings": sum(1 for r in rs if r["rc"] > 0), "errors": sum(1 for r in rs if r["rc"] < 0),
                        "status_counts": {str(c): sum(1 for r in rs if r["rc"] == c)
                                          for c in sorted(set(r["rc"] for r in rs))}}
            log(f"sweep residual-stop {name}: {dt:.2f}s ({rr[name]['solves_per_s']:.2f} solves/s)")
        sgn = [(a - b) / max(abs(b), 1.0) for a, b in zip(Er["mixed"], Er["fp64"])]
        rr["counted"] = sum(1 for x in sgn if abs(x) < DE_GATE)
        rr["lower_energy"] = sum(1 for x in sgn if x <= -DE_GATE)
        rr["higher_energy"] = sum(1 for x in sgn if x >= DE_GATE)
        rr["counted_solves_per_s"] = rr["counted"] / rr["mixed"]["s"]
        rr["speedup_counted"] = rr["counted_solves_per_s"] / rr["fp64"]["solves_per_s"]
        rr["speedup_all"] = rr["mixed"]["solves_per_s"] / rr["fp64"]["solves_per_s"]
        rr["stop"] = "float to max_l ||r_l||_inf < 1e-6, then double to < 1e-10; FP64 to < 1e-10"
        out["residual_stop"] = rr
        out["workload"] = ("96 2D solves, n uniform over {128,256,512}, L=16, Omega~U[0,0.9], SOC~U[0,2], "
                           "c0~U[100,2000], c1~U[-5,5], guesses over {(a,a,a),(b,a,a),(f,f,f)}, seed 17950; "
                           "energy criterion 1e-12 (residual_stop: the residual criterion), one batch")
        out["note"] = ("solves whose mixed and FP64 runs end in different local minima are not counted "
                       "(the landscape of the rotating problems has many); fp64_state_fp32_dir (no float "
                       "phase, only the search direction rounded to float) shows that any float rounding on "
                       "the path moves about half of these solves to another minimum, as often lower as higher")
        line["sweep"] = out
        cap = out["mixed"]["solves_per_s"]
        del sw

    # ------------------------------------------------------------------ gaps
    if "gaps" in sections:
        # Device idle time when the sweep's three grid classes (128^2, 256^2, 512^2,
        # one stream each) share the GPU: its 96 solves with tol 0 and a fixed
        # iteration count, so every slot of every class runs to the end; then each
        # class alone. Every configuration runs a warm-up batch (the first chunk of
        # a class tunes its FFT schedules) and a timed batch, with a host pause
        # before each batch so that a kernel trace splits into one segment per
        # batch; the union of kernel intervals over a segment against its span is
        # the busy fraction.
        spec = inputs.workload_sweep_2d()
        sw = Batch(torch, [(pb, inputs.initial_guess(pb, k)) for pb, k in spec])
        gp = {"iters": args.gap_iters, "segments": [],
              "workload": f"the 96 solves of the sweep, tol 0, {args.gap_iters} iterations each; "
                          "all three classes together, then each class alone"}
        for name, prec, dirp in (("fp64", gs.GS_FP64, gs.GS_FP64), ("fp64_state_fp32_dir", gs.GS_FP64, gs.GS_FP32)):
            opt = gs.default_options(precision=prec, tol=0.0, max_iter=args.gap_iters, dir_precision=dirp)
            reqs_all = sw.requests(opt)
            groups = [("all", reqs_all)] + [(f"n{n}", [q for q in reqs_all if q[0].n[0] == n]) for n in (128, 256, 512)]
            for gname, reqs in groups:
                for phase in ("warm", "timed"):
                    time.sleep(GAP_PAUSE_S)
                    t = time.perf_counter()
                    rs = ctx.batch_solve(reqs)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t
                    gp["segments"].append({"precision": name, "classes": gname, "phase": phase,
                                           "solves": len(reqs), "s": dt,
                                           "iters_min": min(r["iters"] for r in rs)})
                    log(f"gaps {name} {gname} {phase}: {len(reqs)} solves, {dt:.3f}s")
            tm = {g["classes"]: g["s"] for g in gp["segments"] if g["precision"] == name and g["phase"] == "timed"}
            gp[name] = {"together_s": tm["all"], "alone_sum_s": tm["n128"] + tm["n256"] + tm["n512"],
                        "alone_max_s": max(tm["n128"], tm["n256"], tm["n512"])}
        time.sleep(GAP_PAUSE_S)
        line["gaps"] = gp
        del sw

    # ------------------------------------------------------------------ table2
    if "table2" in sections:
        tb = {"rows": {}}
        total_s, nsolve, allmatch = 0.0, 0, True
        combos = list(itertools.product(GUESS_KINDS, repeat=3))
        opt = gs.default_options(precision=gs.GS_MIXED, dir_precision=mdir, tol=1e-14, cm_levels=3)
        for om, (E_paper, cpu_paper) in TABLE2.items():
            kw = dict(dim=2, L=(12.0, 12.0), omega=om, gamma=0.3, c0=50.0, c1=0.5)
            fine, coarse = inputs.Problem(n=(256, 256), **kw), inputs.Problem(n=(64, 64), **kw)
            guess = [torch.from_numpy(inputs.initial_guess(coarse, k)).to("cuda") for k in combos]
            outs = [torch.empty((3, 256, 256), dtype=torch.complex128, device="cuda") for _ in combos]
            torch.cuda.synchronize()
            t = time.perf_counter()
            rs = ctx.batch_solve([(fine, g, o, opt, None) for g, o in zip(guess, outs)])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            E = [r["E"] for r in rs]
            k = int(np.argmin(E))
            match = round(E[k], 4) == E_paper
            allmatch = allmatch and match
            total_s += dt
            nsolve += len(rs)
            tb["rows"][str(om)] = {"s": dt, "solves": len(rs), "E_lowest": E[k], "from": "".join(
                c + " " for c in combos[k]).strip(), "paper_E": E_paper, "match_4_decimals": match,
                "paper_cm_pcg_cpu_s_one_solve": cpu_paper,
                "fine_iters_mean": float(np.mean([r["iters"] for r in rs])),
                "coarse_iters_mean": float(np.mean([r["iters_coarse"] for r in rs])),
                "warnings": sum(1 for r in rs if r["rc"] > 0), "errors": sum(1 for r in rs if r["rc"] < 0)}
            log(f"table2 omega={om}: {dt:.2f}s, lowest E {E[k]:.8f} ({'matches' if match else 'differs from'} "
                f"{E_paper})")
            del guess, outs
        tb.update({"s": total_s, "solves": nsolve, "solves_per_s": nsolve / total_s, "all_match": allmatch,
                   "workload": ("Table 2 (Example 3): for Omega in {0.6,0.7,0.8,0.9}, the 1000 component-wise "
                                "combinations of the ten guesses of Sec. 4 on [-12,12]^2 (gamma 0.3, c0 50, "
                                "c1 0.5), each solved by CM-PCG 64^2->128^2->256^2, mixed precision, energy "
                                "criterion 1e-14; one batch per Omega; the lowest energy is the ground state")})
        line["table2"] = tb

    # ------------------------------------------------------------------- serve
    if "serve" in sections:
        spec = inputs.workload_serve(args.serve_requests)
        sv = Batch(torch, [(pb, inputs.initial_guess(pb, k)) for pb, k in spec])
        opt = gs.default_options(precision=gs.GS_MIXED, tol=1e-12, dir_precision=mdir)
        # capacity of the served mix: its first requests submitted at once (closed loop)
        ncap = min(len(spec), args.serve_capacity_requests)
        t = time.perf_counter()
        ctx.batch_solve([(sv.probs[i], sv.guess[i], sv.out[i], opt, None) for i in range(ncap)])
        torch.cuda.synchronize()
        cap_mix = ncap / (time.perf_counter() - t)
        log(f"serve capacity: {cap_mix:.2f} solves/s over the first {ncap} requests at once")
        serve = {"requests": len(spec), "capacity_solves_per_s": cap_mix, "capacity_requests": ncap, "loads": {}}
        for load in [float(x) for x in args.serve_loads.split(",") if x]:
            rate = load * cap_mix
            rng = np.random.default_rng(2603)
            arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(spec)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pending, tickets, done = 0, {}, {}
            while len(done) < len(spec):
                now = time.perf_counter() - t0
                while pending < len(spec) and arrivals[pending] <= now:
                    tickets[pending] = ctx.submit(sv.probs[pending], sv.guess[pending], sv.out[pending], opt)
                    pending += 1
                for i in list(tickets):
                    r = ctx.poll(tickets[i])
                    if r is not None:
                        done[i] = r
                        del tickets[i]
                        if len(done) % 40 == 0:
                            log(f"serve load {load}: {len(done)} of {len(spec)} done after "
                                f"{time.perf_counter() - t0:.0f}s")
                if len(done) < len(spec):
                    if tickets:
                        ctx.progress(block=pending >= len(spec) or
                                     arrivals[pending] > time.perf_counter() - t0 + 0.005)
                    else:
                        time.sleep(max(0.0, min(0.01, arrivals[pending] - (time.perf_counter() - t0))))
            T = time.perf_counter() - t0
            lat = [done[i]["wall_s"] for i in range(len(spec))]
            serve["loads"][str(load)] = {
                "arrival_rate_per_s": rate, "s": T, "solves_per_s": len(spec) / T,
                "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
                "warnings": sum(1 for r in done.values() if r["rc"] > 0),
                "errors": sum(1 for r in done.values() if r["rc"] < 0)}
            log(f"serve load {load}: {T:.2f}s, p50 {serve['loads'][str(load)]['p50_ms']:.0f} ms "
                f"p99 {serve['loads'][str(load)]['p99_ms']:.0f} ms")
        serve["workload"] = ("Poisson arrivals (seed 2603) at the given fractions of the served mix's capacity "
                             "(its first requests run at once); 75% 2D n in {128,256,512,1024} L=16, 25% 3D n in "
                             "{64,96,128,192} L=10; parameters as the sweep; trap harmonic or 0.5r^2+0.01r^4; "
                             "mixed precision, energy criterion 1e-12; latency = arrival to completion")
        line["serve"] = serve
        del sv

    cpu = None
    if not args.no_cpu_baseline and iters64 is not None:
        log("cpu baseline: timing the oracle ...")
        pb, g0 = inputs.workload_vortex_2d(n=args.n, seed=2602)
        cpu = cpu_baseline(pb, g0, iters64, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} solves/s ({cpu['sample']})")
    line["cpu_baseline"] = cpu
    line["config"] = {
        "workload": (f"2D {args.n}x{args.n} on [-12,12]^2, harmonic trap, Omega=0.6, SOC 1.0, c0=500, c1=-2, "
                     "guess ((x+iy)phi_a, phi_a, phi_a)+1e-3 noise (one seed per solve from 2602); a continuous "
                     f"stream with {B} solves in flight, a step = {B} completions; energy criterion 1e-14; "
                     "mixed FP32->FP64 PCG (double phase with a float search direction: "
                     f"{args.mixed_dir == 'fp32'}), counted against plain FP64 PCG of the same seed"),
        "mixed_dir_precision": args.mixed_dir,
        "parallelism": "single GPU; the running solves of a grid class share every kernel launch",
    }
    line["kernel_source_sha256_16"] = kernel_source_hash()
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
