#!/usr/bin/env python3
"""Benchmark: ground-state solves per second of the rotating SOC spin-1 PCG
solver on one MI355X, mixed FP32->FP64 against plain FP64.

A step is one complete ground-state solve (Algorithm 1 with the line search of
Algorithm 2, to the energy criterion at the paper's default tolerance 1e-14) of
the 2D workload
256x256 on [-12,12]^2, harmonic trap, Omega = 0.6, SOC strength 1.0,
c0 = 500, c1 = -2, initial guess ((x+iy) phi_a, phi_a, phi_a) + 1e-3 complex
noise (seed 2602). The initial guess is resident in device memory before the
timed region. A mixed solve counts only when its energy agrees with the
plain-FP64 solve of the same input to |dE| / max(|E|, 1) < 1e-10.

Prints one JSON line (see the keys below); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
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
KERNEL_SOURCES = ("paper_2602_17950_amd/csrc/fft_kernels.hip", "paper_2602_17950_amd/csrc/gs_internal.h")
TRAFFIC_SUMMARY = "profiles/hbm_traffic_solve256_vortex.md"


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the summary is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(rf"traffic_bytes_per_launch\[{re.escape(kernel)}\]:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * len(xs) + 0.5)) - 1))
    return xs[k]


def cpu_baseline(pb, psi0, iters_per_solve, seconds):
    """The FP64 CPU oracle on the same input, timed on the host cores for a
    bounded number of PCG iterations and scaled to solves/s by the iteration
    count of the FP64 solve."""
    import oracle as O
    threads = max(1, min(16, os.cpu_count() or 1))
    O.set_threads(threads)
    g = O.Grid(pb.dim, pb.n, pb.L)
    t = O.Trap(pb.g, pb.q2, pb.q4)
    p = O.Params(pb.omega, pb.gamma, pb.c0, pb.c1)
    probe = 3
    t0 = time.perf_counter()
    O.pcg(g, t, p, psi0, O.Options(tol=1e-12, max_iter=probe))
    t_probe = time.perf_counter() - t0
    k = int(max(probe + 2, min(2000, seconds / max(t_probe / probe, 1e-6))))
    t0 = time.perf_counter()
    r = O.pcg(g, t, p, psi0, O.Options(tol=1e-12, max_iter=k))
    dt = time.perf_counter() - t0
    done = max(1, r.iters)
    per_iter = dt / done
    return {
        "value": 1.0 / (per_iter * iters_per_solve),
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first {done} PCG iterations of the same 256^2 solve on the host "
                   f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration), scaled by the "
                   f"{iters_per_solve} iterations of the FP64 solve"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis")
    ap.add_argument("--kernel", default="hl_inv", help="kernel kind timed for the roofline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every solve of this workload fits one MI355X "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

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

    pb, psi0 = inputs.workload_vortex_2d(n=args.n)
    ctx = gs.Context(0)
    stream = torch.cuda.Stream()
    d_psi0 = torch.from_numpy(psi0).to("cuda")
    out = torch.empty_like(d_psi0)
    o64 = gs.default_options(precision=gs.GS_FP64, stop_kind=gs.GS_STOP_ENERGY, tol=TOL)
    omx = gs.default_options(precision=gs.GS_MIXED, stop_kind=gs.GS_STOP_ENERGY, tol=TOL)

    def run(opts):
        return ctx.solve_device(pb, d_psi0, out, opts, stream=stream.cuda_stream)

    for w in range(args.warmup):
        r = run(o64)
        log(f"warmup {w}: fp64 E={r['E']:.15f} iters={r['iters']} {r['wall_s']:.3f}s")
        r = run(omx)
        log(f"warmup {w}: mixed E={r['E']:.15f} iters={r['iters']} ({r['iters_fp32']} fp32) {r['wall_s']:.3f}s")

    # plain FP64 PCG: the reference energy and the speedup denominator; the
    # roofline kernel is timed here (HIP events on the solve's stream), where
    # every launch is the double-precision variant
    ctx.kernel_timer_start(args.kernel)
    torch.cuda.synchronize()
    lat64, res64 = [], None
    t0 = time.perf_counter()
    for k in range(args.steps):
        t = time.perf_counter()
        res64 = run(o64)
        lat64.append(time.perf_counter() - t)
        log(f"fp64 {k}: E={res64['E']:.15f} iters={res64['iters']} {lat64[-1]:.3f}s")
    torch.cuda.synchronize()
    T64 = time.perf_counter() - t0
    E64 = res64["E"]
    kt = ctx.kernel_timer_read()
    ctx.kernel_timer_start(None)

    # mixed FP32 -> FP64: the timed region of the metric
    torch.cuda.synchronize()
    latmx, resmx = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        t = time.perf_counter()
        resmx.append(run(omx))
        latmx.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    Tmx = time.perf_counter() - t0
    for k, r in enumerate(resmx):
        log(f"mixed {k}: E={r['E']:.15f} iters={r['iters']} ({r['iters_fp32']} fp32) {latmx[k]:.3f}s")

    dEs = [abs(r["E"] - E64) / max(abs(E64), 1.0) for r in resmx]
    counted = sum(1 for d in dEs if d < DE_GATE)
    value = counted / Tmx
    iters_mx = sum(r["iters"] for r in resmx)

    roof = None
    if kt["launches"] > 0 and kt["ms"] > 0:
        avg_s = kt["ms"] * 1e-3 / kt["launches"]
        bpl = kt["bytes"] / kt["launches"]
        achieved = bpl / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.kernel), "kernel": args.kernel,
                "launches": kt["launches"], "avg_us": avg_s * 1e6, "bytes_per_launch": bpl,
                "timed_in": "plain FP64 solves"}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the oracle ...")
        cpu = cpu_baseline(pb, psi0, res64["iters"], args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} solves/s ({cpu['sample']})")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": Tmx / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32->fp64",
        "data": "synthetic",
        "config": {
            "workload": (f"2D {args.n}x{args.n} on [-12,12]^2, harmonic trap, Omega=0.6, SOC 1.0, "
                         "c0=500, c1=-2, guess ((x+iy)phi_a, phi_a, phi_a)+1e-3 noise (seed 2602), "
                         "energy criterion 1e-14; mixed FP32->FP64 PCG vs plain FP64 PCG"),
            "parallelism": "single GPU, one solve at a time",
        },
        "p50_ms": percentile(latmx, 50) * 1e3,
        "p99_ms": percentile(latmx, 99) * 1e3,
        "iters_per_s": iters_mx / Tmx,
        "mixed": {"iters": resmx[-1]["iters"], "iters_fp32": resmx[-1]["iters_fp32"],
                  "E": resmx[-1]["E"], "dE_rel_max": max(dEs), "counted": counted},
        "fp64": {"solves_per_s": args.steps / T64, "ms_per_solve": T64 / args.steps * 1e3,
                 "iters": res64["iters"], "E": E64,
                 "p50_ms": percentile(lat64, 50) * 1e3, "p99_ms": percentile(lat64, 99) * 1e3},
        "speedup_mixed_vs_fp64": (args.steps / Tmx) / (args.steps / T64),
        "roofline": roof,
        "kernel_source_sha256_16": kernel_source_hash(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
