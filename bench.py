#!/usr/bin/env python3
"""Benchmark: ground-state solves per second of the rotating SOC spin-1 PCG
solver on one MI355X, mixed FP32->FP64 against plain FP64.

Headline (`value`): a step is one batch of B independent solves of the 2D
workload 256x256 on [-12,12]^2, harmonic trap, Omega = 0.6, SOC strength 1.0,
c0 = 500, c1 = -2, initial guess ((x+iy) phi_a, phi_a, phi_a) + 1e-3 complex
noise, seeds 2602 ... 2602+B-1, each to the energy criterion at the paper's
default tolerance 1e-14 (Algorithm 1 with the line search of Algorithm 2). The
guesses are resident in device memory before the timed region; the solves of
a batch share every kernel launch (continuous batching). A mixed solve counts
only when its energy agrees with the plain-FP64 solve of the same seed to
|dE| / max(|E|, 1) < 1e-10.

Further sections of the same JSON line: the same workload one solve at a time
(latency), the 3D 128^3 cascadic-multigrid solve, the 96-solve parameter sweep
of mixed grid sizes, and a served stream with Poisson arrivals.

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
KERNEL_SOURCES = ("paper_2602_17950_amd/csrc/fft_kernels.hip", "paper_2602_17950_amd/csrc/pw_kernels.hip",
                  "paper_2602_17950_amd/csrc/device_common.h", "paper_2602_17950_amd/csrc/control.h",
                  "paper_2602_17950_amd/csrc/gs_internal.h")
TRAFFIC_SUMMARY = "profiles/hbm_traffic_batch256_vortex.md"
SECTIONS = ("batch", "single", "cm3d", "sweep", "table2", "serve")
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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1.0)


def cpu_baseline(pb, psi0, iters_per_solve, seconds):
    """The FP64 CPU oracle on the same input, timed on the host cores for a
    bounded number of PCG iterations and scaled to solves/s by the mean
    iteration count of the GPU's FP64 solves of the workload."""
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
        "sample": (f"first {done} PCG iterations of the seed-2602 256^2 solve on the host "
                   f"({dt:.1f} s, {per_iter * 1e3:.1f} ms/iteration), scaled by the mean "
                   f"{iters_per_solve:.0f} iterations of the GPU's FP64 solves of the workload"),
    }


class Batch:
    """Device-resident guesses and outputs for a list of (Problem, guess)."""

    def __init__(self, torch, probs):
        self.probs = [pb for pb, _ in probs]
        self.guess = [None if g is None else torch.from_numpy(g).to("cuda") for _, g in probs]
        self.out = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device="cuda") for pb in self.probs]

    def requests(self, opt):
        return [(pb, g, o, opt, None) for pb, g, o in zip(self.probs, self.guess, self.out)]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=32, help="solves per headline step")
    ap.add_argument("--n", type=int, default=256, help="grid points per axis of the headline workload")
    ap.add_argument("--kernel", default="pre_inv", help="kernel kind timed for the roofline")
    ap.add_argument("--mixed-dir", choices=("fp32", "fp64"), default="fp32",
                    help="direction precision of the double phase of mixed solves")
    ap.add_argument("--sections", default=",".join(SECTIONS))
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-load", type=float, default=0.5, help="arrival rate / measured sweep capacity")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every solve of these workloads fits one MI355X "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    sections = [s for s in args.sections.split(",") if s]
    for s in sections:
        if s not in SECTIONS:
            sys.exit(f"unknown section {s!r}; choose from {SECTIONS}")

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
    o64 = gs.default_options(precision=gs.GS_FP64, tol=TOL)
    mdir = gs.GS_FP32 if args.mixed_dir == "fp32" else gs.GS_FP64
    omx = gs.default_options(precision=gs.GS_MIXED, tol=TOL, dir_precision=mdir)
    line = {"metric": METRIC, "value": None, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "fp32->fp64", "data": "synthetic"}

    # ------------------------------------------------------------------ headline
    seeds = [2602 + i for i in range(args.batch)]
    work = [inputs.workload_vortex_2d(n=args.n, seed=s) for s in seeds]
    head = Batch(torch, work)
    res64 = None
    if "batch" in sections:
        for w in range(args.warmup):
            t = time.perf_counter()
            ctx.batch_solve(head.requests(omx))
            log(f"warmup {w}: mixed batch of {args.batch} {time.perf_counter() - t:.3f}s")
        # plain FP64 batch: reference energies and the roofline kernel's timing
        ctx.kernel_timer_start(args.kernel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res64 = ctx.batch_solve(head.requests(o64))
        torch.cuda.synchronize()
        T64 = time.perf_counter() - t0
        kt = ctx.kernel_timer_read()
        ctx.kernel_timer_start(None)
        E64 = [r["E"] for r in res64]
        log(f"fp64 batch: {T64:.3f}s iters mean {np.mean([r['iters'] for r in res64]):.0f} "
            f"max {max(r['iters'] for r in res64)}")
        # timed region: K mixed batches
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resmx = []
        for k in range(args.steps):
            resmx.append(ctx.batch_solve(head.requests(omx)))
        torch.cuda.synchronize()
        Tmx = time.perf_counter() - t0
        dEs = [rel(r["E"], e) for rs in resmx for r, e in zip(rs, E64)]
        counted = sum(1 for d in dEs if d < DE_GATE)
        lat = [r["wall_s"] for rs in resmx for r in rs]
        itmx = [r["iters"] for rs in resmx for r in rs]
        log(f"mixed batches: {Tmx:.3f}s for {args.steps} x {args.batch}; counted {counted}; "
            f"iters mean {np.mean(itmx):.0f} max {max(itmx)}")
        line["value"] = counted / Tmx
        line["ms_per_step"] = Tmx / args.steps * 1e3
        line["p50_ms"] = percentile(lat, 50) * 1e3
        line["p99_ms"] = percentile(lat, 99) * 1e3
        line["iters_per_s"] = sum(itmx) / Tmx
        line["batch"] = {
            "solves_per_step": args.batch, "counted": counted, "solves": len(dEs),
            "dE_rel_max": max(dEs), "dE_rel_median": float(np.median(dEs)),
            "mixed_iters_mean": float(np.mean(itmx)), "mixed_iters_fp32_mean":
                float(np.mean([r["iters_fp32"] for rs in resmx for r in rs])),
            "fp64_solves_per_s": args.batch / T64, "fp64_iters_mean": float(np.mean([r["iters"] for r in res64])),
            "fp64_p50_ms": percentile([r["wall_s"] for r in res64], 50) * 1e3,
            "fp64_p99_ms": percentile([r["wall_s"] for r in res64], 99) * 1e3,
            "speedup_mixed_vs_fp64": (len(dEs) / Tmx) / (args.batch / T64),
            "latency_note": "p50/p99: submission to completion of each solve inside its batch",
        }
        roof = None
        if kt["launches"] > 0 and kt["ms"] > 0:
            avg_s = kt["ms"] * 1e-3 / kt["launches"]
            bpl = kt["bytes"] / kt["launches"]
            achieved = bpl / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.kernel),
                    "kernel": args.kernel, "launches": kt["launches"], "avg_us": avg_s * 1e6,
                    "bytes_per_launch": bpl, "timed_in": f"FP64 batch of {args.batch} solves"}
        line["roofline"] = roof

    # ------------------------------------------------------------ single solve
    if "single" in sections:
        pb, g0 = work[0]
        one = Batch(torch, [(pb, g0)])
        single = {}
        for name, opt in (("fp64", o64), ("mixed", omx)):
            ctx.solve_device(pb, one.guess[0], one.out[0], opt)   # warm
            lat, r = [], None
            for k in range(args.steps):
                t = time.perf_counter()
                r = ctx.solve_device(pb, one.guess[0], one.out[0], opt)
                lat.append(time.perf_counter() - t)
            single[name] = {"solves_per_s": len(lat) / sum(lat), "p50_ms": percentile(lat, 50) * 1e3,
                            "p99_ms": percentile(lat, 99) * 1e3, "iters": r["iters"],
                            "iters_fp32": r["iters_fp32"], "E": r["E"]}
            log(f"single {name}: {single[name]['p50_ms']:.1f} ms, iters {r['iters']}")
        single["dE_rel"] = rel(single["mixed"]["E"], single["fp64"]["E"])
        single["speedup_mixed_vs_fp64"] = single["mixed"]["solves_per_s"] / single["fp64"]["solves_per_s"]
        line["single"] = single
        if line["value"] is None:   # headline section skipped
            line["value"] = single["mixed"]["solves_per_s"] if single["dE_rel"] < DE_GATE else 0.0
            line["ms_per_step"] = single["mixed"]["p50_ms"]

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

    # ------------------------------------------------------------------- sweep
    cap = None
    if "sweep" in sections:
        spec = inputs.workload_sweep_2d()
        sw = Batch(torch, [(pb, inputs.initial_guess(pb, k)) for pb, k in spec])
        out = {}
        E = {}
        for name, prec in (("fp64", gs.GS_FP64), ("mixed", gs.GS_MIXED)):
            opt = gs.default_options(precision=prec, tol=1e-12,
                                     dir_precision=mdir if prec == gs.GS_MIXED else gs.GS_FP64)
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
        out["workload"] = ("96 2D solves, n uniform over {128,256,512}, L=16, Omega~U[0,0.9], SOC~U[0,2], "
                           "c0~U[100,2000], c1~U[-5,5], guesses over {(a,a,a),(b,a,a),(f,f,f)}, seed 17950; "
                           "energy criterion 1e-12, one batch")
        out["note"] = ("solves whose mixed and FP64 runs end in different local minima are not counted "
                       "(the landscape of the rotating problems has many)")
        line["sweep"] = out
        cap = out["mixed"]["solves_per_s"]
        del sw

    # ------------------------------------------------------------------ table2
    if "table2" in sections:
        tb = {"rows": {}}
        total, nsolve, allmatch = 0.0, 0, True
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
            total += dt
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
        tb.update({"s": total, "solves": nsolve, "solves_per_s": nsolve / total, "all_match": allmatch,
                   "workload": ("Table 2 (Example 3): for Omega in {0.6,0.7,0.8,0.9}, the 1000 component-wise "
                                "combinations of the ten guesses of Sec. 4 on [-12,12]^2 (gamma 0.3, c0 50, "
                                "c1 0.5), each solved by CM-PCG 64^2->128^2->256^2, mixed precision, energy "
                                "criterion 1e-14; one batch per Omega; the lowest energy is the ground state")})
        line["table2"] = tb

    # ------------------------------------------------------------------- serve
    if "serve" in sections:
        rate = args.serve_load * (cap if cap else 1.0)
        spec = inputs.workload_serve(args.serve_requests)
        sv = Batch(torch, [(pb, inputs.initial_guess(pb, k)) for pb, k in spec])
        rng = np.random.default_rng(2603)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(spec)))
        opt = gs.default_options(precision=gs.GS_MIXED, tol=1e-12, dir_precision=mdir)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending, tickets, done = 0, {}, {}
        while len(done) < len(spec):
            now = time.perf_counter() - t0
            while pending < len(spec) and arrivals[pending] <= now:
                i = pending
                tickets[i] = ctx.submit(sv.probs[i], sv.guess[i], sv.out[i], opt)
                pending += 1
            for i in list(tickets):
                r = ctx.poll(tickets[i])
                if r is not None:
                    done[i] = r
                    del tickets[i]
            if len(done) < len(spec):
                if tickets:
                    ctx.progress(block=pending >= len(spec) or arrivals[pending] > time.perf_counter() - t0 + 0.005)
                else:
                    time.sleep(max(0.0, min(0.01, arrivals[pending] - (time.perf_counter() - t0))))
        T = time.perf_counter() - t0
        lat = [done[i]["wall_s"] for i in range(len(spec))]
        line["serve"] = {
            "requests": len(spec), "arrival_rate_per_s": rate, "load_vs_sweep_capacity": args.serve_load,
            "s": T, "solves_per_s": len(spec) / T, "p50_ms": percentile(lat, 50) * 1e3,
            "p99_ms": percentile(lat, 99) * 1e3,
            "warnings": sum(1 for r in done.values() if r["rc"] > 0),
            "errors": sum(1 for r in done.values() if r["rc"] < 0),
            "workload": ("Poisson arrivals (seed 2603); 75% 2D n in {128,256,512,1024} L=16, 25% 3D n in {64,96,128,192} "
                         "L=10; parameters as the sweep; trap harmonic or 0.5r^2+0.01r^4; mixed precision, "
                         "energy criterion 1e-12; latency = arrival to completion"),
        }
        log(f"serve: {T:.2f}s, p50 {line['serve']['p50_ms']:.0f} ms p99 {line['serve']['p99_ms']:.0f} ms")
        del sv

    cpu = None
    if not args.no_cpu_baseline and res64 is not None:
        log("cpu baseline: timing the oracle ...")
        cpu = cpu_baseline(work[0][0], work[0][1], float(np.mean([r["iters"] for r in res64])), args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} solves/s ({cpu['sample']})")
    line["cpu_baseline"] = cpu
    line["config"] = {
        "workload": (f"2D {args.n}x{args.n} on [-12,12]^2, harmonic trap, Omega=0.6, SOC 1.0, c0=500, c1=-2, "
                     "guess ((x+iy)phi_a, phi_a, phi_a)+1e-3 noise; a step = one batch of "
                     f"{args.batch} solves (noise seeds 2602..{2601 + args.batch}), energy criterion 1e-14; "
                     "mixed FP32->FP64 PCG (double phase with a float search direction: "
                     f"{args.mixed_dir == 'fp32'}), counted against plain FP64 PCG of the same seed"),
        "mixed_dir_precision": args.mixed_dir,
        "parallelism": "single GPU; the solves of a batch share every kernel launch",
    }
    line["kernel_source_sha256_16"] = kernel_source_hash()
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
