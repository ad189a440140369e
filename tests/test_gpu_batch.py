"""Batching and serving through the C ABI.

A solve occupies its own slot; slots of one grid class share every launch but
no arithmetic, and every reduction has a fixed per-slot order. So a solve must
return the same bits alone, in a batch of mixed sizes and precisions, and
under staggered (served) submission; these tests compare bit for bit. Parity
of the solve itself with the CPU oracle is covered by the single-solve tests
and by a batch-vs-oracle check on the smallest problems here.
"""
import os

import numpy as np
import pytest
import torch

from paper_2602_17950_amd import gs, inputs

from helpers import orc, rel
import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def problems():
    """Small problems of three grid classes (two 2D sizes and a 3D one),
    rotating and not, with seeded guesses."""
    out = []
    specs = [
        (2, (32, 32), (6.0, 6.0), 0.0, 0.5, 60.0, -0.5, ("a", "a", "a")),
        (2, (32, 32), (6.0, 6.0), 0.3, 0.8, 90.0, 0.7, ("b", "a", "a")),
        (2, (64, 64), (8.0, 8.0), 0.5, 1.0, 150.0, -1.0, ("b", "a", "a")),
        (2, (64, 64), (8.0, 8.0), 0.0, 0.3, 40.0, 1.5, ("a", "bbar", "a")),
        (3, (16, 16, 16), (5.0, 5.0, 5.0), 0.2, 0.6, 30.0, -0.3, ("a", "a", "a")),
    ]
    for i, (dim, n, L, om, ga, c0, c1, kinds) in enumerate(specs):
        pb = inputs.Problem(dim=dim, n=n, L=L, omega=om, gamma=ga, c0=c0, c1=c1)
        psi0 = inputs.initial_guess(pb, kinds, noise=1e-3, seed=100 + i)
        out.append((pb, psi0))
    return out


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def alone(ctx, pb, psi0, opt):
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    res = ctx.solve_device(pb, dev(psi0), out, options=opt)
    torch.cuda.synchronize()
    return out, res


def same_bits(a, b):
    return torch.equal(a.view(torch.float64), b.view(torch.float64))


@pytest.mark.parametrize("precision,dirp", [(gs.GS_FP64, gs.GS_FP64), (gs.GS_MIXED, gs.GS_FP64),
                                           (gs.GS_FP64, gs.GS_FP32), (gs.GS_MIXED, gs.GS_FP32)])
def test_batch_equals_alone_bitwise(gpu_ctx, precision, dirp):
    print(f"[batch] precision={precision} dir_precision={dirp}", flush=True)
    opt = gs.default_options(precision=precision, tol=1e-11, switch_resid=1e-4, dir_precision=dirp)
    probs = problems()
    ref = [alone(gpu_ctx, pb, psi0, opt) for pb, psi0 in probs]
    outs = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for pb, _ in probs]
    reqs = [(pb, dev(psi0), o, opt, None) for (pb, psi0), o in zip(probs, outs)]
    res = gpu_ctx.batch_solve(reqs)
    torch.cuda.synchronize()
    for i, ((o_ref, r_ref), o, r) in enumerate(zip(ref, outs, res)):
        assert r["rc"] >= 0 and r_ref["rc"] >= 0, (i, r, r_ref)
        assert same_bits(o, o_ref), i
        for k in ("E", "mu", "resid_inf", "iters", "iters_fp32", "backtracks", "dE_last"):
            assert r[k] == r_ref[k], (i, k, r[k], r_ref[k])
        if precision == gs.GS_MIXED:
            assert 0 < r["iters_fp32"] < r["iters"], i
    st = gpu_ctx.memory_stats()
    assert st["reserved"] == 0


def test_batch_matches_oracle_small(gpu_ctx):
    """Converged energies and chemical potentials of batched FP64 solves against
    the oracle from the same guesses (2D problems; residual stop for mu)."""
    probs = problems()[:2]
    opt = gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-10)
    outs = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for pb, _ in probs]
    res = gpu_ctx.batch_solve([(pb, dev(p0), o, opt, None) for (pb, p0), o in zip(probs, outs)])
    for (pb, psi0), r in zip(probs, res):
        g, t, p = orc(pb)
        ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-10))
        ev = O.evaluate(g, t, p, ref.psi)
        assert r["rc"] == gs.GS_OK and ref.status == 0
        assert rel(r["E"], ev["E"]) < 1e-10
        assert rel(r["mu"], ev["mu"]) < 1e-9


def test_serving_staggered_submission(gpu_ctx):
    """Requests that arrive while others run are admitted at chunk boundaries;
    each result equals the solve alone."""
    opt = gs.default_options(precision=gs.GS_MIXED, tol=1e-11, switch_resid=1e-4, check_every=8)
    probs = problems()
    ref = [alone(gpu_ctx, pb, psi0, opt) for pb, psi0 in probs]
    outs = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for pb, _ in probs]
    guesses = [dev(psi0) for _, psi0 in probs]
    tickets = []
    for i, (pb, _) in enumerate(probs):
        tickets.append(gpu_ctx.submit(pb, guesses[i], outs[i], opt))
        # let the earlier requests run a few chunks before the next arrives
        for _ in range(3):
            gpu_ctx.progress(block=True)
    done = {}
    while len(done) < len(tickets):
        for i, t in enumerate(tickets):
            if i in done:
                continue
            r = gpu_ctx.poll(t)
            if r is not None:
                done[i] = r
        if len(done) < len(tickets):
            gpu_ctx.progress(block=True)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        assert done[i]["rc"] >= 0
        assert same_bits(outs[i], ref[i][0]), i
        assert done[i]["E"] == ref[i][1]["E"]
        assert done[i]["wall_s"] > 0
    assert gpu_ctx.memory_stats()["reserved"] == 0


@pytest.mark.timeout(400)
def test_served_mix_subset(gpu_ctx):
    """Requests of the served stream itself (its first ten with a 2D grid of at
    most 256^2 or a 3D grid of 64^3; harmonic and harmonic-plus-quartic traps,
    the served options): each submitted while the earlier ones run, each result
    bit for bit the solve alone, and the final states of the 128^2 and 64^3
    requests evaluated by the oracle (E, mu to 1e-10, the residual)."""
    spec = inputs.workload_serve(400)
    idx = [i for i, (pb, _) in enumerate(spec)
           if (pb.dim == 2 and pb.n[0] <= 256) or (pb.dim == 3 and pb.n[0] <= 64)][:10]
    opt = gs.default_options(precision=gs.GS_MIXED, tol=1e-12, dir_precision=gs.GS_FP32)
    work = [(spec[i][0], inputs.initial_guess(spec[i][0], spec[i][1])) for i in idx]
    guesses = [dev(psi0) for _, psi0 in work]
    outs = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for pb, _ in work]
    print(f"[serve subset] requests {idx}", flush=True)
    tickets = []
    for k, (pb, _) in enumerate(work):
        tickets.append(gpu_ctx.submit(pb, guesses[k], outs[k], opt))
        for _ in range(2):
            gpu_ctx.progress(block=True)
    done = {}
    while len(done) < len(tickets):
        for k, t in enumerate(tickets):
            if k not in done:
                r = gpu_ctx.poll(t)
                if r is not None:
                    done[k] = r
        if len(done) < len(tickets):
            gpu_ctx.progress(block=True)
    torch.cuda.synchronize()
    O.set_threads(min(16, os.cpu_count() or 1))
    try:
        for k, (pb, psi0) in enumerate(work):
            ref, rref = alone(gpu_ctx, pb, psi0, opt)
            r = done[k]
            print(f"[serve subset] {idx[k]}: {pb.dim}D {pb.n[0]} q4={pb.q4} rc={r['rc']} E={r['E']!r} "
                  f"it={r['iters']}", flush=True)
            assert r["rc"] >= 0
            assert same_bits(outs[k], ref) and r["E"] == rref["E"], idx[k]
            small = (pb.dim == 2 and pb.n[0] <= 128) or (pb.dim == 3 and pb.n[0] <= 64)
            if small:
                g, t, p = orc(pb)
                ev = O.evaluate(g, t, p, outs[k].cpu().numpy())
                assert rel(r["E"], ev["E"]) < 1e-10, (idx[k], r["E"], ev["E"])
                assert rel(r["mu"], ev["mu"]) < 1e-10, (idx[k], r["mu"], ev["mu"])
                assert abs(r["resid_inf"] - ev["resid_inf"]) < 1e-9 + 1e-6 * ev["resid_inf"]
    finally:
        O.set_threads(1)


def test_admission_by_footprint(gpu_ctx):
    """With a budget that fits one request, requests run one at a time and all
    complete with the bits of the solve alone."""
    ctx = gs.Context(0)
    try:
        opt = gs.default_options(tol=1e-11)
        probs = [p for p in problems() if p[0].n == (32, 32)]
        need = gs.footprint_bytes(probs[0][0], gs.GS_FP64)
        ref = [alone(ctx, pb, psi0, opt) for pb, psi0 in probs]
        ctx.set_hbm_budget(need + need // 2)
        outs = [torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for pb, _ in probs]
        # the guesses are read when each request is admitted: hold them until then
        guesses = [dev(p0) for _, p0 in probs]
        tickets = [ctx.submit(pb, g0, o, opt) for (pb, _), g0, o in zip(probs, guesses, outs)]
        peak = 0
        results = {}
        while len(results) < len(tickets):
            st = ctx.memory_stats()
            assert st["reserved"] <= st["budget"]
            assert st["allocated"] <= st["budget"]
            peak = max(peak, st["reserved"])
            for i, t in enumerate(tickets):
                if i not in results:
                    r = ctx.poll(t)
                    if r is not None:
                        results[i] = r
            if len(results) < len(tickets):
                ctx.progress(block=True)
        assert peak <= need + need // 2
        torch.cuda.synchronize()
        for i in range(len(probs)):
            assert results[i]["rc"] >= 0
            assert same_bits(outs[i], ref[i][0])
        # a request larger than the whole budget is refused at submission
        big = inputs.Problem(dim=2, n=(256, 256), L=(12.0, 12.0))
        o = torch.empty((3, 256, 256), dtype=torch.complex128, device=DEV)
        with pytest.raises(gs.GsError) as ei:
            ctx.submit(big, None, o, opt)
        assert ei.value.code == gs.GS_ENOMEM
    finally:
        ctx.close()


def test_cancel(gpu_ctx):
    pb, psi0 = problems()[2]
    opt = gs.default_options(tol=0.0, max_iter=100000, check_every=4)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    g0 = dev(psi0)
    t = gpu_ctx.submit(pb, g0, out, opt)
    gpu_ctx.progress(block=True)
    gpu_ctx.cancel(t)
    r = gpu_ctx.wait(t)
    assert r["rc"] == gs.GS_ECANCELED
    with pytest.raises(gs.GsError):
        gpu_ctx.poll(t)   # the ticket was released
    assert gpu_ctx.memory_stats()["reserved"] == 0


def test_cancel_mixed_after_hand_over(gpu_ctx):
    """A mixed request is cancelled around its hand-over to the double-state
    class (switch_resid = 1 hands over after its first float step; it waits in
    the double class's queue while that class runs a chunk of request B). The
    slot it held is taken by a later request C, whose result must equal C
    alone bit for bit, as must B's: the hand-over copy into the released slot
    is ordered before the slot's next use."""
    pb, p0 = problems()[2]
    pc, pc0 = problems()[3]   # the same 64^2 grid class
    optB = gs.default_options(tol=1e-11, check_every=4)
    optA = gs.default_options(precision=gs.GS_MIXED, tol=0.0, max_iter=100000, switch_resid=1.0,
                              check_every=4)
    optC = gs.default_options(tol=1e-11, check_every=4)
    refB = alone(gpu_ctx, pb, p0, optB)
    refC = alone(gpu_ctx, pc, pc0, optC)
    gB, gA, gC = dev(p0), dev(p0), dev(pc0)
    oB, oA, oC = (torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV) for _ in range(3))
    tB = gpu_ctx.submit(pb, gB, oB, optB)
    tA = gpu_ctx.submit(pb, gA, oA, optA)
    for _ in range(2):
        gpu_ctx.progress(block=True)
    gpu_ctx.cancel(tA)
    tC = gpu_ctx.submit(pc, gC, oC, optC)
    rA, rB, rC = gpu_ctx.wait(tA), gpu_ctx.wait(tB), gpu_ctx.wait(tC)
    torch.cuda.synchronize()
    assert rA["rc"] == gs.GS_ECANCELED
    assert rB["rc"] >= 0 and rC["rc"] >= 0
    assert same_bits(oB, refB[0]) and rB["E"] == refB[1]["E"]
    assert same_bits(oC, refC[0]) and rC["E"] == refC[1]["E"]
    assert gpu_ctx.memory_stats()["reserved"] == 0


def test_batch_invalid_request_runs_nothing(gpu_ctx):
    pb, psi0 = problems()[0]
    opt = gs.default_options()
    bad = inputs.Problem(dim=2, n=(40, 40), L=(6.0, 6.0))
    o1 = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    o2 = torch.empty((3, 48, 48), dtype=torch.complex128, device=DEV)
    with pytest.raises(gs.GsError) as ei:
        gpu_ctx.batch_solve([(pb, dev(psi0), o1, opt, None), (bad, None, o2, opt, None)])
    assert ei.value.code == gs.GS_EINVAL
    assert "request 1" in str(ei.value)
    assert gpu_ctx.progress() == 0


# ---------------------------------------------------------------------------
# cascadic multigrid (Algorithm 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,nc,nf,L", [
    (2, (16, 32), (64, 32), (5.0, 7.0)),
    (2, (32, 32), (64, 64), (8.0, 8.0)),
    (3, (16, 16, 16), (32, 16, 32), (5.0, 5.0, 6.0)),
])
def test_interpolate_matches_oracle(gpu_ctx, dim, nc, nf, L):
    from helpers import smooth_field
    pc = inputs.Problem(dim=dim, n=nc, L=L)
    x = smooth_field(pc, seed=5, noise=0.3)
    gc, gf = O.Grid(dim, nc, L), O.Grid(dim, nf, L)
    ref = O.interp(gc, x, gf)
    out = torch.empty((3,) + tuple(reversed(nf)), dtype=torch.complex128, device=DEV)
    gpu_ctx.interpolate(gs.make_grid(dim, nc, L), dev(x), gs.make_grid(dim, nf, L), out)
    got = out.cpu().numpy()
    assert rel(got, ref) < 1e-13


def _cm_problem(dim):
    if dim == 2:
        pb = inputs.Problem(dim=2, n=(64, 64), L=(8.0, 8.0), omega=0.4, gamma=0.7, c0=120.0, c1=-1.0)
        pc = inputs.Problem(dim=2, n=(32, 32), L=(8.0, 8.0), omega=0.4, gamma=0.7, c0=120.0, c1=-1.0)
    else:
        pb = inputs.Problem(dim=3, n=(32, 32, 32), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                            gamma=1.0, c0=200.0, c1=5.0)
        pc = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                            gamma=1.0, c0=200.0, c1=5.0)
    return pb, pc, inputs.initial_guess(pc, ("a", "a", "a"))


@pytest.mark.parametrize("dim", [2, 3])
def test_cm_solve_matches_oracle(gpu_ctx, dim):
    """Two-level cascadic multigrid: the coarse level from the Gaussian guess,
    the fine level from its interpolant; energies, chemical potential and the
    coarse-level iteration count against the oracle's Algorithm 3."""
    print(f"[cm] dim={dim}", flush=True)
    pb, pc, psi0 = _cm_problem(dim)
    tol = 1e-10
    g_f, t, p = orc(pb)
    g_c, _, _ = orc(pc)
    O.set_threads(min(16, os.cpu_count() or 1))   # the 3-D oracle solve takes minutes on one thread
    try:
        rs = O.cmpcg([g_c, g_f], lambda gg: t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol))
        ev = O.evaluate(g_f, t, p, rs[-1].psi)
    finally:
        O.set_threads(1)
    opt = gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol, cm_levels=2)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    r = gpu_ctx.solve_device(pb, dev(psi0), out, options=opt)
    print(f"[cm] gpu E={r['E']!r} it={r['iters']}+{r['iters_coarse']} | oracle E={ev['E']!r} "
          f"it={rs[1].iters}+{rs[0].iters}", flush=True)
    assert r["rc"] == gs.GS_OK and rs[-1].status == 0
    assert rel(r["E"], ev["E"]) < 1e-10
    assert rel(r["mu"], ev["mu"]) < 1e-8
    assert r["iters_coarse"] > 0 and r["iters"] > 0
    assert abs(sum(r["norm_comp"]) - 1.0) < 1e-13


def test_cm_mixed_batch_equals_alone(gpu_ctx):
    """Cascadic multigrid with mixed precision (each level float then double),
    batched with plain solves: bitwise the same as alone."""
    pb, pc, psi0 = _cm_problem(2)
    opt_cm = gs.default_options(precision=gs.GS_MIXED, tol=1e-11, switch_resid=1e-4, cm_levels=2)
    ref, rref = alone(gpu_ctx, pb, psi0, opt_cm)
    others = problems()[:3]
    opt = gs.default_options(precision=gs.GS_MIXED, tol=1e-11, switch_resid=1e-4)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    reqs = [(pb, dev(psi0), out, opt_cm, None)]
    outs = []
    for q, g0 in others:
        o = torch.empty((3,) + q.shape, dtype=torch.complex128, device=DEV)
        outs.append(o)
        reqs.append((q, dev(g0), o, opt, None))
    res = gpu_ctx.batch_solve(reqs)
    torch.cuda.synchronize()
    assert res[0]["rc"] >= 0 and rref["rc"] >= 0
    assert same_bits(out, ref)
    assert res[0]["E"] == rref["E"] and res[0]["iters_coarse"] == rref["iters_coarse"] > 0


def test_cm_rejects_bad_levels(gpu_ctx):
    pb, pc, psi0 = _cm_problem(2)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    with pytest.raises(gs.GsError) as ei:
        gpu_ctx.solve_device(pb, None, out, options=gs.default_options(cm_levels=4))   # 64/8 < 16
    assert ei.value.code == gs.GS_EINVAL
    V = np.zeros(pb.shape)
    with pytest.raises(gs.GsError) as ei:
        gpu_ctx.solve_device(pb, None, out, options=gs.default_options(cm_levels=2), V=V)
    assert ei.value.code == gs.GS_EINVAL
