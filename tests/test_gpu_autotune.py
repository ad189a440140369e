"""The autotuner of the FFT pass schedules.

Every candidate schedule of a pass (lines and threads per block) computes the
same bits: a line's transform does not depend on how its butterflies are
spread over threads, and the reducing passes sum in wave chunks of 64 points.
A tuning chunk cycles through the candidates inside real iterations, so a
solve run with autotuning on (several candidates during its first chunk) must
return exactly the bits of the same solve on the fixed table.
"""
import numpy as np
import pytest
import torch

from paper_2602_17950_amd import gs, inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _cases():
    out = []
    for dim, n, L, om, ga, c0, c1, kinds in [
        (2, (256, 256), (12.0, 12.0), 0.6, 1.0, 500.0, -2.0, ("b", "a", "a")),
        (2, (128, 128), (10.0, 10.0), 0.3, 0.8, 200.0, 1.0, ("a", "b", "a")),
        (2, (48, 96), (6.0, 8.0), 0.2, 0.5, 80.0, -0.5, ("b", "a", "a")),
        (3, (32, 32, 32), (6.0, 6.0, 6.0), 0.5, 1.0, 200.0, 5.0, ("a", "a", "a")),
        # 2400-point x lines (radix-5 passes, tiles of one or two lines)
        (2, (2400, 32), (20.0, 4.0), 0.2, 0.5, 100.0, 1.0, ("a", "a", "a")),
    ]:
        pb = inputs.Problem(dim=dim, n=n, L=L, omega=om, gamma=ga, c0=c0, c1=c1)
        out.append((pb, inputs.initial_guess(pb, kinds, noise=1e-3, seed=7)))
    return out


@pytest.mark.parametrize("prec,dirp", [(gs.GS_FP64, gs.GS_FP64), (gs.GS_MIXED, gs.GS_FP32)])
def test_tuned_schedules_give_the_same_bits(prec, dirp):
    opt = gs.default_options(precision=prec, dir_precision=dirp, tol=0.0, max_iter=96, switch_resid=1e-3)
    outs = {}
    reports = {}
    for tune in (0, 1):
        with gs.Context(0) as ctx:
            ctx.set_autotune(tune)
            probs = _cases()
            guesses = [torch.from_numpy(p0).to(DEV) for _, p0 in probs]
            res = [torch.empty_like(g) for g in guesses]
            rs = ctx.batch_solve([(pb, g, o, opt, None) for (pb, _), g, o in zip(probs, guesses, res)])
            torch.cuda.synchronize()
            outs[tune] = (res, rs)
            reports[tune] = ctx.autotune_report()
    for i, (a, b) in enumerate(zip(outs[0][0], outs[1][0])):
        assert torch.equal(torch.view_as_real(a), torch.view_as_real(b)), i
        assert outs[0][1][i]["E"] == outs[1][1][i]["E"]
        assert outs[0][1][i]["iters"] == outs[1][1][i]["iters"]
    assert reports[0] == []
    rep = reports[1]
    print("[autotune]", rep, flush=True)
    grids = {tuple(r["grid"]) for r in rep}
    assert (256, 256, 1) in grids and (32, 32, 32) in grids and (2400, 32, 1) in grids
    assert any(r["decided"] for r in rep)
    for r in rep:
        for name, p in r["passes"].items():
            assert p["chosen"] in p["us"], (name, p)
            if r["decided"] and p["us"][p["chosen"]] > 0:
                timed = [v for v in p["us"].values() if v > 0]
                assert p["us"][p["chosen"]] == min(timed), (name, p)
