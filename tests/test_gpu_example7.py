"""Example 7, anisotropic cases: 3D harmonic trap with gamma = (0.97, 1.03,
0.05), c0 = 3000, c1 = 1 on the elongated domain [-10,10]^2 x [-80,80], by
cascadic multigrid (Algorithm 3) from 64^3 to 256^3 as the paper runs it.

The z axis is 16 times longer than the x and y axes, so the three axes have
different wavenumber spacings in every spectral symbol. A same-guess oracle
solve at 256^3 would take hours of host time, so the oracle evaluates the GPU's
final state: E and its parts, mu and mu_l, N_l, the residual and the virial
residual of that state must equal what the GPU reports, and the virial
identity of Sec. 2.2 (which holds for any harmonic trap) must be met at
convergence. Guess: the Thomas-Fermi profile (guess (f) of Sec. 4) on the
coarsest grid, whose extent along z (about 56) fits the domain.
"""
import os

import pytest
import torch

import oracle as O
from paper_2602_17950_amd import gs, inputs

from helpers import orc, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _problem(n, omega, gamma):
    return inputs.Problem(dim=3, n=(n, n, n), L=(10.0, 10.0, 80.0), g=(0.97, 1.03, 0.05), omega=omega,
                          gamma=gamma, c0=3000.0, c1=1.0)


def _solve_and_evaluate(gpu_ctx, omega, gamma, opt):
    pb, pc = _problem(256, omega, gamma), _problem(64, omega, gamma)
    assert gs.existence_check(pb) == gs.GS_OK   # |Omega| < min(gamma_x, gamma_y), c0, c1 >= 0
    g0 = torch.from_numpy(inputs.initial_guess(pc, ("f", "f", "f"))).to(DEV)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    print(f"[ex7] Omega={omega} gamma={gamma}: 64^3 -> 128^3 -> 256^3", flush=True)
    r = gpu_ctx.solve_device(pb, g0, out, options=opt)
    torch.cuda.synchronize()
    print(f"[ex7] rc={r['rc']} E={r['E']!r} mu={r['mu']!r} it={r['iters']}+{r['iters_coarse']} "
          f"resid={r['resid_inf']:.2e} virial={r['virial']:.2e}", flush=True)
    assert r["rc"] == gs.GS_OK, r
    assert r["iters"] > 0 and r["iters_coarse"] > 0
    O.set_threads(min(16, os.cpu_count() or 1))   # the oracle's transforms at 256^3 on the host's share
    try:
        g, t, p = orc(pb)
        ev = O.evaluate(g, t, p, out.cpu().numpy())
    finally:
        O.set_threads(1)
    print(f"[ex7] oracle E={ev['E']!r} mu={ev['mu']!r} resid={ev['resid_inf']:.2e} virial={ev['virial']:.2e}",
          flush=True)
    for key in ("E", "mu", "e_kin", "e_pot", "e_rot", "e_spin", "e_soc"):
        assert rel(r[key], ev[key]) < 1e-10, (key, r[key], ev[key])
    for c in range(3):
        assert rel(r["mu_comp"][c], ev["mu_comp"][c]) < 1e-10
        assert rel(r["norm_comp"][c], ev["norm_comp"][c]) < 1e-10
    assert abs(sum(r["norm_comp"]) - 1.0) < 1e-13
    assert rel(r["resid_inf"], ev["resid_inf"]) < 1e-8
    assert abs(r["virial"] - ev["virial"]) < 1e-8
    assert ev["resid_inf"] < opt.tol * 1.01
    assert abs(ev["virial"]) < 1e-6
    return r, ev


@pytest.mark.timeout(400)
def test_example7_case4_fp64(gpu_ctx):
    """Case 4 (Omega = 0.5, SOC strength 0.4), plain FP64, residual stop 1e-9."""
    opt = gs.default_options(precision=gs.GS_FP64, stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-9, cm_levels=3,
                             max_iter=20000)
    _solve_and_evaluate(gpu_ctx, 0.5, 0.4, opt)


@pytest.mark.timeout(400)
def test_example7_case6_mixed(gpu_ctx):
    """Case 6 (Omega = 0.7, SOC strength 0.4), mixed precision with a float
    search direction in the double phase, residual stop 1e-9."""
    opt = gs.default_options(precision=gs.GS_MIXED, dir_precision=gs.GS_FP32, stop_kind=gs.GS_STOP_RESIDUAL,
                             tol=1e-9, cm_levels=3, max_iter=20000)
    _solve_and_evaluate(gpu_ctx, 0.7, 0.4, opt)
