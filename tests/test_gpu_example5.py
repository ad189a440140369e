"""Example 5, second case: the harmonic-plus-quartic trap of eq. (4.1) on
[-20, 20]^2 with N = 2400 (c0 = 1000, c1 = 1, gamma = 0.8, Omega = 3).

The GPU solves it by cascadic multigrid (Algorithm 3) on 300^2, 600^2,
1200^2 and 2400^2 (every transform has radix-5 passes; the 1200- and
2400-point middle axes take the split middle pass). A same-guess oracle run
at this size would take hours of host time, so the oracle evaluates the
GPU's final state instead: E and its parts, mu and mu_l, N_l and the residual
of that state must equal what the GPU reports for it. The iteration is
capped; the test asks for descent from the interpolated coarse solution and
a unit total mass, not for a converged ground state.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_17950_amd import gs, inputs

from helpers import orc, rel

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(400)   # two oracle evaluations at 2400^2 on the host
def test_example5_case2_n2400_evaluated_by_oracle(gpu_ctx):
    pb = inputs.Problem(dim=2, n=(2400, 2400), L=(20.0, 20.0), g=(0.0, 0.0, 0.0), q2=-0.2, q4=0.5,
                        omega=3.0, gamma=0.8, c0=1000.0, c1=1.0)
    pc = inputs.Problem(**{**pb.to_dict(), "n": (300, 300)})
    assert gs.existence_check(pb) == gs.GS_OK   # no verdict for a quartic trap
    psi0 = inputs.initial_guess(pc, ("a", "a", "a"))
    opt = gs.default_options(stop_kind=gs.GS_STOP_ENERGY, tol=1e-10, cm_levels=4, max_iter=1500)
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device="cuda")
    print("[ex5] 2400^2 CM solve, 4 levels", flush=True)
    r = gpu_ctx.solve_device(pb, torch.from_numpy(psi0).to("cuda"), out, options=opt)
    torch.cuda.synchronize()
    print(f"[ex5] rc={r['rc']} E={r['E']!r} mu={r['mu']!r} it={r['iters']}+{r['iters_coarse']} "
          f"resid={r['resid_inf']:.2e}", flush=True)
    assert r["rc"] in (gs.GS_OK, gs.GS_WMAXITER, gs.GS_WSTAGNATED)
    assert r["iters"] > 0 and r["iters_coarse"] > 0
    psi = out.cpu().numpy()
    O.set_threads(min(16, os.cpu_count() or 1))   # the machine's CPU share
    g, t, p = orc(pb)
    ev = O.evaluate(g, t, p, psi)
    print(f"[ex5] oracle E={ev['E']!r} mu={ev['mu']!r} resid={ev['resid_inf']:.2e}", flush=True)
    assert abs(sum(r["norm_comp"]) - 1.0) < 1e-12
    for key in ("E", "mu", "e_kin", "e_pot", "e_rot", "e_spin", "e_soc"):
        assert rel(r[key], ev[key]) < 1e-10, (key, r[key], ev[key])
    for c in range(3):
        assert rel(r["mu_comp"][c], ev["mu_comp"][c]) < 1e-10
        assert rel(r["norm_comp"][c], ev["norm_comp"][c]) < 1e-10
    assert rel(r["resid_inf"], ev["resid_inf"]) < 1e-8
    # descent at the finest level: below the energy of the interpolated coarse solution
    p1200 = inputs.Problem(**{**pb.to_dict(), "n": (1200, 1200)})
    fine0 = torch.empty_like(out)
    coarse = torch.empty((3, 1200, 1200), dtype=torch.complex128, device="cuda")
    opt_c = gs.default_options(stop_kind=gs.GS_STOP_ENERGY, tol=1e-10, cm_levels=3, max_iter=1500)
    rc = gpu_ctx.solve_device(p1200, torch.from_numpy(psi0).to("cuda"), coarse, options=opt_c)
    gpu_ctx.interpolate(gs.grid_of(p1200), coarse, gs.grid_of(pb), fine0)
    torch.cuda.synchronize()
    e0 = O.evaluate(g, t, p, fine0.cpu().numpy())["E"]
    print(f"[ex5] 1200^2 E={rc['E']!r}; interpolated to 2400^2 E={e0!r}; final E={r['E']!r}", flush=True)
    O.set_threads(1)
    assert r["E"] < e0
    assert np.isfinite(r["E"])
