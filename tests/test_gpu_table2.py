"""Table 2 of the paper (Example 3) end to end on the GPU.

Sec. 4 takes every component of Phi^0 independently from ten single-component
guesses (1000 combinations), solves from each and keeps the lowest energy as
the ground state. Here the 1000 solves of each Omega run as one batch of
cascadic-multigrid solves (Algorithm 3, 64^2 -> 128^2 -> 256^2 on [-12,12]^2,
the paper's CM-PCG setting), mixed precision with a float direction in the
double phase, stopping criterion (3.11) at 1e-14. The lowest energy must round
to the printed one; the energies reached from the ten identical-component
guesses are printed beside the paper's row (they are local minima reached
along rounding-dependent paths, so only the lowest is asserted).
"""
import itertools
import json
import os

import numpy as np
import pytest
import torch

from paper_2602_17950_amd import gs, inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "table2_example3_all.json")))


@pytest.mark.parametrize("omega", ["0.6", "0.7", "0.8", "0.9"])
def test_table2_lowest_energy_by_enumeration(gpu_ctx, omega):
    row = GOLD["rows"][omega]
    N, L = GOLD["N"], GOLD["domain_half_width"]
    kw = dict(dim=2, L=(L, L), omega=float(omega), gamma=GOLD["gamma"], c0=GOLD["c0"], c1=GOLD["c1"])
    fine = inputs.Problem(n=(N, N), **kw)
    coarse = inputs.Problem(n=(N // 4, N // 4), **kw)
    kinds = GOLD["guess_order"]
    combos = list(itertools.product(kinds, repeat=3))
    guess = [torch.from_numpy(inputs.initial_guess(coarse, k)).to("cuda") for k in combos]
    outs = [torch.empty((3, N, N), dtype=torch.complex128, device="cuda") for _ in combos]
    opt = gs.default_options(precision=gs.GS_MIXED, dir_precision=gs.GS_FP32, tol=1e-14, cm_levels=3)
    print(f"[table2] omega={omega}: {len(combos)} solves", flush=True)
    res = gpu_ctx.batch_solve([(fine, g, o, opt, None) for g, o in zip(guess, outs)])
    torch.cuda.synchronize()
    assert all(r["rc"] >= 0 for r in res)
    E = np.array([r["E"] for r in res])
    k = int(np.argmin(E))
    same = [E[combos.index((c, c, c))] for c in kinds]
    print(f"[table2] omega={omega}: lowest {E[k]:.8f} from {combos[k]} (paper {row['lowest']}); "
          f"identical guesses {np.round(same, 4).tolist()} | paper CM-PCG {row['cm_pcg']}", flush=True)
    assert round(float(E[k]), GOLD["decimals"]) == row["lowest"]
    # every returned state is a converged stationary state of the fine problem
    assert max(r["resid_inf"] for r in res) < 1e-5
