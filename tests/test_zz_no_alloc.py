"""gs_fft_noalloc (the transform that allocates nothing) against gs_fft.

Both run the same kernels on the same twiddle tables, so the outputs agree
bit for bit; they are also held to the FP64/FP32 transform bars against the
oracle. Two calls in a row on the static scratch, the second with a smaller
grid, must both be right (the scratch keeps the previous call's contents).
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_17950_amd import gs

from helpers import rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _field(dim, n, seed, prec):
    rng = np.random.default_rng(seed)
    shape = (3,) + tuple(reversed(n[:dim]))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dt = torch.complex128 if prec == gs.GS_FP64 else torch.complex64
    return x, torch.from_numpy(x).to(DEV).to(dt)


@pytest.mark.parametrize("prec", [gs.GS_FP64, gs.GS_FP32])
@pytest.mark.parametrize("sign", [-1, 1])
def test_noalloc_matches_fft(gpu_ctx, prec, sign):
    cases = [(3, (64, 32, 128), (6.0, 5.0, 8.0)), (2, (96, 48), (8.0, 6.0)),
             (2, (512, 512), (16.0, 16.0)), (2, (32, 16), (4.0, 3.0))]
    for k, (dim, n, L) in enumerate(cases):
        print(f"[noalloc] prec={prec} sign={sign} dim={dim} n={n}", flush=True)
        g = gs.make_grid(dim, n, L)
        x, xd = _field(dim, n, 10 + k, prec)
        y_ref = torch.empty_like(xd)
        y = torch.full_like(xd, float("nan"))
        gpu_ctx.fft(g, xd, y_ref, sign, prec)
        gpu_ctx.fft_noalloc(g, xd, y, sign, prec)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(y), torch.view_as_real(y_ref)), (dim, n)
        og = O.Grid(dim, n, L)
        ref = np.stack([O.fftn(og, x[c], sign) for c in range(3)])
        tol = 1e-12 if prec == gs.GS_FP64 else 5e-6
        assert rel(y.to(torch.complex128).cpu().numpy(), ref) < tol


def test_noalloc_rejects_oversize(gpu_ctx):
    g = gs.make_grid(3, (128, 64, 64), (6.0, 6.0, 6.0))   # 2^19 points
    x = torch.empty((3, 64, 64, 128), dtype=torch.complex128, device=DEV)
    with pytest.raises(gs.GsError) as ei:
        gpu_ctx.fft_noalloc(g, x, torch.empty_like(x), -1)
    assert ei.value.code == gs.GS_EINVAL
    assert "2^18" in str(ei.value)
