"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison uses the same seeded input on both sides. Floating-point
tolerances: FP64 transforms and operators to 1e-12 (max-norm relative to the
largest entry; the rounding of a radix FFT grows like eps log N), energies and
chemical potentials of converged solves to 1e-10 relative; FP32 to 2e-6 for
transforms and 1e-6 relative for converged energies.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2602_17950_amd import gs, inputs

from helpers import aligned_errors, oracle_solve, orc, rel, smooth_field

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def to_dev(a, prec=gs.GS_FP64):
    dt = torch.complex128 if prec == gs.GS_FP64 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt)


def to_host(t):
    torch.cuda.synchronize()
    return t.to(torch.complex128).cpu().numpy()


GRIDS = [
    (2, (16, 16), (4.0, 4.0)),
    (2, (32, 64), (8.0, 6.0)),
    (2, (256, 128), (12.0, 10.0)),
    (2, (1024, 16), (16.0, 2.0)),
    (3, (16, 32, 16), (6.0, 6.0, 5.0)),
    (3, (32, 16, 64), (6.0, 5.0, 8.0)),
    # lengths 3 * 2^a (a radix-3 pass first)
    (2, (96, 48), (8.0, 6.0)),
    (2, (24, 768), (4.0, 16.0)),
    (3, (48, 24, 96), (6.0, 5.0, 8.0)),
    # factors of 5 (a radix-5 pass) and lines longer than 1024: the x axis in
    # the transposing passes, the y axis as the middle axis
    (2, (2400, 16), (20.0, 2.0)),
    (2, (160, 2400), (8.0, 20.0)),
    (2, (600, 1200), (10.0, 20.0)),
    (2, (80, 600), (8.0, 8.0)),
    (3, (80, 16, 600), (6.0, 5.0, 8.0)),
]


@pytest.mark.parametrize("dim,n,L", GRIDS)
@pytest.mark.parametrize("prec", [gs.GS_FP64, gs.GS_FP32])
def test_fft_forward_inverse(gpu_ctx, dim, n, L, prec):
    print(f"[fft] dim={dim} n={n} prec={prec}", flush=True)
    rng = np.random.default_rng(7)
    g = O.Grid(dim, n, L)
    shape = (3,) + g.shape
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = np.stack([O.fftn(g, x[c], -1) for c in range(3)])
    xd = to_dev(x, prec)
    yd = torch.empty_like(xd)
    gg = gs.make_grid(dim, n, L)
    gpu_ctx.fft(gg, xd, yd, -1, prec)
    y = to_host(yd)
    # FP32: rounding of a radix FFT with correctly rounded twiddles, ~eps log2 N
    tol = 1e-12 if prec == gs.GS_FP64 else 2e-6
    print(f"[fft] forward error {rel(y, ref):.2e}", flush=True)
    assert rel(y, ref) < tol
    # input untouched
    assert np.array_equal(to_host(xd), to_host(to_dev(x, prec)))
    # inverse of the spectrum returns the input
    zd = torch.empty_like(xd)
    gpu_ctx.fft(gg, to_dev(ref, prec), zd, +1, prec)
    assert rel(to_host(zd), x) < tol


def _problems():
    return [
        inputs.Problem(dim=2, n=(64, 64), L=(8.0, 8.0), omega=0.0, gamma=0.5, c0=100.0, c1=-0.5),
        inputs.Problem(dim=2, n=(64, 32), L=(10.0, 8.0), omega=0.6, gamma=1.0, c0=500.0, c1=-2.0),
        inputs.Problem(dim=2, n=(32, 32), L=(8.0, 8.0), g=(1.0, 1.3, 1.0), q2=-0.2, q4=0.05,
                       omega=1.2, gamma=0.8, c0=300.0, c1=3.0),
        inputs.Problem(dim=3, n=(32, 16, 32), L=(8.0, 7.0, 8.0), g=(1.0, 1.0, 2.0), omega=0.5,
                       gamma=1.0, c0=800.0, c1=5.0),
        inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), omega=0.0, gamma=0.3, c0=50.0, c1=-1.0),
        inputs.Problem(dim=2, n=(96, 48), L=(10.0, 8.0), omega=0.6, gamma=1.0, c0=500.0, c1=-2.0),
        inputs.Problem(dim=3, n=(24, 48, 24), L=(7.0, 8.0, 7.0), g=(1.0, 1.0, 2.0), omega=0.5,
                       gamma=1.0, c0=800.0, c1=5.0),
        # the trap of Example 5's second case, eq. (4.1), rotating at Omega = 3, on
        # a strip of its domain with the 2400-point axis as the middle axis
        inputs.Problem(dim=2, n=(160, 2400), L=(8.0, 20.0), g=(0.0, 0.0, 0.0), q2=-0.2, q4=0.5,
                       omega=3.0, gamma=0.8, c0=1000.0, c1=1.0),
        # the 2400-point axis along x (transposing passes), 80 points along y
        inputs.Problem(dim=2, n=(2400, 80), L=(20.0, 8.0), omega=0.6, gamma=1.0, c0=500.0, c1=-2.0),
        # 3D, a 600-point middle axis (line groups that end in a partial wave chunk)
        inputs.Problem(dim=3, n=(16, 80, 600), L=(6.0, 7.0, 9.0), g=(1.0, 1.0, 0.8), omega=0.4,
                       gamma=0.7, c0=300.0, c1=-1.0),
        # 256 x 64 x 64: the pipelined passes have more tiles and line groups than
        # resident blocks, so one slot runs the persistent unit loop and the XCD
        # tile order that batches of slots run
        inputs.Problem(dim=3, n=(256, 64, 64), L=(10.0, 6.0, 6.0), g=(0.5, 1.0, 1.0), omega=0.3,
                       gamma=0.6, c0=400.0, c1=2.0),
    ]


@pytest.mark.parametrize("k", range(11))
@pytest.mark.parametrize("prec", [gs.GS_FP64, gs.GS_FP32])
def test_hamiltonian_and_energy(gpu_ctx, k, prec):
    pb = _problems()[k]
    print(f"[ham] problem {k} {pb.n} prec={prec}", flush=True)
    psi = smooth_field(pb, seed=11 + k)
    g, t, p = orc(pb)
    H_ref = O.apply_H(g, t, p, psi)
    ev = O.evaluate(g, t, p, psi)
    psid = to_dev(psi, prec)
    hd = torch.empty_like(psid)
    res = gpu_ctx.hamiltonian(pb, psid, hd, prec)
    H = to_host(hd)
    # FP32: the float rounding of the input and of the transforms, ~eps log2 N
    op_tol = 1e-12 if prec == gs.GS_FP64 else 3e-6
    sc_tol = 1e-12 if prec == gs.GS_FP64 else 3e-6
    print(f"[ham] operator error {rel(H, H_ref):.2e}, E error {rel(res['E'], ev['E']):.2e}", flush=True)
    assert rel(H, H_ref) < op_tol
    for key in ("E", "mu", "e_kin", "e_pot", "e_rot", "e_spin", "e_soc", "virial", "resid_inf"):
        assert rel(res[key], ev[key]) < sc_tol, (key, res[key], ev[key])
    for c in range(3):
        assert rel(res["mu_comp"][c], ev["mu_comp"][c]) < sc_tol
        assert rel(res["norm_comp"][c], ev["norm_comp"][c]) < sc_tol


def test_hamiltonian_user_potential(gpu_ctx):
    pb = inputs.Problem(dim=2, n=(32, 64), L=(8.0, 8.0), omega=0.3, gamma=0.4, c0=80.0, c1=1.0)
    X = pb.coords()
    V = 0.5 * X[0] ** 2 + 0.7 * X[1] ** 2 + 0.3 * np.sin(X[0]) * np.cos(2 * X[1])
    psi = smooth_field(pb, seed=5)
    g, t, p = orc(pb, V)
    H_ref = O.apply_H(g, t, p, psi)
    ev = O.evaluate(g, t, p, psi)
    psid = to_dev(psi)
    hd = torch.empty_like(psid)
    res = gpu_ctx.hamiltonian(pb, psid, hd, V=V)
    assert rel(to_host(hd), H_ref) < 1e-12
    assert rel(res["E"], ev["E"]) < 1e-12
    assert np.isnan(res["virial"])


@pytest.mark.parametrize("k", [0, 1, 3, 7, 8, 9, 10])
@pytest.mark.parametrize("prec", [gs.GS_FP64, gs.GS_FP32])
def test_preconditioner(gpu_ctx, k, prec):
    pb = _problems()[k]
    print(f"[pre] problem {k} {pb.n} prec={prec}", flush=True)
    psi = smooth_field(pb, seed=21 + k)
    r = smooth_field(pb, seed=31 + k, kinds=("b", "a", "a"), noise=0.2)
    g, t, p = orc(pb)
    al = O.alpha(g, t, p, psi)
    ref = O.precond(g, t, p, psi, al, r)
    out = torch.empty_like(to_dev(psi, prec))
    gpu_ctx.precondition(pb, to_dev(psi, prec), to_dev(r, prec), out, prec)
    tol = 1e-12 if prec == gs.GS_FP64 else 3e-6
    print(f"[pre] error {rel(to_host(out), ref):.2e}", flush=True)
    assert rel(to_host(out), ref) < tol


def _solve_both(gpu_ctx, pb, psi0, stop, tol, prec=gs.GS_FP64, max_iter=20000):
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=stop, tol=tol, max_iter=max_iter))
    ev = O.evaluate(g, t, p, ref.psi)
    psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=stop, tol=tol, precision=prec,
                                                           max_iter=max_iter))
    return ref, ev, psi, res


def test_solve_small_2d_energy_stop(gpu_ctx):
    """64x64 workload, energy criterion 1e-12: E and mu against the oracle."""
    pb, psi0 = inputs.workload_small_2d()
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_ENERGY, 1e-12)
    print(f"[solve small] gpu E={res['E']!r} it={res['iters']} | oracle E={ev['E']!r} it={ref.iters}")
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10
    assert rel(res["mu"], ev["mu"]) < 1e-5     # mu is first order in the state error
    assert abs(sum(res["norm_comp"]) - 1.0) < 1e-13


def test_solve_small_2d_residual_stop(gpu_ctx):
    """Residual criterion 1e-11: E, mu and the component densities."""
    pb, psi0 = inputs.workload_small_2d()
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_RESIDUAL, 1e-11)
    print(f"[solve small res] gpu mu={res['mu']!r} it={res['iters']} | oracle mu={ev['mu']!r} it={ref.iters}")
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-12
    assert rel(res["mu"], ev["mu"]) < 1e-10
    assert res["resid_inf"] < 1e-11
    d_psi, d_rho = aligned_errors(psi, ref.psi)
    print(f"[solve small res] aligned psi {d_psi:.2e} rho {d_rho:.2e}", flush=True)
    assert d_psi < 1e-11 and d_rho < 1e-11


def test_solve_rotating_vortex_2d(gpu_ctx):
    """Rotating SOC case with a vortex guess (the 256^2 workload's parameters on
    64^2), both sides stopping on the residual at 1e-12, where mu and the
    densities (first order in the state error) are converged to ~1e-12: E and
    mu to 1e-10 relative, the wave function after aligning the global phase
    kappa (Sec. 2.2), and the component densities."""
    pb, psi0 = inputs.workload_vortex_2d(n=64)
    ref, ev = oracle_solve(pb, psi0, gs.GS_STOP_RESIDUAL, 1e-12, key="vortex64_r12")
    psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-12,
                                                          max_iter=40000))
    d_psi, d_rho = aligned_errors(psi, ref.psi)
    print(f"[solve vortex64 r12] gpu E={res['E']!r} mu={res['mu']!r} it={res['iters']} | oracle E={ev['E']!r} "
          f"mu={ev['mu']!r} it={ref.iters} | aligned psi {d_psi:.2e} rho {d_rho:.2e}", flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-12
    assert rel(res["mu"], ev["mu"]) < 1e-10
    for a, b in zip(res["mu_comp"], ev["mu_comp"]):
        assert rel(a, b) < 1e-10
    assert d_psi < 1e-10 and d_rho < 1e-10   # measured 2e-13 and 5e-14 (the same 7135 steps)
    assert res["e_soc"] <= 0.0


def test_solve_fp32_matches_oracle(gpu_ctx):
    """Pure FP32 solves (fields, transforms and the pointwise work in float,
    reductions in double) against the oracle's FP64 minimiser: energy to 1e-6
    relative, the FP32 bar."""
    for which in ("small2d", "vortex64"):
        if which == "small2d":
            pb, psi0 = inputs.workload_small_2d()
            ref, ev = oracle_solve(pb, psi0, gs.GS_STOP_RESIDUAL, 1e-11, key="small2d_r11")
        else:
            pb, psi0 = inputs.workload_vortex_2d(n=64)
            ref, ev = oracle_solve(pb, psi0, gs.GS_STOP_RESIDUAL, 1e-12, key="vortex64_r12")
        psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(precision=gs.GS_FP32, tol=1e-9))
        d_psi, d_rho = aligned_errors(psi, ref.psi)
        print(f"[fp32 {which}] gpu E={res['E']!r} mu={res['mu']!r} it={res['iters']} rc={res['rc']} | oracle "
              f"E={ev['E']!r} mu={ev['mu']!r} | E rel {rel(res['E'], ev['E']):.2e} mu rel "
              f"{rel(res['mu'], ev['mu']):.2e} aligned psi {d_psi:.2e} rho {d_rho:.2e}", flush=True)
        assert res["rc"] >= 0 and res["iters_fp32"] == res["iters"]
        assert rel(res["E"], ev["E"]) < 1e-6


def test_solve_mixed_matches_fp64(gpu_ctx):
    pb, psi0 = inputs.workload_vortex_2d(n=64)
    _, r64 = gpu_ctx.solve(pb, psi0, gs.default_options(tol=1e-12, precision=gs.GS_FP64))
    _, rmx = gpu_ctx.solve(pb, psi0, gs.default_options(tol=1e-12, precision=gs.GS_MIXED))
    _, r32 = gpu_ctx.solve(pb, psi0, gs.default_options(tol=1e-9, precision=gs.GS_FP32))
    print(f"[mixed] fp64 E={r64['E']!r} it={r64['iters']} mixed E={rmx['E']!r} it={rmx['iters']} "
          f"(fp32 {rmx['iters_fp32']}) fp32 E={r32['E']!r}")
    assert rmx["iters_fp32"] > 0
    assert rel(rmx["E"], r64["E"]) < 1e-10
    assert rel(r32["E"], r64["E"]) < 1e-6


@pytest.mark.parametrize("which", ["small2d", "vortex64", "3d16"])
def test_solve_fp32_direction_matches_oracle(gpu_ctx, which):
    """Double state with a float search direction (dir_precision GS_FP32): the
    residual, the line search and the stopping test stay double, so the limit
    is the FP64 one; E and mu are held to the FP64 solves' bars against the
    oracle, both sides stopping on the residual."""
    if which == "small2d":
        pb, psi0 = inputs.workload_small_2d()
        tol = 1e-11
    elif which == "vortex64":
        pb, psi0 = inputs.workload_vortex_2d(n=64)
        tol = 1e-9
    else:
        pb = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                            gamma=1.0, c0=200.0, c1=5.0)
        psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
        tol = 1e-10
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol))
    ev = O.evaluate(g, t, p, ref.psi)
    for prec in (gs.GS_FP64, gs.GS_MIXED):
        opt = gs.default_options(precision=prec, stop_kind=gs.GS_STOP_RESIDUAL, tol=tol,
                                 dir_precision=gs.GS_FP32, switch_resid=1e-4)
        psi, res = gpu_ctx.solve(pb, psi0, opt)
        print(f"[fp32 dir {which} prec={prec}] gpu E={res['E']!r} mu={res['mu']!r} it={res['iters']} "
              f"| oracle E={ev['E']!r} mu={ev['mu']!r} it={ref.iters}", flush=True)
        assert res["status"] == 0 and ref.status == 0
        assert res["resid_inf"] < tol
        assert rel(res["E"], ev["E"]) < 1e-10
        assert rel(res["mu"], ev["mu"]) < 1e-8
        assert abs(sum(res["norm_comp"]) - 1.0) < 1e-13


@pytest.mark.parametrize("kind", [gs.GS_PC_KINETIC, gs.GS_PC_POTENTIAL])
@pytest.mark.parametrize("which", ["small2d", "3d16"])
def test_preconditioner_kinds_match_oracle(gpu_ctx, kind, which):
    """Kinetic (3.12) and potential (3.14) preconditioners: the same solve on
    both sides (residual stop), E and mu to the FP64 bars, and iteration
    counts close to the oracle's (the same algorithm; rounding decides the
    rest)."""
    if which == "small2d":
        pb, psi0 = inputs.workload_small_2d()
    else:
        pb = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                            gamma=1.0, c0=200.0, c1=5.0)
        psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
    tol = 1e-9
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol, precond=kind, max_iter=20000))
    ev = O.evaluate(g, t, p, ref.psi)
    psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol, precond=kind,
                                                          max_iter=20000))
    print(f"[precond {kind} {which}] gpu E={res['E']!r} it={res['iters']} | oracle E={ev['E']!r} it={ref.iters}",
          flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10
    assert rel(res["mu"], ev["mu"]) < 1e-8
    assert abs(res["iters"] - ref.iters) <= 0.15 * ref.iters + 5


@pytest.mark.parametrize("which", ["small2d", "3d16", "rot32"])
def test_exact_line_search_matches_oracle(gpu_ctx, which):
    """The exact line-search option (the step minimises E along the curve):
    GPU (Newton refinement of the Algorithm-2 step) and oracle (bracket and
    golden section) reach the same minimiser, residual stop, FP64 bars."""
    if which == "small2d":
        pb, psi0 = inputs.workload_small_2d()
    elif which == "3d16":
        pb = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                            gamma=1.0, c0=200.0, c1=5.0)
        psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
    else:
        pb = inputs.Problem(dim=2, n=(32, 32), L=(6.0, 6.0), omega=0.3, gamma=0.8, c0=90.0, c1=0.7)
        psi0 = inputs.initial_guess(pb, ("b", "a", "a"), noise=1e-3, seed=101)
    tol = 1e-10
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol, exact_ls=1))
    ev = O.evaluate(g, t, p, ref.psi)
    psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol,
                                                          line_search=gs.GS_LS_EXACT))
    _, alg2 = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=tol))
    print(f"[exact ls {which}] gpu E={res['E']!r} it={res['iters']} (Alg. 2: {alg2['iters']}) | oracle "
          f"E={ev['E']!r} it={ref.iters}", flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10
    assert rel(res["mu"], ev["mu"]) < 1e-8


def test_wavefunction_criterion_matches_oracle(gpu_ctx):
    """Criterion (3.9): the GPU stops when the last step changed no component
    anywhere by tol or more, at (nearly) the oracle's iteration, with the same
    energy."""
    pb, psi0 = inputs.workload_small_2d()
    tol = 1e-6
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_WAVEFN, tol=tol))
    ev = O.evaluate(g, t, p, ref.psi)
    psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_WAVEFN, tol=tol))
    print(f"[wavefn] gpu it={res['iters']} dphi={res['dphi_inf']:.3e} E={res['E']!r} | oracle it={ref.iters} "
          f"E={ev['E']!r}", flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert res["dphi_inf"] < tol
    assert abs(res["iters"] - ref.iters) <= 3
    assert rel(res["E"], ev["E"]) < 1e-9


def test_wavefunction_criterion_mixed(gpu_ctx):
    """Criterion (3.9) in a mixed solve applies to steps of the double phase
    only: neither the float phase's last step nor the renormalisation at the
    hand-over may stop it, so the double phase takes steps and the energy
    matches the oracle's FP64 run under the same criterion."""
    pb, psi0 = inputs.workload_small_2d()
    tol = 1e-6
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_WAVEFN, tol=tol))
    ev = O.evaluate(g, t, p, ref.psi)
    for sw in (1e-4, 1e-7):
        psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_WAVEFN, tol=tol,
                                                              precision=gs.GS_MIXED, switch_resid=sw))
        print(f"[wavefn mixed sw={sw}] gpu it={res['iters']} (fp32 {res['iters_fp32']}) "
              f"dphi={res['dphi_inf']:.3e} E={res['E']!r} | oracle it={ref.iters} E={ev['E']!r}", flush=True)
        assert res["status"] == 0 and ref.status == 0
        assert res["iters"] > res["iters_fp32"] > 0
        assert res["dphi_inf"] < tol
        assert rel(res["E"], ev["E"]) < 1e-9


def test_nyquist_readings_match_oracle(gpu_ctx):
    """The two readings of the mode p = -N/2 in the odd symbols (option
    nyquist_odd): Table 1's Case 1 at h = 1 (32^2 on [-16,16]^2), where they
    differ by ~2e-6 in E. Each GPU reading matches the oracle's same reading
    (residual stop 1e-10)."""
    pb = inputs.Problem(dim=2, n=(32, 32), L=(16.0, 16.0), omega=0.1, gamma=0.3, c0=100.0, c1=1.0)
    psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
    E = {}
    for nyq in (gs.GS_NYQ_KEEP, gs.GS_NYQ_ZERO):
        g = O.Grid(2, pb.n, pb.L, nyq)
        _, t, p = orc(pb)
        ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-10))
        ev = O.evaluate(g, t, p, ref.psi)
        psi, res = gpu_ctx.solve(pb, psi0, gs.default_options(stop_kind=gs.GS_STOP_RESIDUAL, tol=1e-10,
                                                              nyquist_odd=nyq))
        print(f"[nyquist {nyq}] gpu E={res['E']!r} mu={res['mu']!r} it={res['iters']} | oracle E={ev['E']!r} "
              f"mu={ev['mu']!r} it={ref.iters}", flush=True)
        assert res["status"] == 0 and ref.status == 0
        assert rel(res["E"], ev["E"]) < 1e-10
        assert rel(res["mu"], ev["mu"]) < 1e-9
        E[nyq] = res["E"]
    assert abs(E[gs.GS_NYQ_KEEP] - E[gs.GS_NYQ_ZERO]) > 1e-7


def test_existence_warning(gpu_ctx):
    """A 3D solve with a weakly attractive c0 < 0 (outside the hypotheses of
    the existence theorem of Sec. 2.1) that converges to the metastable
    trapped state returns GS_WEXISTENCE with valid outputs, which match the
    oracle."""
    pb = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), gamma=0.5, c0=-0.5, c1=0.2)
    assert gs.existence_check(pb) == gs.GS_WEXISTENCE
    psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_RESIDUAL, 1e-10)
    print(f"[existence] gpu rc={res['rc']} E={res['E']!r} | oracle E={ev['E']!r}", flush=True)
    assert res["rc"] == gs.GS_WEXISTENCE and res["status"] == gs.GS_WEXISTENCE
    assert ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10


def test_solve_radix3_grid(gpu_ctx):
    """A 48^2 grid (a radix-3 pass in every transform): the small 2D workload's
    parameters, residual stop, against the oracle (naive DFT for length 48)."""
    pb = inputs.Problem(dim=2, n=(48, 48), L=(8.0, 8.0), omega=0.3, gamma=0.5, c0=100.0, c1=-0.5)
    psi0 = inputs.initial_guess(pb, ("b", "a", "a"))
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_RESIDUAL, 1e-10)
    print(f"[solve 48] gpu E={res['E']!r} it={res['iters']} | oracle E={ev['E']!r} it={ref.iters}", flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10
    assert rel(res["mu"], ev["mu"]) < 1e-8


def test_solve_long_middle_axis(gpu_ctx):
    """A 32 x 1200 grid, rotating: the 1200-point y axis takes the split middle
    pass (line transforms, the operator over the whole spectrum, the rotation
    term in the inverse) in both the preconditioner and H_L, with radix-5
    passes; residual stop, against the oracle's PCG from the same guess."""
    pb = inputs.Problem(dim=2, n=(32, 1200), L=(6.0, 24.0), g=(1.0, 0.25, 1.0), omega=0.2, gamma=0.5,
                        c0=100.0, c1=-0.5)
    psi0 = inputs.initial_guess(pb, ("b", "a", "a"))
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_RESIDUAL, 1e-10)
    d_psi, d_rho = aligned_errors(psi, ref.psi)
    print(f"[solve 32x1200] gpu E={res['E']!r} it={res['iters']} | oracle E={ev['E']!r} it={ref.iters} "
          f"d_psi={d_psi:.1e} d_rho={d_rho:.1e}", flush=True)
    assert res["status"] == 0 and ref.status == 0
    assert rel(res["E"], ev["E"]) < 1e-10
    assert rel(res["mu"], ev["mu"]) < 1e-10
    assert d_rho < 1e-6


def test_solve_3d_small(gpu_ctx):
    pb = inputs.Problem(dim=3, n=(16, 16, 16), L=(6.0, 6.0, 6.0), g=(1.0, 1.0, 2.0), omega=0.5,
                        gamma=1.0, c0=200.0, c1=5.0)
    psi0 = inputs.initial_guess(pb, ("a", "a", "a"))
    ref, ev, psi, res = _solve_both(gpu_ctx, pb, psi0, gs.GS_STOP_ENERGY, 1e-12)
    print(f"[solve 3d] gpu E={res['E']!r} it={res['iters']} | oracle E={ev['E']!r} it={ref.iters}")
    assert rel(res["E"], ev["E"]) < 1e-10


def test_solve_gaussian_default_guess(gpu_ctx):
    pb, psi0 = inputs.workload_small_2d()
    _, r1 = gpu_ctx.solve(pb, psi0, gs.default_options())
    _, r2 = gpu_ctx.solve(pb, None, gs.default_options())
    assert r1["E"] == r2["E"] or rel(r1["E"], r2["E"]) < 1e-13


def test_solve_device_matches_host(gpu_ctx):
    pb, psi0 = inputs.workload_small_2d()
    psi_h, rh = gpu_ctx.solve(pb, psi0, gs.default_options())
    out = torch.empty((3,) + pb.shape, dtype=torch.complex128, device=DEV)
    rd = gpu_ctx.solve_device(pb, to_dev(psi0), out, gs.default_options())
    assert rd["E"] == rh["E"]
    assert np.array_equal(to_host(out), psi_h)


def test_errors_and_warnings(gpu_ctx):
    pb, psi0 = inputs.workload_small_2d()
    bad = inputs.Problem(dim=2, n=(40, 64), L=(8.0, 8.0))
    with pytest.raises(gs.GsError) as e:
        gpu_ctx.solve(bad, None, gs.default_options())
    assert e.value.code == gs.GS_EINVAL
    nan_psi = psi0.copy()
    nan_psi[0, 3, 3] = np.nan
    with pytest.raises(gs.GsError) as e:
        gpu_ctx.solve(pb, nan_psi, gs.default_options())
    assert e.value.code == gs.GS_ENONFINITE
    _, res = gpu_ctx.solve(pb, psi0, gs.default_options(max_iter=3))
    assert res["rc"] == gs.GS_WMAXITER and res["iters"] == 3
    # the library is still usable after errors
    _, res = gpu_ctx.solve(pb, psi0, gs.default_options())
    assert res["rc"] == 0
