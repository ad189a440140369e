"""Shared test helpers: oracle objects for a Problem, relative errors."""
import numpy as np

import oracle as O


def orc(pb, V=None):
    g = O.Grid(pb.dim, pb.n, pb.L)
    t = O.Trap(pb.g, pb.q2, pb.q4, V)
    p = O.Params(pb.omega, pb.gamma, pb.c0, pb.c1)
    return g, t, p


def rel(a, b):
    """|a - b| / max(|b|, 1) (scalars), or max-norm relative to max |b| (arrays)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 0:
        return float(abs(a - b) / max(abs(b), 1.0))
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def smooth_field(pb, seed, kinds=("a", "b", "bbar"), noise=0.05):
    """A smooth, normalised three-component test field with broadband content."""
    from paper_2602_17950_amd import inputs
    rng = np.random.default_rng(seed)
    psi = inputs.initial_guess(pb, kinds)
    X = pb.coords()
    r2 = sum(x ** 2 for x in X)
    env = np.exp(-r2 / 8.0)
    re = rng.standard_normal(psi.shape)
    im = rng.standard_normal(psi.shape)
    psi = psi + noise * env * (re + 1j * im)
    return inputs.normalise(psi, pb.cell)


def aligned_errors(psi, ref):
    """Differences between two wave functions that may differ by the global
    phase kappa of Sec. 2.2 (E(e^{i kappa} Phi) = E(Phi)): kappa is the argument
    of <psi, ref>, and the results are the max-norm difference of
    e^{-i kappa} psi and ref relative to max |ref|, and the largest difference of
    the component densities |phi_l|^2 relative to the largest density."""
    z = np.vdot(ref, psi)
    kap = np.angle(z)
    d_psi = float(np.max(np.abs(psi * np.exp(-1j * kap) - ref)) / np.max(np.abs(ref)))
    rho, rho_r = np.abs(psi) ** 2, np.abs(ref) ** 2
    d_rho = float(np.max(np.abs(rho - rho_r)) / np.max(rho_r))
    return d_psi, d_rho


_ORACLE_CACHE = {}


def oracle_solve(pb, psi0, stop, tol, max_iter=40000, key=None, **opt):
    """The oracle's PCG from psi0, cached for the session under `key` (several
    tests compare against the same reference solve)."""
    if key is not None and key in _ORACLE_CACHE:
        return _ORACLE_CACHE[key]
    g, t, p = orc(pb)
    ref = O.pcg(g, t, p, psi0, O.Options(stop_kind=stop, tol=tol, max_iter=max_iter, **opt))
    ev = O.evaluate(g, t, p, ref.psi)
    if key is not None:
        _ORACLE_CACHE[key] = (ref, ev)
    return ref, ev
