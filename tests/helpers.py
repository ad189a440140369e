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
