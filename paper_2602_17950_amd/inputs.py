"""Seeded synthetic inputs: grids, traps, parameter sets and initial guesses.

This module only builds inputs. It holds none of the solver's arithmetic and is
the one module shared by the GPU path's tests and benchmark and by the checks
that run the CPU oracle: the same numpy arrays are handed to both.

Initial guesses are the single-component guesses (a)-(f) listed at the start of
Sec. 4 of the paper, combined component-wise as Phi^0 = (phi_1, phi_0, phi_-1)
and normalised on the grid (h^d sum |Phi|^2 = 1). Wave functions are complex128
arrays of shape (3, Ny, Nx) in 2D and (3, Nz, Ny, Nx) in 3D, x fastest,
component order (phi_1, phi_0, phi_-1).
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict

import numpy as np


@dataclass
class Problem:
    """One ground-state problem: grid, trap, physical parameters."""
    dim: int
    n: tuple              # (Nx, Ny[, Nz])
    L: tuple              # half-widths: domain prod [-L_a, L_a]
    g: tuple = (1.0, 1.0, 1.0)   # harmonic frequencies gamma_x, gamma_y, gamma_z
    q2: float = 0.0       # extra isotropic r^2 coefficient
    q4: float = 0.0       # r^4 coefficient
    omega: float = 0.0
    gamma: float = 0.0    # SOC strength
    c0: float = 0.0       # beta0 (spin-independent interaction)
    c1: float = 0.0       # beta1 (spin-exchange interaction)

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.dim]))

    @property
    def h(self):
        return tuple(2.0 * self.L[a] / self.n[a] for a in range(self.dim))

    @property
    def cell(self):
        return float(np.prod(self.h))

    @property
    def npts(self):
        return int(np.prod(self.n[: self.dim]))

    def coords(self):
        """Broadcastable coordinate arrays (x, y[, z]) with x_m = -L + m h."""
        ax = [-self.L[a] + np.arange(self.n[a]) * self.h[a] for a in range(self.dim)]
        return np.meshgrid(*reversed(ax), indexing="ij")[::-1]

    def potential(self):
        """V = 1/2 sum g_a^2 x_a^2 + q2 r^2 + q4 r^4 sampled on the grid."""
        X = self.coords()
        V = np.zeros(self.shape)
        r2 = np.zeros(self.shape)
        for a in range(self.dim):
            V += 0.5 * self.g[a] ** 2 * X[a] ** 2
            r2 += X[a] ** 2
        return V + self.q2 * r2 + self.q4 * r2 * r2

    def to_dict(self):
        return asdict(self)


def normalise(psi, cell):
    psi = np.asarray(psi, dtype=np.complex128)
    return psi / np.sqrt(cell * np.sum(np.abs(psi) ** 2))


def _norm1(f, cell):
    return f / np.sqrt(cell * np.sum(np.abs(f) ** 2))


def guess_single(pb: Problem, kind: str):
    """One of the ten single-component initial guesses of Sec. 4:
    'a', 'b', 'bbar', 'c', 'cbar', 'd', 'dbar', 'e', 'ebar', 'f'."""
    X = pb.coords()
    r2 = sum(x ** 2 for x in X)
    d = pb.dim
    phi_a = np.pi ** (-d / 4.0) * np.exp(-r2 / 2.0) + 0j
    phi_b = (X[0] + 1j * X[1]) * phi_a
    W = pb.omega
    if kind == "a":
        return phi_a
    if kind == "b":
        return phi_b
    if kind == "bbar":
        return np.conj(phi_b)
    if kind in ("c", "cbar"):
        f = _norm1(phi_a + phi_b, pb.cell)
        return f if kind == "c" else np.conj(f)
    if kind in ("d", "dbar"):
        f = _norm1((1 - W) * phi_a + W * phi_b, pb.cell)
        return f if kind == "d" else np.conj(f)
    if kind in ("e", "ebar"):
        f = _norm1(W * phi_a + (1 - W) * phi_b, pb.cell)
        return f if kind == "e" else np.conj(f)
    if kind == "f":
        return _norm1(thomas_fermi(pb) + 0j, pb.cell)
    raise ValueError(f"unknown initial guess kind {kind!r}")


def thomas_fermi(pb: Problem):
    """Thomas-Fermi profile sqrt((mu_TF - V)_+ / c0). For a harmonic trap mu_TF is
    the closed form of Sec. 4; otherwise mu_TF is found by bisection so that the
    profile has unit mass on the grid."""
    V = pb.potential()
    c0 = pb.c0 if pb.c0 > 0 else 1.0
    if pb.q2 == 0.0 and pb.q4 == 0.0:
        g = pb.g
        if pb.dim == 2:
            mu = 0.5 * np.sqrt(4.0 * c0 * g[0] * g[1] / np.pi)
        else:
            mu = 0.5 * (15.0 * c0 * g[0] * g[1] * g[2] / (4.0 * np.pi)) ** 0.4
    else:
        lo, hi = float(V.min()), float(V.min()) + 1.0
        mass = lambda m: pb.cell * np.sum(np.maximum(m - V, 0.0)) / c0
        while mass(hi) < 1.0:
            hi = lo + 2.0 * (hi - lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if mass(mid) < 1.0 else (lo, mid)
        mu = 0.5 * (lo + hi)
    return np.sqrt(np.maximum(mu - V, 0.0) / c0)


def initial_guess(pb: Problem, kinds=("a", "a", "a"), noise: float = 0.0, seed: int | None = None):
    """Phi^0 = (phi_1, phi_0, phi_-1)/sqrt(3) from per-component guess kinds,
    plus optional complex Gaussian noise noise*(xi + i eta), xi, eta ~ N(0,1)
    i.i.d. drawn from numpy.random.default_rng(seed) (real parts first, then
    imaginary parts), normalised on the grid."""
    psi = np.stack([guess_single(pb, k) for k in kinds]) / np.sqrt(3.0)
    if noise:
        rng = np.random.default_rng(seed)
        re = rng.standard_normal(psi.shape)
        im = rng.standard_normal(psi.shape)
        psi = psi + noise * (re + 1j * im)
    return normalise(psi, pb.cell)


# ----------------------------------------------------------------------------
# the synthetic workloads (each function states its parameter set)
# ----------------------------------------------------------------------------
def workload_small_2d():
    """2D 64x64 on [-8,8]^2, harmonic, Omega=0, gamma=0.5, c0=100, c1=-0.5,
    Phi^0 = (a, a, a)."""
    pb = Problem(dim=2, n=(64, 64), L=(8.0, 8.0), omega=0.0, gamma=0.5, c0=100.0, c1=-0.5)
    return pb, initial_guess(pb, ("a", "a", "a"))


def workload_vortex_2d(n: int = 256, seed: int = 2602):
    """2D 256x256 on [-12,12]^2, harmonic, Omega=0.6, gamma=1.0, c0=500, c1=-2,
    Phi^0 = ((x+iy) phi_a, phi_a, phi_a) plus 1e-3 complex noise (seeded)."""
    pb = Problem(dim=2, n=(n, n), L=(12.0, 12.0), omega=0.6, gamma=1.0, c0=500.0, c1=-2.0)
    return pb, initial_guess(pb, ("b", "a", "a"), noise=1e-3, seed=seed)


def workload_aniso_3d(n: int = 128):
    """3D n^3 on [-8,8]^3, V = (x^2 + y^2 + 4 z^2)/2, Omega=0.5, gamma=1.0,
    c0=800, c1=5 (antiferromagnetic), Phi^0 = (a, a, a)."""
    pb = Problem(dim=3, n=(n, n, n), L=(8.0, 8.0, 8.0), g=(1.0, 1.0, 2.0),
                 omega=0.5, gamma=1.0, c0=800.0, c1=5.0)
    return pb, initial_guess(pb, ("a", "a", "a"))


def workload_sweep_2d(count: int = 96, seed: int = 17950, sizes=(128, 256, 512)):
    """Batched parameter sweep: grids uniform over ``sizes``, L = 16, harmonic,
    Omega~U[0,0.9], gamma~U[0,2], c0~U[100,2000], c1~U[-5,5], initial guess
    uniform over {Gaussian (a,a,a), vortex (b,a,a), Thomas-Fermi (f,f,f)};
    all draws from one generator in a fixed order."""
    rng = np.random.default_rng(seed)
    kinds = [("a", "a", "a"), ("b", "a", "a"), ("f", "f", "f")]
    out = []
    for _ in range(count):
        n = int(sizes[rng.integers(len(sizes))])
        omega = float(rng.uniform(0.0, 0.9))
        gamma = float(rng.uniform(0.0, 2.0))
        c0 = float(rng.uniform(100.0, 2000.0))
        c1 = float(rng.uniform(-5.0, 5.0))
        k = kinds[int(rng.integers(3))]
        pb = Problem(dim=2, n=(n, n), L=(16.0, 16.0), omega=omega, gamma=gamma, c0=c0, c1=c1)
        out.append((pb, k))
    return out


def workload_serve(count: int = 400, seed: int = 2603, sizes2d=(128, 256, 512, 1024), sizes3d=(64, 96, 128, 192)):
    """Served request stream: 75% 2D (grid uniform over ``sizes2d``, L = 16),
    25% 3D (grid uniform over ``sizes3d``, L = 10); Omega, gamma, c0, c1 and the
    guess kind drawn as in the batched sweep; trap half harmonic, half harmonic
    plus quartic 0.5 r^2 + 0.01 r^4. Returns (Problem, guess kinds) pairs; all
    draws from one generator in a fixed order."""
    rng = np.random.default_rng(seed)
    kinds = [("a", "a", "a"), ("b", "a", "a"), ("f", "f", "f")]
    out = []
    for _ in range(count):
        three = bool(rng.random() < 0.25)
        if three:
            n = int(sizes3d[rng.integers(len(sizes3d))])
        else:
            n = int(sizes2d[rng.integers(len(sizes2d))])
        omega = float(rng.uniform(0.0, 0.9))
        gamma = float(rng.uniform(0.0, 2.0))
        c0 = float(rng.uniform(100.0, 2000.0))
        c1 = float(rng.uniform(-5.0, 5.0))
        k = kinds[int(rng.integers(3))]
        quartic = bool(rng.random() < 0.5)
        q4 = 0.01 if quartic else 0.0
        if three:
            pb = Problem(dim=3, n=(n, n, n), L=(10.0, 10.0, 10.0), q4=q4, omega=omega, gamma=gamma,
                         c0=c0, c1=c1)
        else:
            pb = Problem(dim=2, n=(n, n), L=(16.0, 16.0), q4=q4, omega=omega, gamma=gamma, c0=c0, c1=c1)
        out.append((pb, k))
    return out
