"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and the
oracle checks.

This module holds only random draws and the left-hand-side bands of each
synthetic PDE workload.  It contains none of the solver's arithmetic, imports
nothing from the GPU library or from the oracle, and is the only code both
sides of a parity check have in common.

Array convention: a batch is an (n, m) float64 array, element i of system k at
[i, k] -- the interleaved layout (batch index fastest) of Section 2 of
Carroll et al., arXiv:2107.05395.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2107053950


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_batch(n: int, m: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. uniform[lo, hi) entries, shape (n, m)."""
    return rng(seed).uniform(lo, hi, size=(n, m))


def sine_mode_batch(n: int, m: int, seed: int, modes: int = 8) -> np.ndarray:
    """Random-phase sum of `modes` Dirichlet sine modes per system:
    b[i, k] = sum_j A[j,k] sin(j pi x_i + phi[j,k]), x_i = (i+1)/(n+1),
    A ~ N(0, 1), phi ~ U[0, 2 pi), independent per system."""
    g = rng(seed)
    amp = g.standard_normal((modes, m))
    phase = g.uniform(0.0, 2.0 * math.pi, size=(modes, m))
    x = (np.arange(n, dtype=np.float64) + 1.0) / (n + 1.0)
    # sin(a + p) = sin(a) cos(p) + cos(a) sin(p): two (n x modes) @ (modes x m) products
    arg = np.pi * np.outer(x, np.arange(1, modes + 1))
    return np.sin(arg) @ (amp * np.cos(phase)) + np.cos(arg) @ (amp * np.sin(phase))


# ---------------------------------------------------------------- LHS bands

def diffusion_tri_bands(n: int, r: float):
    """Implicit-Euler diffusion, zero Dirichlet: rows (-r, 1 + 2r, -r)."""
    return np.full(n, -r), np.full(n, 1.0 + 2.0 * r), np.full(n, -r)


def hyperdiffusion_penta_bands(n: int, r: float):
    """Implicit-Euler hyperdiffusion, bands (r, -4r, 1 + 6r, -4r, r) on every row."""
    return (np.full(n, r), np.full(n, -4.0 * r), np.full(n, 1.0 + 6.0 * r),
            np.full(n, -4.0 * r), np.full(n, r))


def ch_penta_bands(n: int, sigma: float):
    """Periodic Cahn-Hilliard LHS: a = e = sigma, b = d = -4 sigma, c = 1 + 6 sigma
    (Section 5.1); the same five values wrap around the corners."""
    return hyperdiffusion_penta_bands(n, sigma)


def cn_diffusion_problem(n: int, sigma: float):
    """Crank-Nicolson periodic diffusion (Section 3 benchmark problem), sigma =
    dt/(2 dx^2): LHS bands (-sigma, 1 + 2 sigma, -sigma) on every row and the
    explicit stencil (sigma, 1 - 2 sigma, sigma) of rows i-1, i, i+1."""
    bands = (np.full(n, -sigma), np.full(n, 1.0 + 2.0 * sigma), np.full(n, -sigma))
    return bands, (sigma, 1.0 - 2.0 * sigma, sigma)


def cn_hyperdiffusion_problem(n: int, sigma: float):
    """Crank-Nicolson periodic hyperdiffusion (Section 4 benchmark problem),
    sigma = dt/(2 dx^4): LHS bands (sigma, -4 sigma, 1 + 6 sigma, -4 sigma, sigma)
    and the explicit stencil (-sigma, 4 sigma, 1 - 6 sigma, 4 sigma, -sigma)."""
    return (hyperdiffusion_penta_bands(n, sigma),
            (-sigma, 4.0 * sigma, 1.0 - 6.0 * sigma, 4.0 * sigma, -sigma))


def variable_diffusion_bands(D: np.ndarray, r: float):
    """A(D) = I + r diag(D) T2, T2 = tridiag(-1, 2, -1): rows (-r D_i, 1 + 2 r D_i, -r D_i)."""
    D = np.asarray(D, dtype=np.float64)
    return -r * D, 1.0 + 2.0 * r * D, -r * D


def random_dominant_tri(n: int, seed: int, margin: float = 1.0):
    """Random row-dependent bands with |b_i| >= |a_i| + |c_i| + margin."""
    g = rng(seed)
    a, c = g.uniform(-1, 1, n), g.uniform(-1, 1, n)
    b = (np.abs(a) + np.abs(c) + margin) * g.choice([-1.0, 1.0], n)
    return a, b, c


def random_dominant_penta(n: int, seed: int, margin: float = 1.0):
    g = rng(seed)
    a, b, d, e = (g.uniform(-1, 1, n) for _ in range(4))
    c = (np.abs(a) + np.abs(b) + np.abs(d) + np.abs(e) + margin) * g.choice([-1.0, 1.0], n)
    return a, b, c, d, e


# ---------------------------------------------------------------- workloads

WORKLOADS = {
    # name: description; seeds are SEED_BASE + index
    "diffusion_n256_m1024": dict(kind="tri", n=256, m=1024, r=0.5, seed=SEED_BASE + 0),
    "diffusion_n512_m1048576": dict(kind="tri", n=512, m=1 << 20, r=1.0, seed=SEED_BASE + 1),
    "hyperdiffusion_n1024_m262144": dict(kind="penta", n=1024, m=1 << 18, r=0.25, seed=SEED_BASE + 2),
    "cahn_hilliard_n256_m1048576": dict(kind="ch", n=256, m=1 << 20, gamma=0.01, dt=1e-3,
                                        steps=5000, seed=SEED_BASE + 3),
    "adjoint_diffusion_n1024_m65536": dict(kind="adjoint", n=1024, m=1 << 16, r=0.5, steps=100,
                                           checkpoint=10, seed=SEED_BASE + 4),
    # Cahn-Hilliard coarsening campaigns (Section 5, batched 1D scaling): 2^20
    # runs, dx = 2 pi / 256, dt = 0.1 dx, T = 100, gamma = 0.01, initial states
    # uniform[-0.1, 0.1); domain lengths 2 pi (n = 256) and 4 pi (n = 512)
    "ch_coarsening_L2pi": dict(kind="ch_coarsening", n=256, length=2.0 * math.pi, m=1 << 20,
                               gamma=0.01, T=100.0, seed=SEED_BASE + 7),
    "ch_coarsening_L4pi": dict(kind="ch_coarsening", n=512, length=4.0 * math.pi, m=1 << 20,
                               gamma=0.01, T=100.0, seed=SEED_BASE + 8),
    # forced Cahn-Hilliard flow-pattern batch (the forced flow-pattern
    # section): L = 2 pi, n = 512, dt = 0.1 dx, T = 50, gamma = 0.01, v and k
    # fixed per batch, a 768 x 768 grid of (f0 in [0, 2], <C> in [0, 1.5]),
    # initial states <C> + uniform[-0.1, 0.1)
    "ch_forced_flowmap_v05": dict(kind="ch_forced", n=512, length=2.0 * math.pi, grid=768,
                                  v=0.5, k=1.0, f0=(0.0, 2.0), mean=(0.0, 1.5), gamma=0.01,
                                  T=50.0, seed=SEED_BASE + 9),
    # Section 5.2 convergence study: C(x, 0) = eps cos(5x), eps = 1e-6,
    # L = 2 pi, gamma = 0.01, dt = 0.1 dx, one run per N = 128 .. 8192 and
    # the N = 16384 reference of E_8192; every N stops at the same time,
    # T = 204 dt_128 (about 1.0014, after the mode has grown to saturation),
    # i.e. 204 N / 128 steps
    "ch_convergence_1d": dict(kind="ch_convergence", ns=(128, 256, 512, 1024, 2048, 4096, 8192),
                              length=2.0 * math.pi, gamma=0.01, eps=1e-6, mode=5, steps128=204),
    # the same study of the forced scheme in the travelling frame (k = 1,
    # v = 0.5, f0 = 1), run to T = 50 (10200 steps at N = 128), the horizon
    # of the flow-pattern runs, where the travelling-frame state has settled
    "ch_forced_convergence_1d": dict(kind="ch_convergence", ns=(256, 512, 1024, 2048, 4096),
                                     length=2.0 * math.pi, gamma=0.01, eps=1e-6, mode=5,
                                     steps128=10200, forced=dict(v=0.5, f0=1.0, k=1.0),
                                     oracle_max_n=1024),
    # long systems (beyond one launch's on-chip limit), small batches where
    # the paper hands the work to the CPU, and one large batch
    "long_small_batch": dict(kind="long", ns=(4096, 8192, 16384), ms=(1, 8, 64, 512),
                             seed=SEED_BASE + 10),
    "long_tri_n8192_m65536": dict(kind="long", ns=(8192,), ms=(1 << 16,), seed=SEED_BASE + 11),
    # the FP64 tridiagonal sweep of the bench matrix (n = 512) over batch sizes
    # 2^16 .. 2^21, i.e. row strides of 512 KiB .. 16 MiB, beside the two
    # reference copies of the same bytes
    "tri_batch_sweep_n512": dict(kind="batch_sweep", n=512, ms=tuple(1 << e for e in range(16, 22)),
                                 r=1.0, seed=SEED_BASE + 12),
    # Crank-Nicolson time stepping on the grid of the paper's benchmark tables
    # (1000 steps; n = 64, 256, 1024; m = 2^6, 2^12, 2^16); the step size is
    # not printed; sigma = 1 is taken here (it does not change the work)
    "cn_diffusion_grid": dict(kind="cn", problem="diffusion", ns=(64, 256, 1024),
                              ms=(1 << 6, 1 << 12, 1 << 16), sigma=1.0, steps=1000,
                              seed=SEED_BASE + 5),
    "cn_hyperdiffusion_grid": dict(kind="cn", problem="hyperdiffusion", ns=(64, 256, 1024),
                                   ms=(1 << 6, 1 << 12, 1 << 16), sigma=1.0, steps=1000,
                                   seed=SEED_BASE + 6),
}
