"""FP64 CPU oracle for batched banded solves with one shared left-hand side.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with the GPU library
(``paper_2107_05395_amd``); neither imports the other.

The arithmetic lives in ``bb_oracle.c`` (plain C, IEEE double, true divisions,
per-system loops); this module only marshals numpy arrays into it and strings
single steps together (time loops, transposition, loss).  Every routine names
the passage of Carroll et al., "A Batched GPU Methodology for Numerical
Solutions of Partial Differential Equations" (arXiv:2107.05395) that it
follows.

Array convention: a batch of m systems of size n is an (n, m) C-contiguous
float64 array -- element i of system k at [i, k], which is the interleaved
layout of Section 2 with leading dimension m.  A single system is a length-n
vector.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_ERRORS = {1: "zero or non-finite pivot", 2: "singular capacitance matrix", 3: "bad size"}


def build(force: bool = False) -> str:
    """Compile bb_oracle.c into liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_tri_solve.argtypes = [i64, P, P, P, P, P, P]
        lib.oracle_penta_solve.argtypes = [i64, P, P, P, P, P, P, P, P]
        lib.oracle_tri_cyclic_solve.argtypes = [i64, P, P, P, P, P, P]
        lib.oracle_penta_cyclic_solve.argtypes = [i64, P, P, P, P, P, P, P, P]
        lib.oracle_tri_transpose_bands.argtypes = [i64, P, P, P, P, P, P]
        lib.oracle_tri_transpose_bands.restype = None
        lib.oracle_penta_transpose_bands.argtypes = [i64] + [P] * 10
        lib.oracle_penta_transpose_bands.restype = None
        lib.oracle_solve_batch.argtypes = [ctypes.c_int, i64, i64, i64, P, P, P, P, P, P, P]
        lib.oracle_band_grad.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64, P, P, P]
        lib.oracle_band_grad.restype = None
        lib.oracle_ch_step_batch.argtypes = [i64, i64, i64, ctypes.c_double, ctypes.c_double, P, P]
        lib.oracle_cn_step_batch.argtypes = [ctypes.c_int, i64, i64, i64] + [P] * 8
        lib.oracle_weno5.argtypes = [P, i64, i64, ctypes.c_int]
        lib.oracle_weno5.restype = ctypes.c_double
        lib.oracle_ch_forced_step_batch.argtypes = [i64, i64, i64, ctypes.c_double, ctypes.c_double,
                                                    P, P, P, P, P]
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(status: int) -> None:
    if status:
        raise ValueError("oracle: " + _ERRORS.get(status, "status %d" % status))


def num_threads() -> int:
    """Threads the oracle's OpenMP regions use (OMP_NUM_THREADS or all cores)."""
    return int(_load().oracle_num_threads())


# --------------------------------------------------------------------------
# single systems (Section 3.1 Thomas, Section 4.1 LR, Section 3.3 Sherman-Morrison,
# rank-2 Woodbury for the periodic pentadiagonal matrix of Section 5.1)

def tri_solve1(a, b, c, d, cyclic: bool = False) -> np.ndarray:
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.shape[0]
    x = np.empty(n)
    w = np.empty(6 * n)
    fn = _load().oracle_tri_cyclic_solve if cyclic else _load().oracle_tri_solve
    _check(fn(n, _p(a), _p(b), _p(c), _p(d), _p(x), _p(w)))
    return x


def penta_solve1(a, b, c, d, e, f, cyclic: bool = False) -> np.ndarray:
    a, b, c, d, e, f = map(_f64, (a, b, c, d, e, f))
    n = f.shape[0]
    x = np.empty(n)
    w = np.empty(14 * n)
    fn = _load().oracle_penta_cyclic_solve if cyclic else _load().oracle_penta_solve
    _check(fn(n, _p(a), _p(b), _p(c), _p(d), _p(e), _p(f), _p(x), _p(w)))
    return x


# --------------------------------------------------------------------------
# batches in interleaved layout (Section 2): rhs is (n, m)

def _batch(kind: int, bands, rhs) -> np.ndarray:
    rhs = _f64(rhs)
    n, m = rhs.shape
    bands = [_f64(v) for v in bands] + [np.zeros(n)] * (5 - len(bands))
    for v in bands:
        if v.shape != (n,):
            raise ValueError("band length must equal n")
    x = np.empty_like(rhs)
    _check(_load().oracle_solve_batch(kind, n, m, m, *(_p(v) for v in bands), _p(rhs), _p(x)))
    return x


def tri_solve(a, b, c, rhs, cyclic: bool = False) -> np.ndarray:
    """x[:, k] = A^{-1} rhs[:, k] for a shared tridiagonal A (Section 3)."""
    return _batch(1 if cyclic else 0, (a, b, c), rhs)


def penta_solve(a, b, c, d, e, rhs, cyclic: bool = False) -> np.ndarray:
    """x[:, k] = A^{-1} rhs[:, k] for a shared pentadiagonal A (Section 4)."""
    return _batch(3 if cyclic else 2, (a, b, c, d, e), rhs)


def tri_transpose_bands(a, b, c):
    a, b, c = map(_f64, (a, b, c))
    n = a.shape[0]
    out = [np.empty(n) for _ in range(3)]
    _load().oracle_tri_transpose_bands(n, _p(a), _p(b), _p(c), *(_p(v) for v in out))
    return out


def penta_transpose_bands(a, b, c, d, e):
    a, b, c, d, e = map(_f64, (a, b, c, d, e))
    n = a.shape[0]
    out = [np.empty(n) for _ in range(5)]
    _load().oracle_penta_transpose_bands(n, _p(a), _p(b), _p(c), _p(d), _p(e),
                                         *(_p(v) for v in out))
    return out


def tri_adjoint(a, b, c, g, cyclic: bool = False) -> np.ndarray:
    """lam = A^{-T} g: an ordinary solve with the transposed bands."""
    return tri_solve(*tri_transpose_bands(a, b, c), g, cyclic=cyclic)


def penta_adjoint(a, b, c, d, e, g, cyclic: bool = False) -> np.ndarray:
    return penta_solve(*penta_transpose_bands(a, b, c, d, e), g, cyclic=cyclic)


def band_grad(lam, x, nbands: int, cyclic: bool = False) -> np.ndarray:
    """(nbands, n) array: grad[band, i] = -sum_k lam[i,k] x[i+off,k], off = band - nbands//2."""
    lam, x = _f64(lam), _f64(x)
    n, m = lam.shape
    g = np.empty((nbands, n))
    _load().oracle_band_grad(nbands, int(cyclic), n, m, m, _p(lam), _p(x), _p(g))
    return g


# --------------------------------------------------------------------------
# Cahn-Hilliard (Section 5.1)

def ch_coefficients(gamma: float, dx: float, dt: float):
    """sigma = gamma dt / dx^4 and alpha = dt / dx^2 of the semi-implicit scheme."""
    return gamma * dt / dx ** 4, dt / dx ** 2


def ch_bands(n: int, sigma: float):
    """Periodic pentadiagonal LHS bands a = e = sigma, b = d = -4 sigma, c = 1 + 6 sigma."""
    return (np.full(n, sigma), np.full(n, -4.0 * sigma), np.full(n, 1.0 + 6.0 * sigma),
            np.full(n, -4.0 * sigma), np.full(n, sigma))


def ch_step(c, sigma: float, alpha: float, steps: int = 1) -> np.ndarray:
    c = np.array(c, dtype=np.float64, order="C", copy=True)   # never write into the caller's array
    n, m = c.shape
    out = np.empty_like(c)
    for _ in range(steps):
        _check(_load().oracle_ch_step_batch(n, m, m, sigma, alpha, _p(c), _p(out)))
        c, out = out, c
    return c


# --------------------------------------------------------------------------
# Crank-Nicolson steppers of the benchmark problems (Section 3: periodic
# diffusion; Section 4: periodic hyperdiffusion).  A step is A C' = B C with B
# the explicit half of the scheme, a constant stencil w of 2K+1 weights.

def cn_diffusion(n: int, sigma: float):
    """LHS bands (-s, 1+2s, -s) and RHS stencil (s, 1-2s, s), s = dt/(2 dx^2)."""
    bands = (np.full(n, -sigma), np.full(n, 1.0 + 2.0 * sigma), np.full(n, -sigma))
    return bands, np.array([sigma, 1.0 - 2.0 * sigma, sigma])


def cn_hyperdiffusion(n: int, sigma: float):
    """LHS bands (s, -4s, 1+6s, -4s, s) and RHS stencil (-s, 4s, 1-6s, 4s, -s), s = dt/(2 dx^4)."""
    bands = (np.full(n, sigma), np.full(n, -4.0 * sigma), np.full(n, 1.0 + 6.0 * sigma),
             np.full(n, -4.0 * sigma), np.full(n, sigma))
    return bands, np.array([-sigma, 4.0 * sigma, 1.0 - 6.0 * sigma, 4.0 * sigma, -sigma])


def cn_step(bands, w, c, steps: int = 1, cyclic: bool = True) -> np.ndarray:
    """`steps` steps C <- A^{-1} (B C) of a batch c (n, m); 3 bands + 3 weights
    (tri) or 5 + 5 (penta).  Cyclic: B wraps mod n like A; else the terms of B
    outside the system are left out."""
    c = np.array(c, dtype=np.float64, order="C", copy=True)
    n, m = c.shape
    nb = len(bands)
    if nb not in (3, 5) or len(w) != nb:
        raise ValueError("need 3 bands and 3 weights (tri) or 5 and 5 (penta)")
    kind = (1 if cyclic else 0) if nb == 3 else (3 if cyclic else 2)
    bands = [_f64(v) for v in bands] + [np.zeros(n)] * (5 - nb)
    for v in bands:
        if v.shape != (n,):
            raise ValueError("band length must equal n")
    w = _f64(w)
    out = np.empty_like(c)
    for _ in range(steps):
        _check(_load().oracle_cn_step_batch(kind, n, m, m, *(_p(v) for v in bands), _p(w),
                                            _p(c), _p(out)))
        c, out = out, c
    return c


# --------------------------------------------------------------------------
# Forced Cahn-Hilliard equation in the frame of the travelling wave (the
# forced flow-pattern section): the Section 5.1 step plus an advection term
# v dC/deta, differenced with the fifth-order Hamilton-Jacobi WENO scheme the
# paper cites, and the forcing f0 k cos(k eta), with v, f0, k per run.

def weno5(phi, plus: bool) -> np.ndarray:
    """dx times the one-sided WENO5 derivative of a periodic grid function at
    every point (right-biased when plus)."""
    phi = _f64(phi)
    n = phi.shape[0]
    return np.array([_load().oracle_weno5(_p(phi), n, i, int(plus)) for i in range(n)])


def ch_forced_parameters(dt: float, dx: float, v, f0, k):
    """Per-run (beta, amp, kdx) = (dt v / dx, dt f0 k, k dx)."""
    v, f0, k = (np.asarray(x, dtype=np.float64) for x in (v, f0, k))
    return dt * v / dx, dt * f0 * k, k * dx


def ch_forced_step(c, sigma: float, alpha: float, beta, amp, kdx, steps: int = 1) -> np.ndarray:
    c = np.array(c, dtype=np.float64, order="C", copy=True)
    n, m = c.shape
    beta, amp, kdx = (np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (m,)))
                      for x in (beta, amp, kdx))
    out = np.empty_like(c)
    for _ in range(steps):
        _check(_load().oracle_ch_forced_step_batch(n, m, m, sigma, alpha, _p(beta), _p(amp),
                                                   _p(kdx), _p(c), _p(out)))
        c, out = out, c
    return c


# --------------------------------------------------------------------------
# Coarsening statistics of Cahn-Hilliard ensembles (Section 5, batched 1D
# scaling): the typical domain size of one run, l = 1 / (1 - <C^2>), with
# <C^2> the mean over the periodic domain (the rectangle rule on the n grid
# points, exact for the grid function), and its mean over the runs.

def ch_domain_size(c) -> np.ndarray:
    """l_k = 1 / (1 - (1/n) sum_i c[i,k]^2) for every run k of an (n, m) batch."""
    c = _f64(c)
    n = c.shape[0]
    return 1.0 / (1.0 - np.sum(c * c, axis=0) / n)


def ch_coarsening(c0, sigma: float, alpha: float, steps: int, every: int):
    """Mean domain size over the runs after every `every` steps: returns
    (lbar of length steps // every, final state)."""
    c = _f64(c0)
    lbar = []
    for _ in range(steps // every):
        c = ch_step(c, sigma, alpha, steps=every)
        lbar.append(float(np.mean(ch_domain_size(c))))
    rest = steps - every * (steps // every)
    if rest:
        c = ch_step(c, sigma, alpha, steps=rest)
    return np.array(lbar), c


# --------------------------------------------------------------------------
# Implicit-Euler diffusion with a spatially varying coefficient, differentiated
# through T steps.  Discretisation: A(D) = I + r diag(D) T2 with T2 the
# zero-Dirichlet second-difference matrix tridiag(-1, 2, -1), i.e. row i is
# (-r D_i, 1 + 2 r D_i, -r D_i).

def diffusion_bands(D, r: float):
    D = _f64(D)
    return -r * D, 1.0 + 2.0 * r * D, -r * D


def diffusion_loss_and_grads(D, r: float, u0, target, steps: int):
    """Loss = mean over all n*m entries of (u_T - target)^2 with u_t = A(D)^{-1} u_{t-1}.

    Returns (loss, dL/dD (n,), dL/du0 (n, m)).  The gradient is the adjoint
    recursion lam_t = A^{-T} g_t, g_{t-1} = lam_t, g_T = 2 (u_T - target)/(n m),
    with dL/dA_ij = -sum_t sum_k lam_t[i,k] u_t[j,k] mapped to D by
    dA/dD_i = r * (row i of T2).  Stores every state (small sizes only).
    """
    a, b, c = diffusion_bands(D, r)
    u = [_f64(u0)]
    for _ in range(steps):
        u.append(tri_solve(a, b, c, u[-1]))
    n, m = u[0].shape
    diff = u[-1] - _f64(target)
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / (n * m)
    gbands = np.zeros((3, n))
    for t in range(steps, 0, -1):
        lam = tri_adjoint(a, b, c, g)
        gbands += band_grad(lam, u[t], 3)
        g = lam
    dD = r * (-gbands[0] + 2.0 * gbands[1] - gbands[2])
    return loss, dD, g
