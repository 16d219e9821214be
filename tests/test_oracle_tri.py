"""Pins for the oracle's tridiagonal (Thomas) solver, Section 3.1.

Each check compares against something other than the oracle's own recurrence:
dense LAPACK with pivoting, exact rational elimination, the closed-form decay
of Dirichlet sine modes, a banded LAPACK routine, and the residual."""
import math

import numpy as np
import pytest
import scipy.linalg

from paper_2107_05395_amd import inputs
from tests.dense import exact_solve, rel_err, tri_dense


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 17, 64])
def test_tri_vs_dense_lapack(oracle, n):
    a, b, c = inputs.random_dominant_tri(n, seed=100 + n)
    rhs = inputs.uniform_batch(n, 7, seed=200 + n)
    x = oracle.tri_solve(a, b, c, rhs)
    ref = np.linalg.solve(tri_dense(a, b, c), rhs)
    assert rel_err(x, ref) < 1e-14


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_tri_vs_exact_rationals(oracle, n):
    g = np.random.default_rng(7 + n)
    a = g.integers(-3, 4, n).astype(float)
    c = g.integers(-3, 4, n).astype(float)
    b = np.abs(a) + np.abs(c) + g.integers(1, 4, n)
    d = g.integers(-9, 10, n).astype(float)
    exact = exact_solve(tri_dense(a, b, c), d)
    x = oracle.tri_solve1(a, b, c, d)
    assert np.max(np.abs(x - np.array([float(v) for v in exact]))) <= 1e-14 * max(1.0, np.max(np.abs(x)))


@pytest.mark.parametrize("n,r", [(256, 0.5), (512, 1.0), (1024, 0.5)])
def test_tri_sine_mode_decay(oracle, n, r):
    """A = I + r T2 (zero Dirichlet) maps sin(k pi i/(n+1)) to itself scaled by
    1 / (1 + r lambda_k), lambda_k = 4 sin^2(k pi / (2(n+1)))."""
    a, b, c = inputs.diffusion_tri_bands(n, r)
    i = np.arange(1, n + 1)
    ks = [1, 2, 7, n // 3, n - 1, n]
    # reduce k*i mod 2(n+1) exactly in integers so the sines carry no argument error
    rhs = np.stack([np.sin(math.pi * ((k * i) % (2 * (n + 1))) / (n + 1)) for k in ks], axis=1)
    lam = np.array([4.0 * math.sin(k * math.pi / (2 * (n + 1))) ** 2 for k in ks])
    ref = rhs / (1.0 + r * lam)[None, :]
    x = oracle.tri_solve(a, b, c, rhs)
    assert rel_err(x, ref) < 1e-13


def test_tri_vs_solve_banded_full_size(oracle):
    n, m = 512, 256
    a, b, c = inputs.diffusion_tri_bands(n, 1.0)
    rhs = inputs.uniform_batch(n, m, seed=inputs.SEED_BASE + 1)
    ab = np.zeros((3, n))
    ab[0, 1:] = c[:-1]
    ab[1] = b
    ab[2, :-1] = a[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    x = oracle.tri_solve(a, b, c, rhs)
    assert rel_err(x, ref) < 1e-14


def test_tri_residual_row_dependent(oracle):
    n, m = 300, 64
    a, b, c = inputs.random_dominant_tri(n, seed=5, margin=0.05)
    rhs = inputs.uniform_batch(n, m, seed=6)
    x = oracle.tri_solve(a, b, c, rhs)
    res = tri_dense(a, b, c) @ x - rhs
    assert np.max(np.linalg.norm(res, axis=0) / np.linalg.norm(rhs, axis=0)) < 1e-14


def test_tri_zero_pivot_detected(oracle):
    # b_1 = 0 stops the factorisation at its first step
    with pytest.raises(ValueError, match="pivot"):
        oracle.tri_solve1([0, 1, 1], [0, 1, 1], [1, 1, 0], [1, 2, 3])
    # nonsingular (det = -1) but its leading 2x2 minor is singular: b^_2 = 0
    a, b, c = [0.0, 1.0, 1.0], [1.0, 1.0, 2.0], [1.0, 1.0, 0.0]
    assert abs(np.linalg.det(tri_dense(a, b, c)) + 1.0) < 1e-12
    with pytest.raises(ValueError, match="pivot"):
        oracle.tri_solve1(a, b, c, [1.0, 2.0, 3.0])


def test_tri_ignores_unused_corners(oracle):
    n = 9
    a, b, c = inputs.random_dominant_tri(n, seed=3)
    d = np.arange(n, dtype=float)
    x1 = oracle.tri_solve1(a, b, c, d)
    a2, c2 = a.copy(), c.copy()
    a2[0], c2[-1] = 1e300, -7.0
    assert np.array_equal(x1, oracle.tri_solve1(a2, b, c2, d))
