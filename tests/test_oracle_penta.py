"""Pins for the oracle's pentadiagonal (LR) solver, Section 4.1."""
import math

import numpy as np
import pytest
import scipy.linalg

from paper_2107_05395_amd import inputs
from tests.dense import exact_solve, penta_dense, rel_err


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 9, 33])
def test_penta_vs_dense_lapack(oracle, n):
    bands = inputs.random_dominant_penta(n, seed=300 + n)
    rhs = inputs.uniform_batch(n, 5, seed=400 + n)
    x = oracle.penta_solve(*bands, rhs)
    ref = np.linalg.solve(penta_dense(*bands), rhs)
    assert rel_err(x, ref) < 1e-14


@pytest.mark.parametrize("n", [3, 4, 6])
def test_penta_vs_exact_rationals(oracle, n):
    g = np.random.default_rng(11 + n)
    a, b, d, e = (g.integers(-2, 3, n).astype(float) for _ in range(4))
    c = np.abs(a) + np.abs(b) + np.abs(d) + np.abs(e) + g.integers(1, 3, n)
    f = g.integers(-9, 10, n).astype(float)
    exact = np.array([float(v) for v in exact_solve(penta_dense(a, b, c, d, e), f)])
    x = oracle.penta_solve1(a, b, c, d, e, f)
    assert np.max(np.abs(x - exact)) <= 1e-14 * max(1.0, np.max(np.abs(exact)))


@pytest.mark.parametrize("n,r", [(64, 0.25), (1024, 0.25), (257, 3.0)])
def test_penta_squared_laplacian_modes(oracle, n, r):
    """I + r T2^2 (T2 = zero-Dirichlet tridiag(-1,2,-1)) has the sine modes as
    eigenvectors with eigenvalues 1 + r lambda_k^2; T2^2 has bands
    (1, -4, 6, -4, 1) except for 5 in its first and last diagonal entries."""
    a, b, c, d, e = inputs.hyperdiffusion_penta_bands(n, r)
    c = c.copy()
    c[0] = c[-1] = 1.0 + 5.0 * r
    i = np.arange(1, n + 1)
    ks = [1, 3, 8, n // 2, n]
    # reduce k*i mod 2(n+1) exactly in integers so the sines carry no argument error
    rhs = np.stack([np.sin(math.pi * ((k * i) % (2 * (n + 1))) / (n + 1)) for k in ks], axis=1)
    lam = np.array([4.0 * math.sin(k * math.pi / (2 * (n + 1))) ** 2 for k in ks])
    ref = rhs / (1.0 + r * lam ** 2)[None, :]
    assert rel_err(oracle.penta_solve(a, b, c, d, e, rhs), ref) < 1e-13


def test_penta_vs_solve_banded_hyperdiffusion(oracle):
    n, m = 1024, 64
    a, b, c, d, e = inputs.hyperdiffusion_penta_bands(n, 0.25)
    rhs = inputs.sine_mode_batch(n, m, seed=inputs.SEED_BASE + 2)
    ab = np.zeros((5, n))
    ab[0, 2:] = e[:-2]
    ab[1, 1:] = d[:-1]
    ab[2] = c
    ab[3, :-1] = b[1:]
    ab[4, :-2] = a[2:]
    ref = scipy.linalg.solve_banded((2, 2), ab, rhs)
    x = oracle.penta_solve(a, b, c, d, e, rhs)
    assert rel_err(x, ref) < 1e-13
    res = penta_dense(a, b, c, d, e) @ x - rhs
    assert np.max(np.linalg.norm(res, axis=0) / np.linalg.norm(rhs, axis=0)) < 1e-14


def test_penta_reduces_to_tri(oracle):
    n = 40
    a, b, c = inputs.random_dominant_tri(n, seed=9)
    z = np.zeros(n)
    rhs = inputs.uniform_batch(n, 3, seed=10)
    assert rel_err(oracle.penta_solve(z, a, b, c, z, rhs), oracle.tri_solve(a, b, c, rhs)) < 1e-15


def test_penta_zero_pivot_detected(oracle):
    n = 6
    a, b, c, d, e = inputs.random_dominant_penta(n, seed=2)
    c = c.copy()
    c[0] = 0.0
    with pytest.raises(ValueError, match="pivot"):
        oracle.penta_solve1(a, b, c, d, e, np.ones(n))
