"""Pins for the oracle's periodic solvers: Sherman-Morrison for the cyclic
tridiagonal matrix (Section 3.3) and the rank-2 Woodbury reading for the
cyclic pentadiagonal matrix of Section 5.1.  Constant periodic bands make a
circulant matrix, which the DFT diagonalises: an independent exact route."""
import math

import numpy as np
import pytest

from paper_2107_05395_amd import inputs
from tests.dense import exact_solve, penta_dense, rel_err, tri_dense


def circulant_solve(coeffs, rhs):
    """Solve sum_o coeffs[o] x_{i+o} = rhs_i (indices mod n) for every column."""
    n = rhs.shape[0]
    theta = 2.0 * math.pi * np.arange(n) / n
    eig = sum(v * np.exp(1j * o * theta) for o, v in coeffs.items())
    return np.real(np.fft.ifft(np.fft.fft(rhs, axis=0) / eig[:, None], axis=0))


@pytest.mark.parametrize("n", [3, 4, 5, 8, 31])
def test_cyclic_tri_vs_dense(oracle, n):
    a, b, c = inputs.random_dominant_tri(n, seed=500 + n)
    rhs = inputs.uniform_batch(n, 6, seed=600 + n)
    x = oracle.tri_solve(a, b, c, rhs, cyclic=True)
    ref = np.linalg.solve(tri_dense(a, b, c, cyclic=True), rhs)
    assert rel_err(x, ref) < 1e-14


def test_cyclic_tri_vs_exact_rationals(oracle):
    a = np.array([1.0, -2.0, 1.0, 0.0, 2.0])
    b = np.array([5.0, 6.0, -7.0, 4.0, 5.0])
    c = np.array([-1.0, 2.0, 3.0, 1.0, -2.0])
    d = np.array([3.0, -1.0, 4.0, 1.0, -5.0])
    exact = np.array([float(v) for v in exact_solve(tri_dense(a, b, c, cyclic=True), d)])
    assert np.max(np.abs(oracle.tri_solve1(a, b, c, d, cyclic=True) - exact)) < 1e-15


@pytest.mark.parametrize("n,sig", [(64, 0.3), (256, 2.0), (1000, 0.01)])
def test_cyclic_tri_vs_fft(oracle, n, sig):
    # periodic Crank-Nicolson diffusion LHS of Section 3.2: (-s, 1 + 2s, -s)
    a, b, c = np.full(n, -sig), np.full(n, 1 + 2 * sig), np.full(n, -sig)
    rhs = inputs.uniform_batch(n, 8, seed=n)
    ref = circulant_solve({-1: -sig, 0: 1 + 2 * sig, 1: -sig}, rhs)
    assert rel_err(oracle.tri_solve(a, b, c, rhs, cyclic=True), ref) < 1e-13


def test_cyclic_tri_nonsymmetric_fft(oracle):
    n = 97
    a, b, c = np.full(n, 0.7), np.full(n, -3.1), np.full(n, 1.9)
    rhs = inputs.uniform_batch(n, 4, seed=1)
    ref = circulant_solve({-1: 0.7, 0: -3.1, 1: 1.9}, rhs)
    assert rel_err(oracle.tri_solve(a, b, c, rhs, cyclic=True), ref) < 1e-13


@pytest.mark.parametrize("n", [5, 6, 7, 12, 40])
def test_cyclic_penta_vs_dense(oracle, n):
    bands = inputs.random_dominant_penta(n, seed=700 + n)
    rhs = inputs.uniform_batch(n, 5, seed=800 + n)
    x = oracle.penta_solve(*bands, rhs, cyclic=True)
    ref = np.linalg.solve(penta_dense(*bands, cyclic=True), rhs)
    assert rel_err(x, ref) < 1e-13


@pytest.mark.parametrize("n,sigma", [(256, 27.557), (64, 0.2), (512, 300.0)])
def test_cyclic_penta_ch_matrix_vs_fft(oracle, n, sigma):
    """Cahn-Hilliard LHS: eigenvalues 1 + sigma (2 - 2 cos theta)^2."""
    rhs = inputs.uniform_batch(n, 8, seed=n + 1)
    ref = circulant_solve({-2: sigma, -1: -4 * sigma, 0: 1 + 6 * sigma, 1: -4 * sigma, 2: sigma}, rhs)
    x = oracle.penta_solve(*inputs.ch_penta_bands(n, sigma), rhs, cyclic=True)
    assert rel_err(x, ref) < 1e-12


def test_cyclic_penta_general_constant_fft(oracle):
    n = 50
    v = {-2: 0.3, -1: -1.2, 0: 4.0, 1: 0.8, 2: -0.5}
    bands = [np.full(n, v[o]) for o in (-2, -1, 0, 1, 2)]
    rhs = inputs.uniform_batch(n, 4, seed=3)
    assert rel_err(oracle.penta_solve(*bands, rhs, cyclic=True), circulant_solve(v, rhs)) < 1e-13


def test_cyclic_sizes_rejected(oracle):
    with pytest.raises(ValueError, match="size"):
        oracle.tri_solve1([1, 1], [4, 4], [1, 1], [1, 1], cyclic=True)
    with pytest.raises(ValueError, match="size"):
        oracle.penta_solve1(*([np.ones(4)] * 5), np.ones(4), cyclic=True)
