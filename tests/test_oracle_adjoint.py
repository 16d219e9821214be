"""Pins for the oracle's adjoint solve, band gradients and the differentiated
implicit-Euler diffusion workload: dense transposed solves, autograd through a
dense torch solve (FP64, CPU), and central finite differences."""
import numpy as np
import pytest
import torch

from paper_2107_05395_amd import inputs
from tests.dense import penta_dense, rel_err, tri_dense


@pytest.mark.parametrize("cyclic", [False, True])
def test_tri_adjoint_vs_dense(oracle, cyclic):
    n = 13
    a, b, c = inputs.random_dominant_tri(n, seed=21)
    g = inputs.uniform_batch(n, 4, seed=22)
    ref = np.linalg.solve(tri_dense(a, b, c, cyclic).T, g)
    assert rel_err(oracle.tri_adjoint(a, b, c, g, cyclic=cyclic), ref) < 1e-14


@pytest.mark.parametrize("cyclic", [False, True])
def test_penta_adjoint_vs_dense(oracle, cyclic):
    n = 11
    bands = inputs.random_dominant_penta(n, seed=23)
    g = inputs.uniform_batch(n, 4, seed=24)
    ref = np.linalg.solve(penta_dense(*bands, cyclic).T, g)
    assert rel_err(oracle.penta_adjoint(*bands, g, cyclic=cyclic), ref) < 1e-14


def _dense_from_bands_torch(bands, cyclic):
    nb = len(bands)
    n = bands[0].shape[0]
    A = torch.zeros(n, n, dtype=torch.float64)
    half = nb // 2
    rows = torch.arange(n)
    for band, vals in enumerate(bands):
        cols = rows + band - half
        keep = (cols >= 0) & (cols < n)
        if cyclic:
            cols = cols % n
            keep = torch.ones(n, dtype=torch.bool)
        A = A.index_put((rows[keep], cols[keep]), vals[keep], accumulate=True)
    return A


@pytest.mark.parametrize("nb,cyclic", [(3, False), (3, True), (5, False), (5, True)])
def test_band_grad_vs_autograd(oracle, nb, cyclic):
    """L = sum(w * x), x = A^{-1} b: dL/dband from autograd through a dense solve
    equals -sum_k lam[i,k] x[i+off,k] with lam = A^{-T} w."""
    n, m = 12, 6
    np_bands = (inputs.random_dominant_tri(n, seed=31) if nb == 3
                else inputs.random_dominant_penta(n, seed=32))
    rhs = inputs.uniform_batch(n, m, seed=33)
    w = inputs.uniform_batch(n, m, seed=34)
    tb = [torch.tensor(v, requires_grad=True) for v in np_bands]
    A = _dense_from_bands_torch(tb, cyclic)
    x = torch.linalg.solve(A, torch.tensor(rhs))
    (x * torch.tensor(w)).sum().backward()
    auto = np.stack([t.grad.numpy() for t in tb])
    if nb == 3:
        lam = oracle.tri_adjoint(*np_bands, w, cyclic=cyclic)
        xs = oracle.tri_solve(*np_bands, rhs, cyclic=cyclic)
    else:
        lam = oracle.penta_adjoint(*np_bands, w, cyclic=cyclic)
        xs = oracle.penta_solve(*np_bands, rhs, cyclic=cyclic)
    g = oracle.band_grad(lam, xs, nb, cyclic=cyclic)
    if not cyclic:  # entries outside the matrix have no gradient
        half = nb // 2
        for band in range(nb):
            off = band - half
            for i in range(n):
                if not 0 <= i + off < n:
                    auto[band, i] = 0.0
    assert np.max(np.abs(g - auto)) < 1e-13 * max(1.0, np.max(np.abs(auto)))


def _dense_diffusion_loss(D, r, u0, target, steps):
    n = D.shape[0]
    T2 = (torch.diag(torch.full((n,), 2.0, dtype=torch.float64))
          - torch.diag(torch.ones(n - 1, dtype=torch.float64), 1)
          - torch.diag(torch.ones(n - 1, dtype=torch.float64), -1))
    A = torch.eye(n, dtype=torch.float64) + r * D[:, None] * T2
    u = u0
    for _ in range(steps):
        u = torch.linalg.solve(A, u)
    return ((u - target) ** 2).mean()


def test_diffusion_gradients_vs_autograd_dense(oracle):
    n, m, steps, r = 16, 5, 7, 0.5
    D = inputs.rng(41).uniform(0.5, 1.5, n)
    u0 = inputs.uniform_batch(n, m, seed=42)
    y = inputs.uniform_batch(n, m, seed=43)
    loss, dD, du0 = oracle.diffusion_loss_and_grads(D, r, u0, y, steps)
    tD = torch.tensor(D, requires_grad=True)
    tu = torch.tensor(u0, requires_grad=True)
    tl = _dense_diffusion_loss(tD, r, tu, torch.tensor(y), steps)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-15 * max(1.0, abs(loss)) + 1e-16
    assert np.max(np.abs(dD - tD.grad.numpy())) < 1e-14 * np.max(np.abs(dD))
    assert np.max(np.abs(du0 - tu.grad.numpy())) < 1e-14 * np.max(np.abs(du0))


def test_diffusion_gradients_vs_central_differences(oracle):
    n, m, steps, r = 20, 3, 10, 0.5
    D = inputs.rng(51).uniform(0.5, 1.5, n)
    u0 = inputs.uniform_batch(n, m, seed=52)
    y = inputs.uniform_batch(n, m, seed=53)
    _, dD, du0 = oracle.diffusion_loss_and_grads(D, r, u0, y, steps)
    g = np.random.default_rng(54)
    h = 1e-5
    for _ in range(3):
        vD = g.standard_normal(n)
        lp = oracle.diffusion_loss_and_grads(D + h * vD, r, u0, y, steps)[0]
        lm = oracle.diffusion_loss_and_grads(D - h * vD, r, u0, y, steps)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dD @ vD) <= 1e-7 * abs(fd) + 1e-12
        vu = g.standard_normal((n, m))
        lp = oracle.diffusion_loss_and_grads(D, r, u0 + h * vu, y, steps)[0]
        lm = oracle.diffusion_loss_and_grads(D, r, u0 - h * vu, y, steps)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.sum(du0 * vu)) <= 1e-7 * abs(fd) + 1e-12
