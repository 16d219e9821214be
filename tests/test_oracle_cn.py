"""Pins for the oracle's Crank-Nicolson steps (Section 3 and Section 4
benchmark problems): dense linear algebra on small systems, the exact discrete
amplification factor of Fourier modes, and conservation of the mean."""
import math

import numpy as np
import pytest

from paper_2107_05395_amd import inputs
from tests.dense import penta_dense, rel_err, tri_dense


def _stencil_dense(w, n, cyclic):
    """The explicit operator B as a dense matrix: constant bands equal to the
    stencil weights, wrapped like A when periodic."""
    bands = [np.full(n, float(x)) for x in w]
    return tri_dense(*bands, cyclic=cyclic) if len(w) == 3 else penta_dense(*bands, cyclic=cyclic)


@pytest.mark.parametrize("nb", [3, 5])
@pytest.mark.parametrize("cyclic", [False, True])
@pytest.mark.parametrize("n", [6, 7, 16])
def test_cn_step_vs_dense(oracle, nb, cyclic, n):
    """Random row-dependent bands and a random non-symmetric stencil (a
    reversed or shifted stencil, a dropped wrap term or a wrong band all
    change the result); three steps against LAPACK."""
    seed = 100 * nb + 10 * cyclic + n
    bands = (inputs.random_dominant_tri(n, seed) if nb == 3 else
             inputs.random_dominant_penta(n, seed))
    w = inputs.rng(seed + 1).uniform(-1, 1, nb)
    c0 = inputs.uniform_batch(n, 4, seed=seed + 2)
    A = tri_dense(*bands, cyclic=cyclic) if nb == 3 else penta_dense(*bands, cyclic=cyclic)
    B = _stencil_dense(w, n, cyclic)
    ref = c0
    for _ in range(3):
        ref = np.linalg.solve(A, B @ ref)
    assert rel_err(oracle.cn_step(bands, w, c0, steps=3, cyclic=cyclic), ref) < 1e-12


@pytest.mark.parametrize("problem", ["diffusion", "hyperdiffusion"])
@pytest.mark.parametrize("n", [64, 256])
def test_cn_fourier_mode_amplification(oracle, problem, n):
    """A periodic constant-coefficient scheme maps a Fourier mode of wavenumber
    k onto itself times G = (1 - sigma L_k) / (1 + sigma L_k), with
    L_k = 2 - 2 cos(theta) (second difference) or (2 - 2 cos(theta))^2 (fourth
    difference), theta = 2 pi k / n."""
    sigma = 0.8
    bands, w = (oracle.cn_diffusion if problem == "diffusion" else oracle.cn_hyperdiffusion)(n, sigma)
    i = np.arange(n)
    steps = 40
    for k in (0, 1, 3, n // 4, n // 2 - 1, n // 2):
        th = 2 * math.pi * k / n
        lam = 2 - 2 * math.cos(th)
        L = lam if problem == "diffusion" else lam * lam
        G = (1 - sigma * L) / (1 + sigma * L)
        c0 = np.stack([np.cos(th * i), np.sin(th * i) + 0.0 * i], axis=1)
        out = oracle.cn_step(bands, w, c0, steps=steps)
        ref = G ** steps * c0
        scale = max(1.0, np.max(np.abs(c0)))
        assert np.max(np.abs(out - ref)) < 1e-12 * scale * steps, k


@pytest.mark.parametrize("problem", ["diffusion", "hyperdiffusion"])
def test_cn_mean_conserved(oracle, problem):
    """Every column of the periodic A and B sums to 1, so the sum over the
    system is unchanged by a step."""
    n, m = 128, 16
    bands, w = (oracle.cn_diffusion if problem == "diffusion" else oracle.cn_hyperdiffusion)(n, 2.5)
    c = inputs.uniform_batch(n, m, seed=inputs.SEED_BASE + 11)
    mass0 = c.sum(axis=0)
    c = oracle.cn_step(bands, w, c, steps=30)
    assert np.max(np.abs(c.sum(axis=0) - mass0)) < 1e-11


@pytest.mark.parametrize("cyclic", [False, True])
def test_cn_identity_stencil_is_a_plain_solve(oracle, cyclic):
    n = 40
    bands = inputs.random_dominant_penta(n, 7)
    c0 = inputs.uniform_batch(n, 3, seed=8)
    out = oracle.cn_step(bands, (0, 0, 1, 0, 0), c0, cyclic=cyclic)
    A = penta_dense(*bands, cyclic=cyclic)
    assert rel_err(out, np.linalg.solve(A, c0)) < 1e-13


def test_cn_problem_inputs_match_the_schemes(oracle):
    """The shared input generators build the same bands and stencils as the
    oracle's own reading of the two schemes."""
    for ours, theirs in ((inputs.cn_diffusion_problem, oracle.cn_diffusion),
                         (inputs.cn_hyperdiffusion_problem, oracle.cn_hyperdiffusion)):
        (b1, w1), (b2, w2) = ours(32, 0.37), theirs(32, 0.37)
        assert all(np.array_equal(x, y) for x, y in zip(b1, b2))
        assert np.array_equal(np.asarray(w1), np.asarray(w2))


def test_cn_step_leaves_its_input_alone(oracle):
    n = 32
    bands, w = oracle.cn_diffusion(n, 0.5)
    c = inputs.uniform_batch(n, 4, seed=5)
    keep = c.copy()
    oracle.cn_step(bands, w, c, steps=3)
    assert np.array_equal(c, keep)
