"""GPU parity of the fused Crank-Nicolson steps (Section 3 and Section 4
benchmark problems: periodic diffusion and hyperdiffusion, and their
non-periodic forms) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2107_05395_amd import inputs
from tests.gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    from paper_2107_05395_amd import solver  # noqa: F401
    oracle.build()


def _problem(kind, n, sigma):
    return (inputs.cn_diffusion_problem(n, sigma) if kind == "tri" else
            inputs.cn_hyperdiffusion_problem(n, sigma))


def _factor(kind, bands, cyclic):
    from paper_2107_05395_amd import Factor
    return Factor.tri(*bands, cyclic=cyclic) if kind == "tri" else Factor.penta(*bands, cyclic=cyclic)


# n: 64 (one chunk per system), 256 and 512 (one chunk per wave, 4 and 8
# waves), 1024 (16 chunks, LDS kernel), ragged 100 / 1000 / 333, tiny 5 / 7
CASES = [(kind, cyc, n) for kind in ("tri", "penta") for cyc in (True, False)
         for n in (64, 256, 512, 1024, 100, 333, 1000, 7)] + [("penta", True, 5), ("tri", True, 3)]


@pytest.mark.parametrize("kind,cyclic,n", CASES)
def test_cn_steps_match_oracle(kind, cyclic, n):
    m, steps = 300, 6   # 300 systems: several groups and a ragged last group
    say("cn", kind, "cyclic" if cyclic else "open", "n", n, "m", m)
    bands, w = _problem(kind, n, 0.7)
    if not cyclic:   # a non-symmetric stencil and row-dependent bands as well
        bands = (inputs.random_dominant_tri(n, n) if kind == "tri" else inputs.random_dominant_penta(n, n))
        w = tuple(inputs.rng(n + 1).uniform(-1, 1, len(w)))
    f = _factor(kind, bands, cyclic)
    c0 = inputs.uniform_batch(n, m, seed=40 + n)
    ref = oracle.cn_step(bands, w, c0, steps=steps, cyclic=cyclic)
    out = host(f.cn_step(dev(c0), w, steps=steps))
    err = rel_err(out, ref)
    say("  rel err", err)
    assert err < 1e-12


@pytest.mark.parametrize("kind", ["tri", "penta"])
@pytest.mark.parametrize("chunk", ["4", "8", "16", "32"])
def test_cn_chunk_sizes_match_oracle(kind, chunk, tuning):
    """Every chunk size the stepper is built for, full (n = 256) and ragged
    (n = 250) decompositions, against the oracle."""
    tuning.set("max_chunk", chunk)
    for n in (256, 250):
        bands, w = _problem(kind, n, 1.3)
        f = _factor(kind, bands, True)
        c0 = inputs.uniform_batch(n, 130, seed=50 + n)
        ref = oracle.cn_step(bands, w, c0, steps=5)
        assert rel_err(host(f.cn_step(dev(c0), w, steps=5)), ref) < 1e-12, (n, chunk)


@pytest.mark.parametrize("kind,n", [("tri", 64), ("tri", 256), ("tri", 512), ("tri", 1024),
                                    ("tri", 2048), ("penta", 64), ("penta", 256), ("penta", 512),
                                    ("penta", 1024)])
def test_cn_kernel_variants_agree_bitwise(kind, n, tuning):
    """One chunk per wave with scalar coefficients, a group split over several
    waves with the table in LDS, and one wave per group with the table in LDS
    do the same arithmetic in the same order: bitwise equal results, at a
    batch large enough for 64-row chunks (2^16 + 37 systems, ragged last
    group); sampled systems against the oracle."""
    m, steps = (1 << 16) + 37, 3
    say("cn variants", kind, n)
    bands, w = _problem(kind, n, 0.9)
    f = _factor(kind, bands, True)
    c0h = inputs.uniform_batch(n, m, seed=60 + n)
    c0 = dev(c0h)
    say("  plan", f.plan(m, stepper=True))
    a = host(f.cn_step(c0, w, steps=steps))
    cols = np.r_[np.arange(0, m, 997), m - 5:m]
    ref = oracle.cn_step(bands, w, np.ascontiguousarray(c0h[:, cols]), steps=steps)
    assert rel_err(a[:, cols], ref) < 1e-12
    tuning.set("ch_uniform", "0")
    b = host(f.cn_step(c0, w, steps=steps))
    assert np.array_equal(a, b)
    tuning.set("waves_per_system", "1")
    b = host(f.cn_step(c0, w, steps=steps))
    assert np.array_equal(a, b)
    for q in ("2", "4", "8"):
        if (1 << {"2": 1, "4": 2, "8": 3}[q]) <= n // 64:
            tuning.set("waves_per_system", q)
            assert np.array_equal(a, host(f.cn_step(c0, w, steps=steps))), q


@pytest.mark.parametrize("kind", ["tri", "penta"])
def test_cn_split_groups_with_32_row_chunks(kind, tuning):
    """32-row chunks split over 2, 4 and 8 waves (LDS table) equal one wave per
    group, bitwise, and match the oracle."""
    tuning.set("max_chunk", "32")
    n, m = 1024, 5000
    bands, w = _problem(kind, n, 1.1)
    f = _factor(kind, bands, True)
    c0h = inputs.uniform_batch(n, m, seed=65)
    c0 = dev(c0h)
    a = host(f.cn_step(c0, w, steps=4))
    assert rel_err(a, oracle.cn_step(bands, w, c0h, steps=4)) < 1e-12
    for q in ("1", "2", "4", "8"):
        tuning.set("waves_per_system", q)
        assert np.array_equal(a, host(f.cn_step(c0, w, steps=4))), q


@pytest.mark.parametrize("kind", ["tri", "penta"])
def test_cn_fused_steps_equal_single_steps_and_in_place(kind):
    """k steps in one launch equal k launches of one step (the state passes
    through memory unchanged in double), and in-place calls equal
    out-of-place ones."""
    n, m = 512, 777
    bands, w = _problem(kind, n, 2.0)
    f = _factor(kind, bands, True)
    c0 = dev(inputs.uniform_batch(n, m, seed=70))
    fused = host(f.cn_step(c0, w, steps=8))
    t = c0.clone()
    for _ in range(8):
        t = f.cn_step(t, w)
    assert np.array_equal(host(t), fused)
    t = c0.clone()
    f.cn_step(t, w, steps=8, out=t)
    assert np.array_equal(host(t), fused)


@pytest.mark.parametrize("kind", ["tri", "penta"])
def test_cn_fourier_modes_and_mean_at_size(kind):
    """A Fourier mode of wavenumber k is multiplied by the exact factor
    G_k = (1 - s L_k)/(1 + s L_k) per step, and the mean is conserved, at a
    workload size of the paper's grid (n = 1024, 2^12 systems, 100 steps)."""
    n, m, steps, s = 1024, 1 << 12, 100, 0.6
    bands, w = _problem(kind, n, s)
    f = _factor(kind, bands, True)
    i = np.arange(n)
    ks = np.arange(m) % (n // 2 + 1)
    c0 = np.cos(2 * math.pi * np.outer(i, ks) / n)
    out = host(f.cn_step(dev(c0), w, steps=steps))
    lam = 2 - 2 * np.cos(2 * math.pi * ks / n)
    L = lam if kind == "tri" else lam * lam
    G = (1 - s * L) / (1 + s * L)
    err = np.max(np.abs(out - c0 * G ** steps))
    say("cn", kind, "mode error", err)
    assert err < 1e-12 * steps
    # the sum is exact in exact arithmetic; each step may move it by a few
    # n eps |f|, with |f| <= sum |w| max |c| and max |c| <= 1 here
    rnd = inputs.uniform_batch(n, 256, seed=71)
    out = host(f.cn_step(dev(rnd), w, steps=steps))
    bound = 8 * steps * n * np.finfo(float).eps * float(np.sum(np.abs(w)))
    assert np.max(np.abs(out.sum(axis=0) - rnd.sum(axis=0))) < bound


def test_cn_rejects_wrong_stencil_length():
    bands, w = _problem("tri", 64, 0.5)
    f = _factor("tri", bands, True)
    with pytest.raises(ValueError):
        f.cn_step(dev(inputs.uniform_batch(64, 4, seed=1)), (1, 2, 3, 4, 5))


@pytest.mark.parametrize("kind,n", [("tri", 64), ("tri", 128), ("tri", 256), ("penta", 64),
                                    ("penta", 256)])
def test_cn_short_chunk_scalar_kernel_matches_lds(kind, n, tuning):
    """Small batches take 16- or 32-row chunks; when they tile n into at most
    eight the scalar-coefficient kernel runs them: bitwise what the LDS
    kernel gives, and the oracle's result."""
    m = 1000
    bands, w = _problem(kind, n, 0.8)
    f = _factor(kind, bands, True)
    c0h = inputs.uniform_batch(n, m, seed=80 + n)
    c0 = dev(c0h)
    pl = f.plan(m, stepper=True)
    assert pl["scalar"] and pl["chunk"] in (16, 32), pl
    a = host(f.cn_step(c0, w, steps=7))
    assert rel_err(a, oracle.cn_step(bands, w, c0h, steps=7)) < 1e-12
    tuning.set("ch_uniform", "0")
    assert not f.plan(m, stepper=True)["scalar"]
    assert np.array_equal(a, host(f.cn_step(c0, w, steps=7)))


# decompositions: n = 256 one chunk per wave (scalar coefficients), 1024 the
# LDS split kernel (16 chunks, 8 waves), 1000 / 333 ragged (one wave per
# group), 7 tiny; m = 300 takes the small-batch chunks, 5000 the large ones
TRAJ_CASES = [("tri", True, 256, 5000), ("tri", False, 1024, 5000), ("tri", True, 1000, 300),
              ("penta", True, 256, 5000), ("penta", False, 1024, 5000), ("penta", True, 333, 300),
              ("tri", False, 7, 70), ("penta", True, 5, 33)]


@pytest.mark.parametrize("kind,cyclic,n,m", TRAJ_CASES)
def test_cn_trajectory_equals_single_steps(kind, cyclic, n, m):
    """Every state of a trajectory launch is bitwise the state after the same
    number of single-step launches, the last one equals the fused launch, and
    the states match the oracle."""
    say("trajectory", kind, cyclic, n, m)
    bands, w = _problem(kind, n, 0.9)
    f = _factor(kind, bands, cyclic)
    c0h = inputs.uniform_batch(n, m, seed=90 + n)
    c0 = dev(c0h)
    steps = 6
    traj = f.cn_trajectory(c0, w, steps)
    assert traj.shape == (steps, n, m)
    t = c0
    for s in range(steps):
        t = f.cn_step(t, w)
        assert np.array_equal(host(traj[s]), host(t)), s
    assert np.array_equal(host(traj[-1]), host(f.cn_step(c0, w, steps=steps)))
    assert rel_err(host(traj[2]), oracle.cn_step(bands, w, c0h, steps=3, cyclic=cyclic)) < 1e-12


def test_cn_trajectory_strided_and_identity_stencil():
    """A strided batch (ld > m) gives the same states as a contiguous one;
    with the identity stencil the states are implicit solves A u' = u,
    checked against the oracle's solves."""
    n, m, ld, steps = 512, 1000, 1152, 4
    bands = inputs.diffusion_tri_bands(n, 0.7)
    f = _factor("tri", bands, False)
    c0h = inputs.uniform_batch(n, m, seed=95)
    big = torch.zeros(n, ld, dtype=torch.float64, device="cuda")
    big[:, :m] = dev(c0h)
    ident = (0.0, 1.0, 0.0)
    ts = f.cn_trajectory(big[:, :m], ident, steps)
    assert ts.stride(1) == ld
    tc = f.cn_trajectory(dev(c0h), ident, steps)
    u = c0h
    for s in range(steps):
        assert np.array_equal(host(ts[s]), host(tc[s])), s
        u = oracle.tri_solve(*bands, u)
        assert rel_err(host(tc[s]), u) < 1e-12, s
    with pytest.raises(ValueError):
        f.cn_trajectory(dev(c0h), ident, 0)


@pytest.mark.parametrize("kind,n,m", [("tri", 256, 5000), ("penta", 512, 3000), ("tri", 1024, 3000)])
def test_cn_grid_shapes_agree_bitwise(kind, n, m, tuning):
    """The scalar-coefficient stepper runs one workgroup per group by
    default, the LDS kernels a persistent grid; forcing either grid shape
    everywhere changes which workgroup runs a group, never its arithmetic."""
    bands, w = _problem(kind, n, 0.7)
    f = _factor(kind, bands, True)
    c0 = dev(inputs.uniform_batch(n, m, seed=97))
    ref = host(f.cn_step(c0, w, steps=4))
    for v in ("0", "1"):
        tuning.set("grid_linear", v)
        assert np.array_equal(host(f.cn_step(c0, w, steps=4)), ref), v
        assert np.array_equal(host(f.cn_trajectory(c0, w, 4)[-1]), ref), v


@pytest.mark.parametrize("kind,cyclic,n,m", [("tri", False, 1024, 3000), ("tri", True, 512, 700),
                                             ("penta", False, 1024, 2000), ("penta", True, 256, 5000),
                                             ("tri", False, 64, 70000), ("penta", True, 7, 33)])
def test_adjoint_trajectory_is_repeated_transposed_solves(kind, cyclic, n, m):
    """bb_adjoint_trajectory: lam_{s+1} = A^{-T} lam_s with the factor's own
    transposed solve, every state against the oracle's transposed solves
    (row-dependent, non-symmetric bands)."""
    say("adjoint trajectory", kind, cyclic, n, m)
    from paper_2107_05395_amd import Factor
    bands = (inputs.random_dominant_tri(n, seed=n) if kind == "tri"
             else inputs.random_dominant_penta(n, seed=n))
    f = Factor.tri(*bands, cyclic=cyclic) if kind == "tri" else Factor.penta(*bands, cyclic=cyclic)
    gh = inputs.uniform_batch(n, m, seed=7 * n + m)
    steps = 5
    traj = f.adjoint_trajectory(dev(gh), steps)
    assert traj.shape == (steps, n, m)
    lam = gh
    adj = oracle.tri_adjoint if kind == "tri" else oracle.penta_adjoint
    for s in range(steps):
        lam = adj(*bands, lam, cyclic=cyclic)
        assert rel_err(host(traj[s]), lam) < 1e-12, s
